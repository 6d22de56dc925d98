"""GPU parity of the binning step (Sec. 2.2: escaped rays binned by asymptotic direction
and energy at infinity) against the oracle's histogram, on synthetic final records.

Counts are integers and must agree bit for bit.  Weighted sums differ from the oracle's
only in the order of the FP64 additions of positive terms, each side within (c - 1) u of
the exact sum of a bin with c rays (u = 2^-53): 2 c u relative per bin.
The maps span one LDS tile, many tiles (the partitioned path), more tiles than the
partition has buckets (one atomic pair per ray), several instances, ragged lengths,
an empty input and a pile-up of every ray into eight bins.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08655_amd as rt
    rt.lib()
    return rt


def _gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _oracle_maps(orc, fin, ifin, w, bins, off=None):
    if off is None:
        return orc.bin_flux(fin, ifin, w, bins)
    hs, cs, over = [], [], np.zeros(2)
    for k in range(len(off) - 1):
        sl = slice(int(off[k]), int(off[k + 1]))
        h, c, o = orc.bin_flux(fin[:, sl], ifin[:, sl], w[sl], bins)
        hs.append(h); cs.append(c); over += o
    return np.stack(hs), np.stack(cs), over


def _check(hg, cg, og, ho, co, oo):
    hg, cg, og = hg.cpu().numpy(), cg.cpu().numpy(), og.cpu().numpy()
    assert hg.shape == ho.shape
    assert np.array_equal(cg, co), int((cg != co).sum())
    nz = co > 0
    assert np.all(hg[~nz] == 0.0)
    u = 2.0 ** -53
    if nz.any():
        rel = np.abs(hg[nz] / ho[nz] - 1.0)
        assert np.all(rel <= 2.0 * co[nz] * u), (rel / co[nz]).max() / u
    assert og[1] == oo[1]
    if oo[1] > 0:
        assert abs(og[0] / oo[0] - 1.0) <= 2.0 * oo[1] * u


CASES = [
    ("one-tile", dict(n_theta=8, n_psi=16, n_omega=8, d_omega=1e-3), 5003, 0.3),
    ("forward-flat-iso bins", W.CFG1["bins"], 100003, 0.3),
    ("full-size bins, 1e6 rays", W.CFG2["bins"], 1_000_017, 0.3),
    ("all rays in eight bins", W.CFG2["bins"], 200_000, 1.0),
    ("33.5M bins (direct path)", dict(n_theta=256, n_psi=512, n_omega=256, d_omega=1e-4), 200_001, 0.3),
    ("3e6 rays (256 sorting workgroups, ragged chunks)", W.CFG1["bins"], 3_000_001, 0.3),
]


@pytest.mark.parametrize("name,bins,n,hot", CASES, ids=[c[0] for c in CASES])
def test_bin_matches_oracle(rt, orc, name, bins, n, hot):
    print(f"bin {name} n={n}", flush=True)
    fin, ifin, w = W.final_records(n, bins, seed=n, hot_frac=hot)
    hg, cg, og = rt.rt_bin_flux(_gpu(fin), _gpu(ifin), _gpu(w), bins)
    _check(hg, cg, og, *_oracle_maps(orc, fin, ifin, w, bins))
    assert int(cg.sum().item()) + int(og[1].item()) == int((ifin[2] == W.STATUS_ESCAPED).sum())


def test_bin_instances_match_oracle(rt, orc):
    """Consecutive instances (one empty) share one launch; each gets its own map."""
    bins = W.CFG1["bins"]
    counts = [7001, 0, 30000, 1, 12345]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(off[-1])
    fin, ifin, w = W.final_records(n, bins, seed=11)
    print(f"bin instances n={n} n_inst={len(counts)}", flush=True)
    hg, cg, og = rt.rt_bin_flux(_gpu(fin), _gpu(ifin), _gpu(w), bins, inst_offset=_gpu(off), n_inst=len(counts))
    _check(hg, cg, og, *_oracle_maps(orc, fin, ifin, w, bins, off))


def test_bin_repeat_and_empty(rt, orc):
    """A second call on a shorter input into the same buffers gives the shorter input's
    maps (nothing left over from the first); an empty input gives empty maps."""
    import torch
    bins = W.CFG1["bins"]
    ws = rt.workspace(rt.OP_BIN, 60000)
    fin, ifin, w = W.final_records(60000, bins, seed=5)
    h, c, o = rt.rt_bin_flux(_gpu(fin), _gpu(ifin), _gpu(w), bins, ws=ws)
    _check(h, c, o, *_oracle_maps(orc, fin, ifin, w, bins))
    fin2, ifin2, w2 = W.final_records(999, bins, seed=6)
    h2, c2, o2 = rt.rt_bin_flux(_gpu(fin2), _gpu(ifin2), _gpu(w2), bins, ws=ws, hist=h.unsqueeze(0), cnt=c.unsqueeze(0),
                                over=o)
    _check(h2, c2, o2, *_oracle_maps(orc, fin2, ifin2, w2, bins))
    e = torch.empty((16, 0), dtype=torch.float64, device="cuda")
    ei = torch.empty((3, 0), dtype=torch.int32, device="cuda")
    ew = torch.empty(0, dtype=torch.float64, device="cuda")
    h3, c3, o3 = rt.rt_bin_flux(e, ei, ew, bins, ws=ws, hist=h.unsqueeze(0), cnt=c.unsqueeze(0), over=o)
    assert float(h3.abs().sum()) == 0.0 and float(c3.sum()) == 0.0 and float(o3.abs().sum()) == 0.0
