"""The no-allocation binning entry point (rt_bin_flux_noalloc: the scratch in a static
device array of the library) against rt_bin_flux with a caller workspace, through the C
ABI, on two calls in a row on one device: first at the entry point's maximum size (2^20
rays into the 64 x 128 x 64 map of the full forward workload, the tile-partitioned path),
then a smaller ragged batch of three instances' 64 x 128 maps, so the second call runs on
what the first left in the array.  Counts and out-of-band counts bit for bit; weighted
sums differ only in the order of FP64 additions of positive terms: 2 c u relative in a
bin of c rays (u = 2^-53).  Sizes above the maximum are refused before any launch."""
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


def _same(a, b):
    ha, ca, oa = (t.cpu().numpy() for t in a)
    hb, cb, ob = (t.cpu().numpy() for t in b)
    assert np.array_equal(ca, cb), int((ca != cb).sum())
    nz = cb > 0
    assert np.all(ha[~nz] == 0.0) and np.all(hb[~nz] == 0.0)
    u = 2.0 ** -53
    rel = np.abs(ha[nz] / hb[nz] - 1.0)
    assert np.all(rel <= 2.0 * cb[nz] * u), float((rel / cb[nz]).max() / u)
    assert oa[1] == ob[1]
    if ob[1] > 0:
        assert abs(oa[0] / ob[0] - 1.0) <= 2.0 * ob[1] * u
    return int(nz.sum())


def test_noalloc_binning_equals_workspace_binning_on_two_calls(rt):
    import torch
    dev = torch.device("cuda")
    n_max = rt.NOALLOC_BIN_MAX_RAYS
    # call 1: the maximum size, one map of the full forward workload
    bins1 = W.CFG2["bins"]
    fin, ifin, w = W.final_records(n_max, bins1, seed=3)
    fin_t, ifin_t, w_t = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (fin, ifin, w))
    print(f"noalloc call 1: n={n_max}, bins {bins1}", flush=True)
    out_n = rt.rt_bin_flux_noalloc(fin_t, ifin_t, w_t, bins1)
    out_w = rt.rt_bin_flux(fin_t, ifin_t, w_t, bins1)
    torch.cuda.synchronize()
    touched = _same(out_n, out_w)
    assert touched > 10000
    # call 2: smaller, three instances of ragged length, on what call 1 left in the array
    bins2 = W.CFG4["bins"]
    counts = [100003, 1, 199997]
    n2 = sum(counts)
    fin2, ifin2, w2 = W.final_records(n2, bins2, seed=4)
    off = torch.tensor(np.concatenate([[0], np.cumsum(counts)]), dtype=torch.int64, device=dev)
    fin2_t, ifin2_t, w2_t = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (fin2, ifin2, w2))
    print(f"noalloc call 2: n={n2}, {len(counts)} instances", flush=True)
    hist = torch.full((3, 64, 128, 1), 7.0, dtype=torch.float64, device=dev)  # overwritten, not added to
    cnt = torch.full_like(hist, 7.0)
    over = torch.full((2,), 7.0, dtype=torch.float64, device=dev)
    out_n2 = rt.rt_bin_flux_noalloc(fin2_t, ifin2_t, w2_t, bins2, inst_offset=off, n_inst=3, hist=hist, cnt=cnt,
                                    over=over)
    out_w2 = rt.rt_bin_flux(fin2_t, ifin2_t, w2_t, bins2, inst_offset=off, n_inst=3)
    torch.cuda.synchronize()
    assert _same(out_n2, out_w2) > 1000
    # the same small call again gives the same counts and sums to roundoff
    out_n3 = rt.rt_bin_flux_noalloc(fin2_t, ifin2_t, w2_t, bins2, inst_offset=off, n_inst=3)
    torch.cuda.synchronize()
    _same(out_n3, out_w2)
    # an empty input clears the maps
    out_e = rt.rt_bin_flux_noalloc(fin2_t[:, :0].contiguous(), ifin2_t[:, :0].contiguous(), w2_t[:0], bins2)
    torch.cuda.synchronize()
    assert float(out_e[0].abs().sum()) == 0.0 and float(out_e[1].sum()) == 0.0


def test_noalloc_refuses_sizes_above_its_maximum(rt):
    import torch
    dev = torch.device("cuda")
    n = rt.NOALLOC_BIN_MAX_RAYS + 1
    fin = torch.zeros((rt.RT_NFIN, n), dtype=torch.float64, device=dev)
    ifin = torch.zeros((rt.RT_NIFIN, n), dtype=torch.int32, device=dev)
    w = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(rt.RtError, match="RT_NOALLOC_BIN_MAX_RAYS"):
        rt.rt_bin_flux_noalloc(fin, ifin, w, W.CFG2["bins"])
