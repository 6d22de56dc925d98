"""GPU parity of the forward path (seeding, tracing, binning) against the CPU oracle.

All calls go through the C ABI (librt.so) via the thin Python binding.  Inputs are
seeded and synthetic; expected values come only from the oracle.
Tolerances: seeds (positions, momenta) 1e-12 relative, weights 1e-9 relative (two
different derivative routes: dual numbers in the oracle, implicit differentiation of
the hand-derived gradient on the GPU); asymptotic directions 1e-9 rad and energies at
infinity 1e-12 on well-conditioned rays, which must be every escaped ray here (the null-
surface cut leaves no ill-conditioned forward ray; the general bound is at most 0.1% flip
rays at 1e-6 rad, tests/parity.py); binned flux 1e-6 relative in every bin whose member rays are the same
in both runs, total escaped weight 1e-9.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.parity import assert_trace_parity, angle_between, oracle_conditioning, same_bin_mask

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08655_amd as rt
    rt.lib()
    return rt


def _np(t):
    return t.cpu().numpy()


# the full forward workload with Maxwellian axion momenta at infinity (Sec. 4.3)
CFG2M = dict(W.CFG2, name="forward-gr-aniso-oblique-maxwellian", star=dict(W.CFG2["star"], speeds=W.SPEEDS_MAXWELL))
CFG1M = dict(W.CFG1, name="forward-flat-iso-maxwellian", star=dict(W.CFG1["star"], speeds=W.SPEEDS_MAXWELL))


def _cfg2_small(n):
    c = dict(W.CFG2)
    c["n"] = n
    return c


@pytest.mark.parametrize("cfg,n", [(W.CFG1, 4096), (W.CFG2, 3000), (W.CFG1, 37), (CFG1M, 4096), (CFG2M, 3000)])
def test_sample_matches_oracle(rt, orc, cfg, n):
    print(f"sample parity {cfg['name']} n={n}", flush=True)
    rays_g, st_g = rt.rt_sample_resonance(cfg["star"], cfg["seed"], n)
    rays_g, st_g = _np(rays_g), _np(st_g)
    rays_o, st_o = orc.sample(cfg["star"], cfg["seed"], n)
    assert np.array_equal(st_g, st_o)
    ok = st_o == 0
    scale = np.maximum(np.abs(rays_o[:8]), 1e-3)
    assert np.max(np.abs(rays_g[:8, ok] - rays_o[:8, ok]) / scale[:, ok]) < 1e-12
    assert np.max(np.abs(rays_g[8, ok] / rays_o[8, ok] - 1)) < 1e-9
    assert np.all(rays_g[8, ~ok] == 0)


def test_sample_offset_and_instance(rt, orc):
    cfg = W.CFG2
    rays_g, st_g = rt.rt_sample_resonance(cfg["star"], 7, 100, instance=3, first=123456)
    rays_o, st_o = orc.sample(cfg["star"], 7, 100, instance=3, first=123456)
    assert np.array_equal(_np(st_g), st_o)
    ok = st_o == 0
    assert np.allclose(_np(rays_g)[:8, ok], rays_o[:8, ok], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("cfg,n", [(W.CFG1, 4096), (W.CFG2, 2048), (W.CFG1, 4096 + 37), (CFG2M, 2048)])
def test_trace_matches_oracle(rt, orc, cfg, n):
    """Tracer parity from the oracle's own seeds."""
    import torch
    print(f"trace parity {cfg['name']} n={n}", flush=True)
    rays_o, st_o = orc.sample(cfg["star"], cfg["seed"], n)
    fin_o, ifin_o = orc.trace_forward(cfg["star"], cfg["tol"], rays_o, st_o)
    rays_t = torch.from_numpy(rays_o).cuda()
    st_t = torch.from_numpy(st_o).cuda()
    fin_g, ifin_g = rt.rt_trace_forward(cfg["star"], cfg["tol"], rays_t, st_t)
    fin_g, ifin_g = _np(fin_g), _np(ifin_g)
    sd, ch = oracle_conditioning(orc, cfg["star"], cfg["tol"], rays_o, st_o, fin_o, ifin_o)
    out = assert_trace_parity(fin_g, ifin_g, fin_o, ifin_o, sd, ch)
    print(out)
    assert out["well"] == out["escaped"]
    esc = ifin_g[2] == 1
    assert np.abs(fin_g[14][esc] / cfg["tol"]["r_max_km"] - 1).max() < 1e-12
    assert np.abs(fin_g[12][esc]).max() < 1e-4


@pytest.mark.parametrize("cfg", [W.CFG1, W.CFG2])
def test_end_to_end_binned_flux(rt, orc, cfg):
    """seed -> trace -> bin on the GPU vs the oracle's own pipeline."""
    n = 4096 if cfg is W.CFG1 else 2048
    print(f"end-to-end {cfg['name']} n={n}", flush=True)
    rays_g, st_g = rt.rt_sample_resonance(cfg["star"], cfg["seed"], n)
    fin_g, ifin_g = rt.rt_trace_forward(cfg["star"], cfg["tol"], rays_g, st_g)
    hist_g, cnt_g, over_g = rt.rt_bin_flux(fin_g, ifin_g, rays_g[8].contiguous(), cfg["bins"])
    rays_o, st_o = orc.sample(cfg["star"], cfg["seed"], n)
    fin_o, ifin_o = orc.trace_forward(cfg["star"], cfg["tol"], rays_o, st_o)
    hist_o, cnt_o, over_o = orc.bin_flux(fin_o, ifin_o, rays_o[8], cfg["bins"])
    fin_gn, ifin_gn = _np(fin_g), _np(ifin_g)
    sd, ch = oracle_conditioning(orc, cfg["star"], cfg["tol"], rays_o, st_o, fin_o, ifin_o)
    assert_trace_parity(fin_gn, ifin_gn, fin_o, ifin_o, sd, ch)
    esc = (ifin_o[2] == 1) & (ifin_gn[2] == 1)
    wg = _np(rays_g[8])
    assert np.allclose(wg[esc], rays_o[8][esc], rtol=1e-9, atol=0)
    assert abs(wg[ifin_gn[2] == 1].sum() / rays_o[8][ifin_o[2] == 1].sum() - 1) < 1e-9
    hg, ho = _np(hist_g), hist_o
    # bins whose member rays are identical in both runs must agree to 1e-6
    same, kg, ko = same_bin_mask(fin_gn, ifin_gn, fin_o, ifin_o, cfg["bins"])
    moved = np.unique(np.concatenate([kg[~same], ko[~same]]))
    moved = moved[moved >= 0]
    excused = np.zeros(ho.size, dtype=bool)
    in_range = moved[moved < ho.size]
    excused[in_range] = True
    excused = excused.reshape(ho.shape)
    ok = (~excused) & (ho > 0)
    rel = np.abs(hg[ok] / ho[ok] - 1)
    assert rel.max() < 1e-6, rel.max()
    assert np.array_equal(_np(cnt_g)[~excused], cnt_o[~excused])
    assert excused.sum() <= 0.02 * max(1, (ho > 0).sum()), (excused.sum(), (ho > 0).sum())
    print("bins compared", int(ok.sum()), "excused", int(excused.sum()))


def test_full_size_sampled_rays_match_oracle(rt, orc):
    """Full 1e6-ray workload in the benchmark's launch configuration; 256 strided rays are
    re-derived by the oracle one by one (its own seeding) and compared."""
    cfg = W.CFG2
    n = cfg["n"]
    print(f"full-size {cfg['name']} n={n}", flush=True)
    rays_g, st_g = rt.rt_sample_resonance(cfg["star"], cfg["seed"], n)
    fin_g, ifin_g = rt.rt_trace_forward(cfg["star"], cfg["tol"], rays_g, st_g)
    fin_g, ifin_g, st_g = _np(fin_g), _np(ifin_g), _np(st_g)
    idx = np.arange(0, n, n // 256)[:256]
    fo, io = [], []
    for i in idx:
        r, s = orc.sample(cfg["star"], cfg["seed"], 1, first=int(i))
        f, fi = orc.trace_forward(cfg["star"], cfg["tol"], r, s)
        fo.append(f[:, 0]); io.append(fi[:, 0])
    fo, io = np.array(fo).T, np.array(io).T
    ro = np.array([orc.sample(cfg["star"], cfg["seed"], 1, first=int(i))[0][:, 0] for i in idx]).T
    so = np.array([orc.sample(cfg["star"], cfg["seed"], 1, first=int(i))[1][0] for i in idx]).astype(np.int32)
    sd, ch = oracle_conditioning(orc, cfg["star"], cfg["tol"], ro, so, fo, io)
    assert_trace_parity(fin_g[:, idx], ifin_g[:, idx], fo, io, sd, ch)
    # properties at full size
    esc = ifin_g[2] == 1
    assert esc.mean() > 0.5
    assert np.abs(fin_g[14][esc] / cfg["tol"]["r_max_km"] - 1).max() < 1e-12
    assert np.abs(fin_g[12][esc]).max() < 1e-3
    assert set(np.unique(ifin_g[2])) <= {1, 2, 3, 4, 5}


def test_edge_cases(rt, orc):
    import torch
    cfg = W.CFG1
    # empty input: nothing launched, nothing fails
    rays, st = rt.rt_sample_resonance(cfg["star"], 0, 0)
    fin, ifin = rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, st)
    assert fin.shape == (16, 0)
    # every seed without a resonance (m_a above the largest plasma frequency)
    s = W.star(M_Msun=0.0, plasma=W.PLASMA_ISO, m_a_eV=1e-4, kdir=W.KDIR_OUTWARD)
    rays, st = rt.rt_sample_resonance(s, 0, 500)
    assert np.all(_np(st) == W.STATUS_NO_RESONANCE)
    fin, ifin = rt.rt_trace_forward(s, cfg["tol"], rays, st)
    assert np.all(_np(ifin)[2] == W.STATUS_NO_RESONANCE)
    hist, cnt, over = rt.rt_bin_flux(fin, ifin, rays[8].contiguous(), cfg["bins"])
    assert float(hist.sum()) == 0.0 and float(cnt.sum()) == 0.0
    # step cap: status MAX_STEPS on both sides
    t = W.tol(max_steps=10)
    rays_o, st_o = orc.sample(cfg["star"], 0, 300)
    fin_o, ifin_o = orc.trace_forward(cfg["star"], t, rays_o, st_o)
    fin_g, ifin_g = rt.rt_trace_forward(cfg["star"], t, torch.from_numpy(rays_o).cuda(),
                                        torch.from_numpy(st_o).cuda())
    assert np.array_equal(_np(ifin_g)[2], ifin_o[2])
    assert (ifin_o[2] == W.STATUS_MAX_STEPS).sum() > 100
    # invalid arguments are rejected before any launch
    bad = dict(cfg["star"])
    bad["B0_G"] = float("nan")
    with pytest.raises(rt.RtError, match="non-finite"):
        rt.rt_sample_resonance(bad, 0, 10)
    with pytest.raises(rt.RtError, match="workspace"):
        rt.rt_trace_forward(cfg["star"], cfg["tol"], rays_o_t := torch.from_numpy(rays_o).cuda(),
                            torch.from_numpy(st_o).cuda(), ws=torch.empty(16, dtype=torch.uint8, device="cuda"))
    bad_t = dict(cfg["tol"])
    bad_t["rtol"] = -1.0
    with pytest.raises(rt.RtError, match="rt_tol"):
        rt.rt_trace_forward(cfg["star"], bad_t, rays_o_t)


@pytest.mark.parametrize("sched", [dict(block=64, refill_min=1), dict(block=128, refill_min=8),
                                   dict(block=256, refill_min=32, waves_per_cu=8),
                                   dict(block=256, refill_min=16, occupancy=2),
                                   dict(block=256, refill_min=4, chunk=64), dict(block=128, refill_min=8, chunk=1024)])
def test_schedules_give_identical_rays(rt, orc, sched):
    """Per-ray results do not depend on the launch schedule (bit-identical)."""
    cfg = W.CFG2
    rays, st = rt.rt_sample_resonance(cfg["star"], 0, 3000)
    f0, i0 = rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, st)
    f1, i1 = rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, st, schedule=sched)
    assert np.array_equal(_np(i0), _np(i1))
    assert np.array_equal(_np(f0), _np(f1))


def test_kernel_timing_records_each_launch(rt):
    """rt_timing / rt_kernel_times bracket every launch of the tracing kernel with a HIP
    event pair on the caller's stream; stopping keeps the records, starting clears them."""
    import torch
    cfg = W.CFG1
    rays, st = rt.rt_sample_resonance(cfg["star"], 0, 2000)
    rt.timing(True)
    for _ in range(3):
        rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, st)
    rt.timing(False)
    rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, st)  # not recorded
    torch.cuda.synchronize()
    kt = rt.kernel_times()
    assert [name for name, _ in kt] == ["trace_fwd_kernel"] * 3
    assert all(ms > 0.0 for _, ms in kt)
    rt.timing(True)
    rt.timing(False)
    assert rt.kernel_times() == []
