"""Batched persistent launch: per-ray results identical to one launch per instance,
maps equal up to FP64 atomic summation order (1e-12 relative), oracle parity on
individual instances, hipGraph capture replayed several times with eager work in
between, and empty instances."""
import numpy as np
import pytest

import workloads as W
from tests.parity import assert_trace_parity, oracle_conditioning

pytestmark = pytest.mark.gpu

BINS = dict(n_theta=64, n_psi=128, n_omega=1, d_omega=1.0)


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08655_amd as rt
    rt.lib()
    return rt


def small_batch():
    spec = [(1e-6, 0.0, 700), (1e-5, 0.0, 1500), (2e-5, 0.6, 333), (1e-5, 1.2, 2000), (1e-4, 0.3, 400),
            (3e-6, 0.9, 1024), (1e-5, 0.3, 1)]
    stars = [W.star(M_Msun=0.0, theta_m=t, plasma=W.PLASMA_ISO, m_a_eV=m, kdir=W.KDIR_OUTWARD) for m, t, _ in spec]
    return stars, [c for _, _, c in spec]


def _np(t):
    return t.cpu().numpy()


def test_batched_equals_per_instance_launches(rt):
    stars, counts = small_batch()
    tol = W.tol()
    print("batched vs per-instance", counts, flush=True)
    b = rt.Batch(stars, counts, 1, tol, BINS)
    b.run()
    off = b.offsets
    maps, cnt = _np(b.maps), _np(b.cnt)
    for k, s in enumerate(stars):
        sl = slice(off[k], off[k + 1])
        rays_k, st_k = rt.rt_sample_resonance(s, 1, counts[k], instance=k)
        fin_k, ifin_k = rt.rt_trace_forward(s, tol, rays_k, st_k)
        h_k, c_k, _ = rt.rt_bin_flux(fin_k, ifin_k, rays_k[8].contiguous(), BINS)
        assert np.array_equal(_np(b.status)[sl], _np(st_k))
        assert np.array_equal(_np(b.rays)[:, sl], _np(rays_k))
        assert np.array_equal(_np(b.ifin)[:, sl], _np(ifin_k))
        fb, fk = _np(b.fin)[:, sl], _np(fin_k)
        assert np.allclose(fb, fk, rtol=1e-13, atol=1e-300), np.abs(fb - fk).max()
        assert np.array_equal(cnt[k], _np(c_k))
        hk = _np(h_k)
        nz = hk > 0
        assert np.allclose(maps[k][nz], hk[nz], rtol=1e-12, atol=0)
        assert np.all(maps[k][~nz] == 0)
    # the empty instance (m_a = 1e-4 eV above every plasma frequency) contributes nothing
    assert maps[4].sum() == 0 and np.all(_np(b.status)[off[4]:off[5]] == W.STATUS_NO_RESONANCE)


def test_batched_instances_match_oracle(rt, orc):
    stars, counts = small_batch()
    tol = W.tol()
    b = rt.Batch(stars, counts, 1, tol, BINS)
    b.run()
    off = b.offsets
    for k in (0, 2, 3):
        print(f"batched instance {k} vs oracle", flush=True)
        sl = slice(off[k], off[k + 1])
        rays_o, st_o = orc.sample(stars[k], 1, counts[k], instance=k)
        fin_o, ifin_o = orc.trace_forward(stars[k], tol, rays_o, st_o)
        assert np.array_equal(_np(b.status)[sl], st_o)
        sd, ch = oracle_conditioning(orc, stars[k], tol, rays_o, st_o, fin_o, ifin_o)
        assert_trace_parity(_np(b.fin)[:, sl], _np(b.ifin)[:, sl], fin_o, ifin_o, sd, ch)


def test_batched_graph_replays(rt):
    import torch
    stars, counts = small_batch()
    tol = W.tol()
    b = rt.Batch(stars, counts, 1, tol, BINS)
    b.run()
    torch.cuda.synchronize()
    ref_fin, ref_ifin, ref_maps = b.fin.clone(), b.ifin.clone(), b.maps.clone()
    g = b.capture()
    other = W.CFG1
    for rep in range(3):
        print(f"graph replay {rep}", flush=True)
        # eager work between replays, on the same device and stream
        rays, st = rt.rt_sample_resonance(other["star"], rep, 300)
        rt.rt_trace_forward(other["star"], other["tol"], rays, st)
        b.fin.zero_()
        b.maps.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.ifin, ref_ifin)
        assert torch.allclose(b.fin, ref_fin, rtol=0, atol=0, equal_nan=True)
        nz = ref_maps > 0
        assert torch.allclose(b.maps[nz], ref_maps[nz], rtol=1e-12, atol=0)
        assert float(b.maps[~nz].abs().sum()) == 0.0


def test_batched_rejects_mixed_plasma(rt):
    stars, counts = small_batch()
    stars[1] = dict(stars[1])
    stars[1]["plasma"] = W.PLASMA_ANISO
    with pytest.raises(rt.RtError, match="share plasma"):
        rt.Batch(stars, counts, 1, W.tol(), BINS)
