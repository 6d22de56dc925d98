"""GPU parity of the magnetar options of Sec. 6 against the CPU oracle: conversion removed on
open field lines (seed statuses and weights, bit-identical elsewhere to the unflagged run) and
the resonant cyclotron optical depth of escaped rays (rt_cyclotron_depth; the GPU refines the
resonance by log-space steps, the oracle bisects: radii 1e-13, depths 1e-12 relative), on the
four magnetar models M1-M4 and a fast aligned rotator whose light cylinder cuts the
conversion surface."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FAST = W.star(M_Msun=0.0, theta_m=0.0, P_s=2e-3, m_a_eV=1e-4, plasma=W.PLASMA_ISO, density=W.DENSITY_SPHERICAL,
              flags=W.FLAG_EXCISE_OPEN)


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08655_amd as rt
    rt.lib()
    return rt


@pytest.mark.parametrize("name", ["fast", "M1", "M2", "M3", "M4"])
def test_excised_seeds_match_oracle(rt, orc, name):
    s = FAST if name == "fast" else W.MAGNETAR_MODELS[name]
    n = 4096
    print(f"excised seeds {name}", flush=True)
    rays_g, st_g = rt.rt_sample_resonance(s, 3, n)
    rays_g, st_g = rays_g.cpu().numpy(), st_g.cpu().numpy()
    rays_o, st_o = orc.sample(s, 3, n)
    assert np.array_equal(st_g, st_o)
    if name == "fast":
        assert 0.2 < (st_o == W.STATUS_EXCISED).mean() < 0.8
    ok = st_o == 0
    scale = np.maximum(np.abs(rays_o[:8]), 1e-3)
    assert np.max(np.abs(rays_g[:8, ok] - rays_o[:8, ok]) / scale[:, ok]) < 1e-12
    assert np.max(np.abs(rays_g[8, ok] / rays_o[8, ok] - 1)) < 1e-9
    exc = st_o == W.STATUS_EXCISED
    assert np.all(rays_g[:9, exc] == 0.0)
    assert np.allclose(rays_g[9, exc], rays_o[9, exc], rtol=1e-13, atol=0)
    # the unflagged run differs only in the excised seeds
    plain, st_p = rt.rt_sample_resonance(dict(s, flags=0), 3, n)
    assert np.array_equal(plain.cpu().numpy()[:, ~exc], rays_g[:, ~exc])


@pytest.mark.parametrize("name", ["gj_iso_oblique", "M1", "M4"])
def test_cyclotron_depth_matches_oracle(rt, orc, name):
    import torch
    s = W.star(M_Msun=1.0, theta_m=0.4, plasma=W.PLASMA_ISO, m_a_eV=1e-5) if name == "gj_iso_oblique" \
        else W.MAGNETAR_MODELS[name]
    t = W.tol()
    n = 600
    print(f"cyclotron depth {name}", flush=True)
    rays, st = orc.sample(s, 4, n)
    fin, ifin = orc.trace_forward(s, t, rays, st)
    tau_o, rc_o = orc.cyclotron_depth(s, fin, ifin, rays[9])
    esc = ifin[2] == W.STATUS_ESCAPED
    assert esc.sum() >= 100 and (tau_o > 0).sum() >= 100
    tau, rcyc, w_out = rt.rt_cyclotron_depth(s, torch.from_numpy(rays).cuda(), torch.from_numpy(fin).cuda(),
                                             torch.from_numpy(ifin).cuda())
    tau, rcyc, w_out = tau.cpu().numpy(), rcyc.cpu().numpy(), w_out.cpu().numpy()
    assert np.all(tau[~esc] == 0.0) and np.all(rcyc[~esc] == -1.0)
    assert np.allclose(rcyc[esc], rc_o[esc], rtol=1e-13, atol=0)
    assert np.allclose(tau, tau_o, rtol=1e-12, atol=0)
    assert np.allclose(w_out, rays[8] * np.exp(-tau_o), rtol=1e-12, atol=0)


def test_magnetar_models_end_to_end(rt, orc):
    """M1-M4 on the GPU: seeding with excision, tracing, cyclotron attenuation and binning;
    the larger multiplicity and field move the conversion surface outward (the density grows
    with lambda B0), the attenuated power never exceeds the unattenuated one, and the binned
    total equals the sum of the attenuated escaped weights."""
    import torch
    t = W.tol()
    bins = dict(n_theta=32, n_psi=64, n_omega=1, d_omega=1.0)
    n = 65536
    rc_med = {}
    for name, s in W.MAGNETAR_MODELS.items():
        print(f"magnetar model {name}", flush=True)
        rays, st = rt.rt_sample_resonance(s, 9, n)
        fin, ifin = rt.rt_trace_forward(s, t, rays, st)
        tau, rcyc, w_out = rt.rt_cyclotron_depth(s, rays, fin, ifin)
        hist, cnt, over = rt.rt_bin_flux(fin, ifin, w_out, bins)
        torch.cuda.synchronize()
        esc = ifin[2] == 1
        P0 = float(rays[8][esc].sum())
        P1 = float(w_out[esc].sum())
        assert 0 < P1 <= P0
        assert abs(float(hist.sum()) + float(over[0]) - P1) <= 1e-9 * P1
        ok = st == 0
        rc_med[name] = float(rays[9][ok].median())
    assert rc_med["M2"] > rc_med["M1"] and rc_med["M3"] > rc_med["M1"] and rc_med["M4"] > rc_med["M2"]


def test_cyclotron_depth_errors(rt):
    import torch
    s = W.MAGNETAR_MODELS["M1"]
    z = torch.zeros((16, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        rt.rt_cyclotron_depth(s, z[:10, :3].contiguous(), z, torch.zeros((3, 4), dtype=torch.int32, device="cuda"))
    with pytest.raises(rt.RtError, match="enumeration"):
        rt.rt_cyclotron_depth(dict(s, flags=64), z[:10].contiguous(), z, torch.zeros((3, 4), dtype=torch.int32,
                                                                                     device="cuda"))
