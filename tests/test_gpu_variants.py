"""GPU parity of the approximation variants (App. B; Sec. 6 eq. (reweight)) and of the
Schwarzschild vacuum dipole against the CPU oracle: flat propagation of curved initial
conditions, renormalised weights, the thin resonance surface w_p = m_a, the GR dipole field.  Seeds: statuses equal, states 1e-12, weights 1e-9 relative (the
same criteria as the plain method); traces with the conditioning-aware criterion; the
smoothed-flux adjoint on the kink-free spherical star (every ray well conditioned) per ray
1e-8 and in total; unsupported combinations are refused."""
import numpy as np
import pytest

import workloads as W
from tests.parity import angle_between, assert_trace_parity, oracle_conditioning
from tests.test_gpu_adjoint import PER_RAY_TOL, SPHERICAL, gpu_flux_grad, per_ray_errors

pytestmark = pytest.mark.gpu

FLAGS = {"flat": W.FLAG_FLAT_PROPAGATION, "renorm": W.FLAG_RENORM_WEIGHTS, "thin": W.FLAG_THIN_SURFACE,
         "gr_dipole": W.FLAG_GR_DIPOLE}


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08655_amd as rt
    rt.lib()
    return rt


@pytest.mark.parametrize("variant", sorted(FLAGS))
@pytest.mark.parametrize("base", ["cfg1", "cfg2"])
def test_variant_seeds_match_oracle(rt, orc, variant, base):
    cfg = {"cfg1": W.CFG1, "cfg2": W.CFG2}[base]
    s = dict(cfg["star"], flags=FLAGS[variant])
    n = 3000
    print(f"variant seeds {variant} {base}", flush=True)
    rays_g, st_g = rt.rt_sample_resonance(s, cfg["seed"], n)
    rays_g, st_g = rays_g.cpu().numpy(), st_g.cpu().numpy()
    rays_o, st_o = orc.sample(s, cfg["seed"], n)
    assert np.array_equal(st_g, st_o)
    ok = st_o == 0
    assert ok.sum() > n // 2
    scale = np.maximum(np.abs(rays_o[:8]), 1e-3)
    assert np.max(np.abs(rays_g[:8, ok] - rays_o[:8, ok]) / scale[:, ok]) < 1e-12
    assert np.max(np.abs(rays_g[8, ok] / rays_o[8, ok] - 1)) < 1e-9


@pytest.mark.parametrize("variant", ["flat", "thin", "gr_dipole"])
def test_variant_traces_match_oracle(rt, orc, variant):
    import torch
    cfg = W.CFG2
    s = dict(cfg["star"], flags=FLAGS[variant])
    n = 2048
    print(f"variant traces {variant}", flush=True)
    rays_o, st_o = orc.sample(s, cfg["seed"], n)
    fin_o, ifin_o = orc.trace_forward(s, cfg["tol"], rays_o, st_o)
    fin_g, ifin_g = rt.rt_trace_forward(s, cfg["tol"], torch.from_numpy(rays_o).cuda(), torch.from_numpy(st_o).cuda())
    sd, ch = oracle_conditioning(orc, s, cfg["tol"], rays_o, st_o, fin_o, ifin_o)
    out = assert_trace_parity(fin_g.cpu().numpy(), ifin_g.cpu().numpy(), fin_o, ifin_o, sd, ch)
    print(out, flush=True)
    assert out["well"] == out["escaped"]


@pytest.mark.parametrize("variant", ["renorm", "thin", "gr_dipole"])
def test_variant_adjoint_matches_oracle(rt, orc, variant):
    s = dict(SPHERICAL, flags=FLAGS[variant])
    tol = W.tol()
    obs = W.observers(32)
    n = 300
    gbar = np.random.default_rng(12).standard_normal(32)
    print(f"variant adjoint {variant}", flush=True)
    F, g, gr, info = gpu_flux_grad(rt, s, tol, 0, n, obs, 0.05, gbar)
    Fo, dFo, fray, dray, sto = orc.flux_fwdmode(s, tol, 0, n, obs, 0.05, per_ray=True)
    assert np.array_equal(info[2], sto)
    esc = sto == W.STATUS_ESCAPED
    assert esc.sum() > 100
    go = np.einsum("j,njq->nq", gbar, dray)
    err = per_ray_errors(gr, go)
    assert err[esc].max() <= PER_RAY_TOL, err[esc].max()
    assert np.abs(F - Fo).max() <= 1e-9 * np.abs(Fo).max()
    assert np.linalg.norm(g - gbar @ dFo) <= PER_RAY_TOL * np.linalg.norm(gbar @ dFo)


def test_unsupported_combinations_are_refused(rt):
    import torch
    flat = dict(W.CFG2["star"], flags=W.FLAG_FLAT_PROPAGATION)
    with pytest.raises(rt.RtError, match="flat-propagation"):
        rt.FluxGrad(flat, W.tol(), 0, 64, W.observers(4), 0.05, 64, 64).forward()
    image = dict(D_km=1e5, incl=1.0, phi_o=0.0, half_width_km=40.0, nx=8, ny=8)
    with pytest.raises(rt.RtError, match="forward only"):
        rt.rt_trace_backward(flat, W.tol(r_max_km=1e5), image, K=2)
    ev, nev, _, _ = rt.rt_trace_backward(W.CFG3["star"], W.CFG3["tol"], image, K=2)
    with pytest.raises(rt.RtError, match="forward only"):
        rt.rt_backward_power(dict(W.CFG3["star"], flags=W.FLAG_RENORM_WEIGHTS), ev, nev, pixel_area_km2=1.0)
    with pytest.raises(rt.RtError, match="flat-propagation"):
        rt.Batch([flat, flat], [10, 10], 0, W.tol(), W.CFG4["bins"])
    with pytest.raises(rt.RtError, match="enumeration"):
        rt.rt_sample_resonance(dict(W.CFG2["star"], flags=64), 0, 8)


def test_gr_dipole_backward_matches_oracle(rt, orc):
    """Backward rays and event weights through the GR dipole field (magnetar star): events and
    statuses as the oracle's where it is well conditioned, per-ray weights 1e-6."""
    s = dict(W.CFG3["star"], flags=W.FLAG_GR_DIPOLE)
    t = W.tol(r_max_km=1e5)
    rng = np.random.default_rng(21)
    n = 300
    b1, b2 = rng.uniform(-35, 35, n), rng.uniform(-35, 35, n)
    print("gr dipole backward", flush=True)
    ev, nev, fin, ifin = rt.rt_trace_backward_rays(s, t, 1e5, 0.8, 0.1, b1, b2, K=4)
    wsum, total = rt.rt_backward_power(s, ev, nev, pixel_area_km2=1.0)
    w_o, ev_o, nev_o, fin_o, ifin_o = orc.backward_rays(s, t, 1e5, 0.8, 0.1, b1, b2, K=4)
    bad = np.zeros(n, dtype=bool)
    for fac in (1 + 2.0 ** -50, 1 - 2.0 ** -50):
        w2, ev2, nev2, fin2, ifin2 = orc.backward_rays(s, t, 1e5 * fac, 0.8, 0.1, b1, b2, K=4)
        bad |= (nev2 != nev_o) | (ifin2[2] != ifin_o[2]) | (ifin2[0] != ifin_o[0])
        bad |= (nev2 > 0) & (np.abs(w2 - w_o) > 1e-8 * np.abs(w_o))
    assert bad.mean() <= 0.03
    ok = ~bad
    nev_g, ifin_g, w_g = nev.cpu().numpy(), ifin.cpu().numpy(), wsum.cpu().numpy()
    assert np.array_equal(nev_g[ok], nev_o[ok]) and np.array_equal(ifin_g[2][ok], ifin_o[2][ok])
    m = ok & (nev_o > 0)
    assert m.sum() >= 30
    assert np.allclose(w_g[m], w_o[m], rtol=1e-6, atol=0), np.abs(w_g[m] / w_o[m] - 1).max()


# ---------------------------------------------------------------- finite magnetisation
LARMOR_STARS = {"weak_field": W.WEAK_FIELD["star"],
                "weak_field_gr_dipole": dict(W.WEAK_FIELD["star"], flags=W.FLAG_FINITE_LARMOR | W.FLAG_GR_DIPOLE),
                "weak_field_gj_aligned": dict(W.WEAK_FIELD["star"], theta_m=0.0, density=W.DENSITY_GJ,
                                              multiplicity=1e8, kdir=W.KDIR_ISOTROPIC),
                "weak_field_aligned": dict(W.WEAK_FIELD["star"], theta_m=0.0),
                "cfg2": dict(W.CFG2["star"], flags=W.FLAG_FINITE_LARMOR)}


@pytest.mark.parametrize("name", sorted(LARMOR_STARS))
def test_finite_larmor_seeds_match_oracle(rt, orc, name):
    """Seeds of the finite-magnetisation Hamiltonian (Sec. 4.1 eq. (DisRel)): the resonance,
    momenta and weights against the oracle, which takes the photon energy's gradient by
    Newton's method on the dispersion relation where the kernels take it implicitly from
    the hand-derived gradient.  Statuses equal, states 1e-12, weights 1e-9."""
    s = LARMOR_STARS[name]
    n = 3000
    print(f"finite-larmor seeds {name}", flush=True)
    rays_g, st_g = rt.rt_sample_resonance(s, 0, n)
    rays_g, st_g = rays_g.cpu().numpy(), st_g.cpu().numpy()
    rays_o, st_o = orc.sample(s, 0, n)
    assert np.array_equal(st_g, st_o)
    ok = st_o == 0
    assert ok.sum() > n // 2
    scale = np.maximum(np.abs(rays_o[:8]), 1e-3)
    assert np.max(np.abs(rays_g[:8, ok] - rays_o[:8, ok]) / scale[:, ok]) < 1e-12
    assert np.max(np.abs(rays_g[8, ok] / rays_o[8, ok] - 1)) < 1e-9


@pytest.mark.parametrize("name", ["weak_field", "weak_field_gr_dipole", "weak_field_aligned"])
def test_finite_larmor_traces_match_oracle(rt, orc, name):
    """Rays of the finite-magnetisation Hamiltonian on the weakly magnetised test stars
    (cyclotron frequency 2-26 times the photon frequency along the path; the kink-free
    spherical density, on which the two magnetoionic modes stay apart) against the
    oracle's, from the oracle's seeds, with the per-ray tolerances; and the variant moves
    the rays away from the strong-field ones by far more than those tolerances."""
    import torch
    s, t = LARMOR_STARS[name], W.WEAK_FIELD["tol"]
    n = 2048
    print(f"finite-larmor traces {name}", flush=True)
    rays_o, st_o = orc.sample(s, 0, n)
    fin_o, ifin_o = orc.trace_forward(s, t, rays_o, st_o)
    rays_t, st_t = torch.from_numpy(rays_o).cuda(), torch.from_numpy(st_o).cuda()
    fin_g, ifin_g = rt.rt_trace_forward(s, t, rays_t, st_t)
    fin_g, ifin_g = fin_g.cpu().numpy(), ifin_g.cpu().numpy()
    sd, ch = oracle_conditioning(orc, s, t, rays_o, st_o, fin_o, ifin_o)
    out = assert_trace_parity(fin_g, ifin_g, fin_o, ifin_o, sd, ch)
    print(out, flush=True)
    assert out["escaped"] > n // 2 and out["well"] == out["escaped"]
    assert np.abs(fin_g[12][ifin_g[2] == 1]).max() < 1e-7
    strong = dict(s, flags=s["flags"] & ~W.FLAG_FINITE_LARMOR)
    fin_s, ifin_s = rt.rt_trace_forward(strong, t, rays_t, st_t)
    fin_s, ifin_s = fin_s.cpu().numpy(), ifin_s.cpu().numpy()
    both = (ifin_g[2] == 1) & (ifin_s[2] == 1)
    d = angle_between(fin_g[8], fin_g[9], fin_s[8], fin_s[9])[both]
    assert np.median(d) > 1e-6, np.median(d)


def test_finite_larmor_unsupported_combinations_are_refused(rt):
    s = W.WEAK_FIELD["star"]
    with pytest.raises(rt.RtError, match="anisotropic"):
        rt.rt_sample_resonance(dict(s, plasma=W.PLASMA_ISO), 0, 8)
    with pytest.raises(rt.RtError, match="thin-surface"):
        rt.rt_sample_resonance(dict(s, flags=W.FLAG_FINITE_LARMOR | W.FLAG_THIN_SURFACE), 0, 8)
    image = dict(D_km=1e5, incl=1.0, phi_o=0.0, half_width_km=40.0, nx=8, ny=8)
    with pytest.raises(rt.RtError, match="forward only"):
        rt.rt_trace_backward(s, W.tol(r_max_km=1e5), image, K=2)
    with pytest.raises(rt.RtError, match="finite-magnetisation"):
        rt.Batch([s, s], [10, 10], 0, W.WEAK_FIELD["tol"], W.CFG4["bins"])


def test_finite_larmor_adjoint_matches_oracle(rt, orc):
    """The smoothed-flux adjoint with the finite-magnetisation Hamiltonian (its stage products
    carry the plasma and cyclotron coefficients as tangents) against the oracle's forward
    mode on the weakly magnetised star: per ray 1e-8, flux 1e-9 and gradient 1e-8 in total
    (every ray well conditioned)."""
    s, tol = W.WEAK_FIELD["star"], W.WEAK_FIELD["tol"]
    obs = W.observers(32)
    n = 300
    gbar = np.random.default_rng(13).standard_normal(32)
    print("finite-larmor adjoint", flush=True)
    F, g, gr, info = gpu_flux_grad(rt, s, tol, 0, n, obs, 0.05, gbar)
    Fo, dFo, fray, dray, sto = orc.flux_fwdmode(s, tol, 0, n, obs, 0.05, per_ray=True)
    assert np.array_equal(info[2], sto)
    esc = sto == W.STATUS_ESCAPED
    assert esc.sum() > 200
    go = np.einsum("j,njq->nq", gbar, dray)
    err = per_ray_errors(gr, go)
    assert err[esc].max() <= PER_RAY_TOL, err[esc].max()
    assert np.abs(F - Fo).max() <= 1e-9 * np.abs(Fo).max()
    assert np.linalg.norm(g - gbar @ dFo) <= PER_RAY_TOL * np.linalg.norm(gbar @ dFo)
    # the cyclotron channel is live: the strong-field star's gradient differs
    _, g0, _, _ = gpu_flux_grad(rt, dict(s, flags=0), tol, 0, n, obs, 0.05, gbar)
    assert np.linalg.norm(g - g0) > 1e-6 * np.linalg.norm(g0)
