"""Comparison helpers for GPU-vs-oracle parity tests.

Conditioning.  The Goldreich-Julian density is |rho|/e: the plasma frequency has a
V-shaped minimum on the null surface Omega.B = 0, where the force -grad(w_p^2) jumps.
Integrated as it stands, rays that cross or graze that surface are ill-conditioned at
rtol 1e-8 (a 2^-50 change of the seed moves the arrival direction by up to ~1e-5 rad).
Both the oracle and the kernels integrate one smooth piece of |rho| at a time and
restart on the other piece at the located crossing (Sec. 5 eq. (GJDensity) with the
discontinuity treatment of Hairer-Norsett-Wanner I, Sec. II.6); with that cut every
forward ray of the test workloads is well conditioned (oracle self-difference ~1e-12 rad).

Each ray's conditioning is still measured with the oracle alone (the oracle re-run from
seeds perturbed by 2^-50 relative), as a guard, and the per-ray tolerances are:
  rays on which the GPU takes the oracle's step sequence (accepted and rejected counts
      equal, lambda_f to 1e-12): direction <= 1e-9 rad, |d omega| <= 1e-12;
  "flip" rays (another step sequence): direction <= 1e-6 rad, and those beyond 1e-9 rad
      at most 0.1% of the escaped rays;
  at most 0.5% of the escaped rays ill-conditioned by the oracle's own measure (self-
      difference above 1e-11 rad, or a changed step sequence, under the perturbations).
Statuses must agree on every well-conditioned ray; a ray may switch between escaping
and hitting the star only if it is ill-conditioned, on at most 0.1% of the rays."""
import numpy as np

WELL_TOL = 1e-11     # oracle self-difference defining a well-conditioned ray [rad]
DIR_TOL = 1e-9       # direction tolerance, rays with the oracle's step sequence [rad]
OMEGA_TOL = 1e-12    # energy at infinity, rays with the oracle's step sequence
FLIP_DIR_TOL = 1e-6  # direction tolerance for flip rays [rad]
MAX_FLIP_FRAC = 1e-3  # flip rays (and status changes) per escaped ray (per ray)
MAX_ILL_FRAC = 5e-3   # ill-conditioned escaped rays the oracle may show (a guard on the cut)


def unit(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def angle_between(th1, ph1, th2, ph2):
    """angular distance, accurate for tiny angles"""
    a, b = unit(th1, ph1), unit(th2, ph2)
    return 2.0 * np.arcsin(np.clip(np.linalg.norm(a - b, axis=0) / 2.0, 0.0, 1.0))


def oracle_conditioning(orc, star, tol, rays, status, fin_o, ifin_o, kinks=True):
    """Per-ray self-difference of the oracle under 2^-50 relative perturbations (both
    signs) of the seed position and momentum.  Returns (selfdiff[n], seq_changed[n]).
    kinks selects the oracle's forward integration (see oracle.trace_forward)."""
    eps = 2.0 ** -50
    sd = np.zeros(rays.shape[1])
    changed = np.zeros(rays.shape[1], dtype=bool)
    for sl, f in ((slice(0, 3), 1 + eps), (slice(4, 7), 1 - eps), (slice(0, 3), 1 - eps), (slice(4, 7), 1 + eps)):
        r2 = np.array(rays, copy=True)
        r2[sl] *= f
        fin2, ifin2 = orc.trace_forward(star, tol, r2, status, kinks=kinks)
        d = angle_between(fin2[8], fin2[9], fin_o[8], fin_o[9])
        sd = np.maximum(sd, np.where((ifin2[2] == 1) & (ifin_o[2] == 1), d, 0.0))
        changed |= (ifin2[0] != ifin_o[0]) | (ifin2[1] != ifin_o[1]) | (ifin2[2] != ifin_o[2])
    return sd, changed


def assert_trace_parity(fin_g, ifin_g, fin_o, ifin_o, selfdiff, seq_changed, max_flip_frac=MAX_FLIP_FRAC,
                        max_ill_frac=MAX_ILL_FRAC, compare_lambda=True):
    """GPU final records (fin_g, ifin_g) against the oracle's on the same seeds.

    Same-sequence rays (escaped on both sides with equal accepted and rejected step counts
    and path parameter lambda_f to 1e-12): direction <= 1e-9 rad, |d omega| <= 1e-12.
    Flip rays (another step sequence; the direction may then move by up to the
    discretisation error): those beyond 1e-9 rad at most max_flip_frac of the escaped
    rays, each within 1e-6 rad.  Statuses equal on every well-conditioned ray, and at most
    max_flip_frac of all rays switch.  The oracle's own ill-conditioned share of the
    escaped rays stays below max_ill_frac.  compare_lambda=False: records without
    lambda_f (a host loop that returns the final state only) are sequenced by counts."""
    st_g, st_o = ifin_g[2], ifin_o[2]
    n = len(st_o)
    well = (selfdiff <= WELL_TOL) & ~seq_changed
    mism = st_g != st_o
    assert not (mism & well).any(), ("status mismatch on well-conditioned rays", np.nonzero(mism & well)[0][:10])
    assert mism.sum() <= max_flip_frac * n, ("status mismatches", int(mism.sum()), n)
    esc = (st_o == 1) & (st_g == 1)
    lam_g, lam_o = fin_g[13], fin_o[13]
    same = (ifin_g[0] == ifin_o[0]) & (ifin_g[1] == ifin_o[1])
    if compare_lambda:
        same &= np.abs(lam_g - lam_o) <= 1e-12 * np.abs(lam_o)
    d = angle_between(fin_g[8], fin_g[9], fin_o[8], fin_o[9])
    dw = np.abs(fin_g[11] - fin_o[11])
    sq = esc & same
    fl = esc & ~same
    far = fl & (d > DIR_TOL)
    ill = esc & ~well
    out = dict(n=int(n), escaped=int(esc.sum()), same_sequence=int(sq.sum()), flips=int(fl.sum()),
               flips_far=int(far.sum()), well=int((esc & well).sum()), ill=int(ill.sum()),
               status_mismatch=int(mism.sum()),
               max_dir_same=float(d[sq].max()) if sq.any() else 0.0,
               max_domega_same=float(dw[sq].max()) if sq.any() else 0.0,
               max_dir_flip=float(d[fl].max()) if fl.any() else 0.0)
    assert out["max_dir_same"] <= DIR_TOL, out
    assert out["max_domega_same"] <= OMEGA_TOL, out
    assert out["flips_far"] <= max_flip_frac * out["escaped"], ("too many flip rays beyond 1e-9 rad", out)
    assert out["max_dir_flip"] <= FLIP_DIR_TOL, out
    assert out["ill"] <= max_ill_frac * out["escaped"], ("too many ill-conditioned rays", out)
    return out


def same_bin_mask(fin_a, ifin_a, fin_b, ifin_b, bins):
    """rays that both runs put in the same (theta, psi, omega) bin"""
    import math
    dth, dps = math.pi / bins["n_theta"], 2 * math.pi / bins["n_psi"]

    def key(fin, ifin):
        it = np.minimum(np.floor(fin[8] / dth).astype(np.int64), bins["n_theta"] - 1)
        ip = np.minimum(np.floor(fin[10] / dps).astype(np.int64), bins["n_psi"] - 1)
        iw = np.floor((fin[11] - 1.0) / bins["d_omega"] + 0.5).astype(np.int64) + bins["n_omega"] // 2
        k = (it * bins["n_psi"] + ip) * bins["n_omega"] + iw
        return np.where(ifin[2] == 1, k, -1)

    ka, kb = key(fin_a, ifin_a), key(fin_b, ifin_b)
    return ka == kb, ka, kb


def per_ray_errors(g, go, floor=1e-6):
    """Relative error of each ray's gradient share g[i] against go[i]: the norm over the six
    parameters, each scaled by its RMS over the rays.  A ray's own norm is floored at
    `floor` times the largest ray's: a ray deep in the smoothing kernel's tail (share
    exp(-(1 - c) / sigma^2) far below the others) has its relative derivative moved by
    direction differences at the conditioning level times the exponent's slope, up to
    1 / sigma^2 per radian, and it counts for nothing in the total; such rays are compared
    in absolute terms at that floor."""
    sc = np.sqrt((go ** 2).mean(axis=0))
    sc = np.where(sc > 0, sc, 1.0)
    num = np.linalg.norm((g - go) / sc, axis=1)
    den = np.linalg.norm(go / sc, axis=1)
    den = np.maximum(den, floor * den.max()) if den.size else den
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
