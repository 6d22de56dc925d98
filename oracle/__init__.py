"""CPU oracle of the ray-tracing hot path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library it wraps (``liboracle.so``,
built from ``rt_oracle.cpp`` with g++) shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "rt_oracle.cpp"), os.path.join(_HERE, "dual.hpp"), os.path.join(_HERE, "oracle.h")]

NFIN = 16
NIFIN = 3
NEV = 10
FIN_FIELDS = ["x", "y", "z", "t", "kx", "ky", "kz", "kt", "theta", "phi", "psi", "omega", "H", "lam", "r", "h"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (plain FP64: no fast-math, no contraction)."""
    if not force and os.path.exists(_LIB_PATH) and all(
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in _SRC):
        return _LIB_PATH
    cmd = ["g++", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-std=c++17", "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "rt_oracle.cpp")]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Star(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("B0_G", "P_s", "theta_m", "M_Msun", "R_km", "m_a_eV", "g_agg_GeV",
                                          "v0_kms", "rho_GeVcm3", "multiplicity", "psi_twist", "B_test_G")] + \
               [(n, C.c_int32) for n in ("plasma", "density", "weights", "kdir", "speeds", "flags")]


class Tol(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("r_max_km", C.c_double), ("max_steps", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        sp = C.POINTER(Star)
        tp = C.POINTER(Tol)
        L.orc_constants.argtypes = [dp, C.c_int]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_int32, C.c_int64, dp]
        L.orc_wp2.argtypes = [sp, dp, C.c_double]
        L.orc_wp2.restype = C.c_double
        L.orc_bfield.argtypes = [sp, dp, C.c_double, dp]
        L.orc_hamiltonian.argtypes = [sp, dp]
        L.orc_hamiltonian.restype = C.c_double
        L.orc_grad_h.argtypes = [sp, dp, dp]
        L.orc_inverse_metric.argtypes = [sp, dp, dp]
        L.orc_resonance_radius.argtypes = [sp, dp, dp, C.c_double]
        L.orc_resonance_radius.restype = C.c_double
        L.orc_energy_aniso.argtypes = [sp, dp, C.c_double, dp]
        L.orc_energy_aniso.restype = C.c_double
        L.orc_sample.argtypes = [sp, C.c_uint64, C.c_int32, C.c_int64, C.c_int64, dp, ip, C.c_int]
        L.orc_trace_forward.argtypes = [sp, tp, dp, ip, C.c_int64, dp, ip, C.c_int, C.c_int]
        L.orc_trace_reverse.argtypes = [sp, tp, dp, C.c_int64, C.c_double, dp, ip, C.c_int]
        L.orc_bin.argtypes = [dp, ip, dp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_double, dp, dp, dp]
        L.orc_trace_backward.argtypes = [sp, tp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                         C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                         C.c_int32, dp, ip, dp, ip, C.c_int]
        L.orc_backward_rays.argtypes = [sp, tp, C.c_double, C.c_double, C.c_double, dp, dp, C.c_int64, C.c_int32,
                                        C.c_double, dp, dp, ip, dp, ip, C.c_int]
        L.orc_event_weight.argtypes = [sp, dp, C.c_double, dp, dp]
        L.orc_cyclotron_depth.argtypes = [sp, dp, ip, dp, C.c_int64, dp, dp]
        L.orc_open_field.argtypes = [sp, dp, C.c_double]
        L.orc_maxwell_x.argtypes = [C.c_double]
        L.orc_maxwell_x.restype = C.c_double
        L.orc_dopri_test.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, dp, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), C.c_double, dp]
        L.orc_flux_fwdmode.argtypes = [sp, tp, C.c_uint64, C.c_int64, dp, C.c_int32, C.c_double, dp, dp, dp, dp, ip,
                                        C.c_int]
        L.orc_flux_replay.argtypes = [sp, tp, C.c_uint64, C.c_int64, dp, C.c_int32, C.c_double, C.c_int32,
                                      C.c_int32, dp, ip, ip, dp, C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def make_star(d: dict) -> Star:
    s = Star()
    for name, _ in Star._fields_:
        setattr(s, name, d[name])
    return s


def make_tol(d: dict) -> Tol:
    return Tol(d["rtol"], d["atol"], d["r_max_km"], int(d["max_steps"]))


def constants() -> dict:
    out = np.zeros(16)
    m = lib().orc_constants(_dp(out), 16)
    names = ["c_kms", "hbarc_eVkm", "alpha", "m_e_eV", "e_statC", "GMsun_km", "gauss_eV2", "wp2_per_ne",
             "hbar_omega_c_per_G"]
    return dict(zip(names, out[:m]))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniforms(seed, instance, i):
    u = np.zeros(6)
    lib().orc_uniforms(seed, instance, i, _dp(u))
    return u


def wp2(s, x, t):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_wp2(C.byref(make_star(s)), _dp(x), t)


def bfield(s, x, t):
    x = np.ascontiguousarray(x, dtype=np.float64)
    B = np.zeros(3)
    lib().orc_bfield(C.byref(make_star(s)), _dp(x), t, _dp(B))
    return B


def hamiltonian(s, y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_hamiltonian(C.byref(make_star(s)), _dp(y))


def grad_h(s, y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(8)
    lib().orc_grad_h(C.byref(make_star(s)), _dp(y), _dp(g))
    return g


def inverse_metric(s, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.zeros(9)
    lib().orc_inverse_metric(C.byref(make_star(s)), _dp(x), _dp(g))
    return g.reshape(3, 3)


def resonance_radius(s, nhat, khat, t0):
    nh = np.ascontiguousarray(nhat, dtype=np.float64)
    kh = np.ascontiguousarray(khat, dtype=np.float64)
    return lib().orc_resonance_radius(C.byref(make_star(s)), _dp(nh), _dp(kh), t0)


def energy(s, x, t, k):
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    return lib().orc_energy_aniso(C.byref(make_star(s)), _dp(x), t, _dp(k))


def sample(s, seed, n, instance=0, first=0, nthreads=0):
    """Seeds: returns (rays[10, n] = x, y, z, t, kx, ky, kz, kt, w, r_c; status[n])."""
    rays = np.zeros((10, n))
    st = np.zeros(n, dtype=np.int32)
    lib().orc_sample(C.byref(make_star(s)), seed, instance, first, n, _dp(rays), _ip(st), nthreads)
    return rays, st


def trace_forward(s, t, rays, status=None, nthreads=0, kinks=True):
    """Trace seeds to r_max.  Returns (fin[16, n], ifin[3, n] = n_acc, n_rej, status).
    kinks: cut and restart steps at the GJ density's null surface (the forward-tracing
    definition); False integrates |g| as it stands (the adjoint's discretised map)."""
    rays = np.ascontiguousarray(rays, dtype=np.float64)
    n = rays.shape[1]
    if rays.shape[0] < 10:
        full = np.zeros((10, n))
        full[:rays.shape[0]] = rays
        rays = full
    fin = np.zeros((NFIN, n))
    ifin = np.zeros((NIFIN, n), dtype=np.int32)
    stp = None if status is None else _ip(np.ascontiguousarray(status, dtype=np.int32))
    lib().orc_trace_forward(C.byref(make_star(s)), C.byref(make_tol(t)), _dp(rays), stp, n, _dp(fin), _ip(ifin),
                            nthreads, 1 if kinks else 0)
    return fin, ifin


def trace_reverse(s, t, states, lam, nthreads=0):
    states = np.ascontiguousarray(states, dtype=np.float64)
    n = states.shape[1]
    buf = np.zeros((10, n))
    buf[:8] = states[:8]
    buf[8] = lam
    fin = np.zeros((NFIN, n))
    ifin = np.zeros((NIFIN, n), dtype=np.int32)
    lib().orc_trace_reverse(C.byref(make_star(s)), C.byref(make_tol(t)), _dp(buf), n, -1.0, _dp(fin), _ip(ifin),
                            nthreads)
    return fin, ifin


def bin_flux(fin, ifin, w, bins):
    fin = np.ascontiguousarray(fin)
    ifin = np.ascontiguousarray(ifin)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = fin.shape[1]
    nt, npsi, nw = bins["n_theta"], bins["n_psi"], bins["n_omega"]
    hist = np.zeros((nt, npsi, nw))
    cnt = np.zeros((nt, npsi, nw))
    over = np.zeros(2)
    lib().orc_bin(_dp(fin), _ip(ifin), _dp(w), n, nt, npsi, nw, bins["d_omega"], _dp(hist), _dp(cnt), _dp(over))
    return hist, cnt, over


def trace_backward(s, t, image, K=8, i0=0, j0=0, stride=1, ni=None, nj=None, nthreads=0):
    nx, ny = image["nx"], image["ny"]
    ni = nx if ni is None else ni
    nj = ny if nj is None else nj
    n = ni * nj
    ev = np.zeros((K, NEV, n))
    nev = np.zeros(n, dtype=np.int32)
    fin = np.zeros((NFIN, n))
    ifin = np.zeros((NIFIN, n), dtype=np.int32)
    lib().orc_trace_backward(C.byref(make_star(s)), C.byref(make_tol(t)), image["D_km"], image["incl"],
                             image["phi_o"], image["half_width_km"], nx, ny, i0, j0, stride, ni, nj, K, _dp(ev),
                             _ip(nev), _dp(fin), _ip(ifin), nthreads)
    return ev, nev, fin, ifin


def backward_rays(s, t, D_km, incl, phi_o, b1, b2, K=8, Lc_max_km=0.0, nthreads=0):
    """Backward rays through the image-plane points (b1[q], b2[q]) [km].  Returns the
    per-ray sum of event weights wsum[n] (dP/dOmega per unit image area, eV^4; multiply
    by the pixel area in eV^-2), and the events, counts and final states."""
    b1 = np.ascontiguousarray(b1, dtype=np.float64)
    b2 = np.ascontiguousarray(b2, dtype=np.float64)
    n = b1.shape[0]
    wsum = np.zeros(n)
    ev = np.zeros((K, NEV, n))
    nev = np.zeros(n, dtype=np.int32)
    fin = np.zeros((NFIN, n))
    ifin = np.zeros((NIFIN, n), dtype=np.int32)
    lib().orc_backward_rays(C.byref(make_star(s)), C.byref(make_tol(t)), D_km, incl, phi_o, _dp(b1), _dp(b2), n, K,
                            Lc_max_km, _dp(wsum), _dp(ev), _ip(nev), _dp(fin), _ip(ifin), nthreads)
    return wsum, ev, nev, fin, ifin


def cyclotron_depth(s, fin, ifin, r_emit):
    """Resonant cyclotron optical depth tau[n] of escaped forward rays and the resonance radius
    r_cyc[n] (-1 where there is none)."""
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    ifin = np.ascontiguousarray(ifin, dtype=np.int32)
    r_emit = np.ascontiguousarray(r_emit, dtype=np.float64)
    n = fin.shape[1]
    tau, rc = np.zeros(n), np.zeros(n)
    lib().orc_cyclotron_depth(C.byref(make_star(s)), _dp(fin), _ip(ifin), _dp(r_emit), n, _dp(tau), _dp(rc))
    return tau, rc


def open_field(s, x, t):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return bool(lib().orc_open_field(C.byref(make_star(s)), _dp(x), float(t)))


def maxwell_x(u):
    """(|k_inf|/k0)^2 at quantile u of the Maxwellian momentum distribution."""
    return lib().orc_maxwell_x(float(u))


def event_weight(s, y, Lc_max_km=0.0):
    """Weight [eV^4] and conversion length [km] of one production event at state y[8]."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = C.c_double()
    lc = C.c_double()
    lib().orc_event_weight(C.byref(make_star(s)), _dp(y), Lc_max_km, C.byref(w), C.byref(lc))
    return w.value, lc.value


def dopri_test(problem, rtol, atol, t_end, h_fixed=0.0):
    y = np.zeros(8)
    na = C.c_int64()
    nr = C.c_int64()
    de = C.c_double()
    lib().orc_dopri_test(problem, rtol, atol, t_end, _dp(y), C.byref(na), C.byref(nr), h_fixed, C.byref(de))
    return y, na.value, nr.value, de.value


def flux_fwdmode(s, t, seed, n, obs, sigma, nthreads=0, per_ray=False):
    """Smoothed flux F[n_obs] and dF/dp [n_obs, 6] by forward mode (steps frozen).
    per_ray=True also returns each ray's share fray[n, n_obs], dray[n, n_obs, 6]
    and status[n]."""
    obs = np.ascontiguousarray(obs, dtype=np.float64)
    nobs = obs.shape[0]
    flux = np.zeros(nobs)
    dflux = np.zeros((nobs, 6))
    if per_ray:
        fray, dray, st = np.zeros((n, nobs)), np.zeros((n, nobs, 6)), np.zeros(n, dtype=np.int32)
        pf, pd, ps = _dp(fray), _dp(dray), _ip(st)
    else:
        pf = pd = None
        ps = None
    lib().orc_flux_fwdmode(C.byref(make_star(s)), C.byref(make_tol(t)), seed, n, _dp(obs), nobs, sigma, _dp(flux),
                           _dp(dflux), pf, pd, ps, nthreads)
    if per_ray:
        return flux, dflux, fray, dray, st
    return flux, dflux


def flux_replay(s, t, seed, n, obs, sigma, record, hseq=None, nseq=None, stat=None, max_rec=4096, nthreads=0):
    obs = np.ascontiguousarray(obs, dtype=np.float64)
    nobs = obs.shape[0]
    if record:
        hseq = np.zeros((n, max_rec))
        nseq = np.zeros(n, dtype=np.int32)
        stat = np.zeros(n, dtype=np.int32)
    flux = np.zeros(nobs)
    lib().orc_flux_replay(C.byref(make_star(s)), C.byref(make_tol(t)), seed, n, _dp(obs), nobs, sigma,
                          1 if record else 0, hseq.shape[1], _dp(hseq), _ip(nseq), _ip(stat), _dp(flux), nthreads)
    return flux, hseq, nseq, stat


def smoothed_flux(fin, ifin, w, obs, sigma, n_total):
    """F_j = (1/N) sum over escaped rays of w K(n.o_j), K(c) = exp((c - 1)/s^2) / (2 pi s^2)."""
    esc = ifin[2] == 1
    th, ps = fin[8][esc], fin[10][esc]
    nh = np.stack([np.sin(th) * np.cos(ps), np.sin(th) * np.sin(ps), np.cos(th)], axis=1)
    c = nh @ np.asarray(obs).T
    K = np.exp((c - 1.0) / sigma ** 2) / (2.0 * np.pi * sigma ** 2)
    return (w[esc][:, None] * K).sum(axis=0) / n_total
