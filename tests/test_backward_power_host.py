"""The library's backward event weight and resonant cyclotron depth
(paper_2309_08655_amd/csrc/rt_seed.hpp), compiled for the host from the same source, against
the oracle's on the oracle's own events and rays.  The two share no code: the library
derives dE/dx implicitly from H = 0 with its hand-written gradient of H, the oracle
differentiates the LO energy with dual numbers; the library refines the cyclotron
resonance by log-space steps, the oracle bisects.  Runs without a GPU."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hpow(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hostpow") / "host_power.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.run([hipcc, "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", out,
                    os.path.join(ROOT, "tests", "host_power.cpp")], check=True, capture_output=True)
    L = C.CDLL(out)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    L.host_event_weight.restype = C.c_double
    L.host_event_weight.argtypes = [dp, dp, ip, dp, C.c_double, dp]
    L.host_cyclotron_tau.restype = C.c_double
    L.host_cyclotron_tau.argtypes = [dp, dp, ip, dp, C.c_double, dp]
    return L


def _star_arrays(s):
    p = np.array([s[k] for k in ("B0_G", "P_s", "theta_m", "M_Msun", "R_km", "m_a_eV")])
    fd = np.array([s[k] for k in ("g_agg_GeV", "v0_kms", "rho_GeVcm3", "multiplicity", "psi_twist", "B_test_G")])
    fi = np.array([s["plasma"], s["density"], s["weights"], s["kdir"], s["speeds"], s["flags"]], dtype=np.int32)
    return p, fd, fi


def host_weight(L, s, y, Lc_max=0.0):
    P = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    p, fd, fi = _star_arrays(s)
    lc = C.c_double()
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = L.host_event_weight(P(p), P(fd), fi.ctypes.data_as(C.POINTER(C.c_int)), P(y), Lc_max, C.byref(lc))
    return w, lc.value


CASES = {
    "magnetar_aniso_gr": (W.CFG3["star"], 1.0, 0.0, 30.0),
    "magnetar_iso_gr": (dict(W.CFG3["star"], plasma=W.PLASMA_ISO), 1.0, 0.0, 30.0),
    "spherical_constb_gr": (W.star(M_Msun=1.4, density=W.DENSITY_SPHERICAL, plasma=W.PLASMA_ISO,
                                   weights=W.WEIGHTS_CONST_B), 0.4, 1.1, 12.0),
    "gj_aniso_oblique": (W.star(M_Msun=1.4, theta_m=0.3, plasma=W.PLASMA_ANISO, m_a_eV=1e-5), 1.0, 0.3, 30.0),
    "magnetar_M2_excised": (W.MAGNETAR_MODELS["M2"], 1.0, 0.0, 30.0),
    "spherical_aniso_oblique": (W.star(M_Msun=1.4, density=W.DENSITY_SPHERICAL, plasma=W.PLASMA_ANISO,
                                       theta_m=0.7, m_a_eV=1e-5), 0.9, 0.2, 12.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_event_weight_matches_oracle(orc, hpow, name):
    s, incl, phi_o, half = CASES[name]
    rng = np.random.default_rng(11)
    b1, b2 = rng.uniform(-half, half, 48), rng.uniform(-half, half, 48)
    t = W.tol(r_max_km=1e5, rtol=1e-10, atol=1e-14)
    wsum, ev, nev, fin, ifin = orc.backward_rays(s, t, 1e5, incl, phi_o, b1, b2, K=8)
    checked = 0
    lcs, errs, lerrs = [], [], []
    for q in np.nonzero(nev)[0]:
        for e in range(min(nev[q], 8)):
            y = ev[e, :8, q]
            wo, lo = orc.event_weight(s, y)
            wh, lh = host_weight(hpow, s, y)
            # off the dispersion shell the two routes to dE/dx differ at O(H)
            scale = 1.0 if s["plasma"] == W.PLASMA_ISO else 1e-11 + 2.0 * abs(orc.hamiltonian(s, y))
            errs.append(abs(wh / wo - 1) / scale)
            lerrs.append(abs(lh / lo - 1) / scale)
            lcs.append(lo)
            checked += 1
    assert checked >= 8
    # isotropic: the same arithmetic up to rounding.  Anisotropic: dE/dx by two routes, the
    # library's implicit one from H(x, k_t, k) = 0 at the event's k_t and the oracle's LO
    # energy differentiated at the event's k; on the shell they coincide, so they may
    # differ by twice the event's own |H| (integration drift) plus rounding
    tol = 1e-13 if s["plasma"] == W.PLASMA_ISO else 1.0
    assert max(errs) < tol and max(lerrs) < tol, (max(errs), max(lerrs))
    # the cutoff keeps or drops an event on both sides alike
    cut = float(np.median(lcs))
    for q in np.nonzero(nev)[0]:
        for e in range(min(nev[q], 8)):
            y = ev[e, :8, q]
            wo, lo = orc.event_weight(s, y, cut)
            wh, _ = host_weight(hpow, s, y, cut)
            if abs(lo / cut - 1) > 1e-9:
                assert (wo == 0.0) == (wh == 0.0)


@pytest.mark.parametrize("name", ["gj_iso_oblique", "magnetar_M4"])
def test_cyclotron_depth_matches_oracle(orc, hpow, name):
    s = {"gj_iso_oblique": W.star(M_Msun=1.0, theta_m=0.4, plasma=W.PLASMA_ISO, m_a_eV=1e-5),
         "magnetar_M4": W.MAGNETAR_MODELS["M4"]}[name]
    t = W.tol()
    rays, st = orc.sample(s, 4, 300)
    fin, ifin = orc.trace_forward(s, t, rays, st)
    tau, rcyc = orc.cyclotron_depth(s, fin, ifin, rays[9])
    esc = np.nonzero(ifin[2] == W.STATUS_ESCAPED)[0]
    assert len(esc) >= 50
    p, fd, fi = _star_arrays(s)
    P = lambda a: np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))
    nres = 0
    for q in esc:
        rr = C.c_double()
        th = hpow.host_cyclotron_tau(P(p), P(fd), fi.ctypes.data_as(C.POINTER(C.c_int)), P(fin[:, q]), rays[9, q],
                                     C.byref(rr))
        assert abs(rr.value - rcyc[q]) <= 1e-13 * abs(rcyc[q]), (q, rr.value, rcyc[q])
        assert abs(th - tau[q]) <= 1e-12 * abs(tau[q]), (q, th, tau[q])
        nres += tau[q] > 0
    assert nres >= 50
