"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds parameter sets only (star, plasma, axion, tolerances, bins,
image plane, instance grids).  It contains none of the ray-tracing arithmetic,
so both the GPU path and the CPU oracle can take their inputs from it without
sharing any of the method's code.

Physical parameters follow the fiducial set of the paper (Sec. 5): coupling
g = 1e-12 GeV^-1, dark-matter density 0.45 GeV cm^-3, axion speed 220 km/s,
R = 10 km; each workload states its own deviations.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# enumerations of the star/plasma description (same numbering on both sides of the
# boundary; they are part of the interface)
PLASMA_ISO, PLASMA_ANISO = 0, 1
DENSITY_GJ, DENSITY_MAGNETAR, DENSITY_SPHERICAL, DENSITY_NONE = 0, 1, 2, 3
WEIGHTS_UNIT, WEIGHTS_CONVERSION, WEIGHTS_CONST_B = 0, 1, 2
KDIR_ISOTROPIC, KDIR_OUTWARD = 0, 1
SPEEDS_MONO, SPEEDS_MAXWELL = 0, 1
FLAG_EXCISE_OPEN = 1  # no conversion on open magnetic field lines (Sec. 6)
FLAG_FLAT_PROPAGATION = 2  # curved initial conditions, M = 0 in the tracing (App. B)
FLAG_RENORM_WEIGHTS = 4  # P_ag = 1 and the rescaling R_i of Sec. 6 eq. (reweight)
FLAG_THIN_SURFACE = 8  # resonance on w_p = m_a instead of k^a = k^gamma (App. B)
FLAG_GR_DIPOLE = 16  # the Schwarzschild vacuum dipole field instead of the flat one
FLAG_FINITE_LARMOR = 32  # the cold magnetised plasma at finite cyclotron frequency (Sec. 4.1)

STATUS_OK, STATUS_ESCAPED, STATUS_HIT_STAR, STATUS_NO_RESONANCE = 0, 1, 2, 3
STATUS_MAX_STEPS, STATUS_STEP_UNDERFLOW, STATUS_NONFINITE, STATUS_EXCISED = 4, 5, 6, 7

FIDUCIAL = dict(
    B0_G=1e14, P_s=1.0, theta_m=0.0, M_Msun=1.0, R_km=10.0, m_a_eV=1e-5,
    g_agg_GeV=1e-12, v0_kms=220.0, rho_GeVcm3=0.45, multiplicity=1.0, psi_twist=0.2,
    B_test_G=1e12, plasma=PLASMA_ANISO, density=DENSITY_GJ, weights=WEIGHTS_CONVERSION,
    kdir=KDIR_ISOTROPIC, speeds=SPEEDS_MONO, flags=0,
)

TOL = dict(rtol=1e-8, atol=1e-12, r_max_km=1e4, max_steps=1 << 20)


def star(**over) -> dict:
    s = copy.deepcopy(FIDUCIAL)
    for k, v in over.items():
        if k not in s:
            raise KeyError(f"unknown star field {k}")
        s[k] = v
    return s


def tol(**over) -> dict:
    t = dict(TOL)
    t.update(over)
    return t


# -- the workloads ----------------------------------------------------------------------
# plain forward trace, small: flat metric, aligned dipole, isotropic plasma,
#    outward axion directions, 32 x 64 x 32 bins.
CFG1 = dict(
    name="forward-small-flat-iso-4096",
    star=star(M_Msun=0.0, theta_m=0.0, plasma=PLASMA_ISO, m_a_eV=1e-5, kdir=KDIR_OUTWARD),
    tol=tol(), n=4096, seed=0,
    bins=dict(n_theta=32, n_psi=64, n_omega=32, d_omega=6.25e-5),
)
# full forward trace: Schwarzschild M = 1.4, oblique rotator, anisotropic LO plasma.
CFG2 = dict(
    name="forward-full-gr-aniso-oblique-1e6",
    star=star(M_Msun=1.4, theta_m=0.3, plasma=PLASMA_ANISO, m_a_eV=2e-5, kdir=KDIR_ISOTROPIC),
    tol=tol(), n=1_000_000, seed=0,
    bins=dict(n_theta=64, n_psi=128, n_omega=64, d_omega=3.125e-5),
)
# backward image: 1024^2 pixels at 1e5 km, inclination 60 deg, magnetar-like star
#    with the twisted-magnetosphere density (model M1: lambda = 1, psi = 0.2).
CFG3 = dict(
    name="backward-image-1024sq-magnetar",
    star=star(B0_G=1.6e14, P_s=3.76, theta_m=0.5, M_Msun=1.4, plasma=PLASMA_ANISO,
              density=DENSITY_MAGNETAR, m_a_eV=1e-4, multiplicity=1.0, psi_twist=0.2),
    tol=tol(r_max_km=1e5),
    image=dict(D_km=1e5, incl=math.radians(60.0), phi_o=0.0, half_width_km=80.0, nx=1024, ny=1024),
    K=8,
)
# adjoint: the small forward trace's star (flat metric, aligned rotator, isotropic plasma,
# GJ density) with 1e6 rays, Gaussian-smoothed flux at 32 observers.
CFG5 = dict(
    name="adjoint-smoothed-flux-1e6",
    star=CFG1["star"], tol=tol(), n=1_000_000, seed=0, n_obs=32, sigma=0.02, ckpt_every=64,
)


# The four magnetar models of Sec. 6 (the twisted-magnetosphere density, psi = 0.2, P = 3.76 s,
# M = 1.4, theta_m = 0.5 as in the backward workload): (lambda, B0) = M1 (1, 1.6e14 G),
# M2 (20, 1.6e14 G), M3 (1, 4e14 G), M4 (20, 4e14 G), with conversion on open field lines
# removed.
MAGNETAR_MODELS = {
    name: star(B0_G=B0, P_s=3.76, theta_m=0.5, M_Msun=1.4, plasma=PLASMA_ANISO, density=DENSITY_MAGNETAR,
               m_a_eV=1e-4, multiplicity=lam, psi_twist=0.2, flags=FLAG_EXCISE_OPEN)
    for name, lam, B0 in (("M1", 1.0, 1.6e14), ("M2", 20.0, 1.6e14), ("M3", 1.0, 4e14), ("M4", 20.0, 4e14))
}


# A weakly magnetised test star for the finite-magnetisation Hamiltonian (Sec. 4.1 eq.
# (DisRel)): the kink-free spherical density of the fiducial star (B0 multiplicity kept at
# 1e14 G) under a 1e6 G dipole, so that the electron cyclotron frequency is 11-26 times the
# photon frequency on the resonance (about 35 km) and still above twice it at r_max = 60 km,
# where the finite-magnetisation terms change the rays at the 1e-3 level.  Everywhere on the
# traced path the plasma stays magnetised (the two magnetoionic modes well separated).
WEAK_FIELD = dict(
    name="weak-field-finite-larmor",
    star=star(M_Msun=1.4, theta_m=0.3, plasma=PLASMA_ANISO, density=DENSITY_SPHERICAL, m_a_eV=1e-5, B0_G=1e6,
              multiplicity=1e8, kdir=KDIR_OUTWARD, flags=FLAG_FINITE_LARMOR),
    tol=tol(r_max_km=60.0), seed=0,
)


def observers(n_obs: int = 32) -> np.ndarray:
    """Observer directions in the (x, z) plane at polar angles (j + 1/2) pi / n_obs."""
    th = (np.arange(n_obs) + 0.5) * math.pi / n_obs
    return np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=1)


def batched_instances(n_inst: int = 256, seed: int = 1, n_lo: float = 1e4, n_hi: float = 2e5):
    """The batched scan: 16 axion masses (log-spaced over [1e-6, 1e-4] eV) x 16 inclinations
    (linear over [0, 1.2] rad) of the small forward trace's star; ray counts log-uniform over
    [n_lo, n_hi] drawn with numpy's PCG64 seeded `seed`."""
    side = int(round(math.sqrt(n_inst)))
    rng = np.random.default_rng(seed)
    u = rng.random(n_inst)
    counts = np.floor(np.exp(math.log(n_lo) + u * (math.log(n_hi) - math.log(n_lo)))).astype(np.int64)
    stars = []
    for k in range(n_inst):
        ia, it = k % side, k // side
        ma = 10.0 ** (-6.0 + 2.0 * ia / (side - 1))
        thm = 1.2 * it / (side - 1)
        stars.append(star(M_Msun=0.0, theta_m=thm, plasma=PLASMA_ISO, m_a_eV=ma, kdir=KDIR_OUTWARD))
    return stars, counts


def final_records(n: int, bins: dict, seed: int = 0, hot_frac: float = 0.3, out_frac: float = 0.02):
    """Synthetic final records of n traced rays for binning tests: float64 fin [16, n] and
    int32 ifin [3, n] in the tracer's layout (theta in fin[8], co-rotating azimuth in fin[10],
    energy at infinity in fin[11], status in ifin[2]) and positive weights w [n].

    Directions are uniform on the sphere, energies spread over the frequency bins with a
    fraction out_frac beyond them; a fraction hot_frac of the rays is piled into eight
    directions at omega = 1 (the sharp line of the signal), which makes hot bins; 10 %
    of the rays carry a status other than escaped.  numpy PCG64 seeded `seed`."""
    rng = np.random.default_rng(seed)
    fin = np.zeros((16, n))
    ifin = np.zeros((3, n), dtype=np.int32)
    fin[8] = np.arccos(1.0 - 2.0 * rng.random(n))
    fin[10] = 2.0 * math.pi * rng.random(n)
    half = 0.5 * bins["n_omega"] * bins["d_omega"]
    fin[11] = 1.0 + (2.0 * rng.random(n) - 1.0) * half * (1.0 + 2.0 * out_frac)
    hot = rng.random(n) < hot_frac
    spot = rng.integers(0, 8, n)
    fin[8][hot] = (0.3 + 0.3 * spot[hot]) % math.pi
    fin[10][hot] = 0.7 * spot[hot] + 0.1
    fin[11][hot] = 1.0
    ifin[2] = np.where(rng.random(n) < 0.9, STATUS_ESCAPED,
                       rng.choice([STATUS_HIT_STAR, STATUS_MAX_STEPS, STATUS_NO_RESONANCE], n)).astype(np.int32)
    w = np.exp(rng.normal(0.0, 2.0, n))
    return fin, ifin, w


CFG4 = dict(name="batched-256-instances", n_inst=256, seed=1, bins=dict(n_theta=64, n_psi=128, n_omega=1,
                                                                        d_omega=1.0))
