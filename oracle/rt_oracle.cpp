// CPU oracle for the ray-tracing hot path of McDonald & Witte,
// "Generalized Ray Tracing for Axions in Astrophysical Plasmas" (arXiv:2309.08655).
//
// TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
// baseline leg of the benchmark, never by the product path.  Plain scalar FP64
// C++, one ray at a time (OpenMP over rays).  Every derivative comes from
// forward-mode dual numbers (dual.hpp) applied to the defining formulas.  The
// code follows the paper's statement of the method, section by section:
//
//   Sec. 2, eq. (Hamilton)            rays are characteristics x' = dH/dk, k' = -dH/dx
//   Sec. 4.1, eqs. (StrongBHam), (SchwarzshildMetric1)
//                                     H = g^{mu nu} k k + (w^2 - k_par^2) w_p^2 / w^2,
//                                     static plasma frame, Schwarzschild metric
//   Sec. 4.1, eq. (AnisotropicDisp)   LO-mode energy (+ branch)
//   Sec. 4.2, eqs. (RaidalHypersurface), (PowerCurved), (redshift)
//                                     surface measure sqrt|g_tt| sqrt|h_k| of the foliation
//   Sec. 4.3, eq. (fa_approx)         monochromatic axions, focused density n_c
//   Sec. 4.4, eqs. (ProbIsoCurved), (CPAnisoCurved), (CosIso), (AngleDefAniso)
//                                     conversion probability times the flux projection
//   Sec. 5, eq. (GJDensity), Sec. 6, eq. (neMag)
//                                     Goldreich-Julian and twisted-magnetar densities
//   Sec. 2.2, eq. (Power)             forward Monte Carlo estimator binned with a top-hat window
//   Sec. 2.1, eq. (BackPower), Sec. 3 backward rays from an image plane; every level crossing
//                                     k_gamma = k_a along the ray is a production site
//
// Where the paper is silent or ambiguous the reading taken is stated in place.
// The integrator is Dormand-Prince 5(4) (Dormand & Prince 1980) with the
// continuous extension, error norm, step controller and starting-step rule of
// Hairer, Norsett & Wanner, "Solving ODEs I", Sec. II.4-II.6.  The random
// numbers are Philox4x32-10 (Salmon et al., SC'11).

#include "oracle.h"
#include "dual.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------------------
// Units and constants: CODATA 2018 and the IAU 2015 nominal solar mass
// parameter.  Natural units are Heaviside-Lorentz with hbar = c = 1.
// ---------------------------------------------------------------------------
static const double PI = 3.14159265358979323846;
static const double C_KMS = 299792.458;           // speed of light [km/s]
static const double C_CMS = 2.99792458e10;         // [cm/s]
static const double HBARC_EVKM = 1.973269804e-10;  // hbar c [eV km]
static const double HBARC_EVCM = 1.973269804e-5;   // hbar c [eV cm]
static const double ALPHA = 1.0 / 137.035999084;   // fine-structure constant
static const double M_E_EV = 510998.95;            // electron mass [eV]
static const double E_STATC = 4.803204712570263e-10;  // elementary charge [statC]
static const double GM_SUN_KM = 1.4766250;         // G M_sun / c^2 [km]
static const double EV_PER_ERG = 1.0 / 1.602176634e-12;

// 1 gauss in eV^2: equate the field energy density B^2/(8 pi) [erg cm^-3]
// (Gaussian) with B^2/2 (Heaviside-Lorentz natural units).
static double gauss_in_eV2() { return std::sqrt(EV_PER_ERG * HBARC_EVCM * HBARC_EVCM * HBARC_EVCM / (4.0 * PI)); }
// plasma frequency squared per unit electron density: w_p^2 = 4 pi alpha n_e / m_e  [eV^2 cm^3]
// (the paper writes 4 pi n_e / m_e with e^2 absorbed; the textbook factor alpha is restored)
static double wp2_per_ne() { return 4.0 * PI * ALPHA * HBARC_EVCM * HBARC_EVCM * HBARC_EVCM / M_E_EV; }

enum { PL_ISO = 0, PL_ANISO = 1 };
enum { DEN_GJ = 0, DEN_MAG = 1, DEN_SPH = 2, DEN_NONE = 3 };
enum { W_UNIT = 0, W_CONV = 1, W_CONV_CONSTB = 2 };
enum { SP_MONO = 0, SP_MAXWELL = 1 };
enum { KD_ISO = 0, KD_OUT = 1 };

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw 2011).
// ---------------------------------------------------------------------------
static void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k[0] += W0; k[1] += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// 52 random bits -> a double strictly inside (0, 1): (m + 1/2) 2^-52, exact.
static double bits_to_unit(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)m + 0.5) * (1.0 / 4503599627370496.0);
}

// Six uniforms for ray i of an instance: three Philox blocks with
// counter (i_lo, i_hi, instance, block) and key (seed_lo, seed_hi).
static void ray_uniforms(uint64_t seed, int32_t instance, int64_t i, double u[6]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t blk = 0; blk < 3; ++blk) {
        uint32_t ctr[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)instance, blk};
        uint32_t o[4];
        philox(ctr, key, o);
        u[2 * blk] = bits_to_unit(o[0], o[1]);
        u[2 * blk + 1] = bits_to_unit(o[2], o[3]);
    }
}

// ---------------------------------------------------------------------------
// Maxwellian momenta at infinity, eq. (GaussianDist): f ~ exp(-k^2/k0^2), so x = (k/k0)^2
// has the Gamma(3/2) distribution (density x^{1/2} e^{-x} / Gamma(3/2)), with distribution
// function G(x) = P(3/2, x), the regularised lower incomplete gamma function:
//   G(x)     = x^{3/2} e^{-x} / Gamma(5/2) sum_{j>=0} x^j / ((5/2)(7/2)...(3/2 + j))
//              (the power series, every term positive),
//   1 - G(x) = erfc(sqrt x) + (2/sqrt pi) sqrt(x) e^{-x}.
// x is the root of G(x) = u (u < 1/2, by the series) or of 1 - G(x) = 1 - u (u >= 1/2, where
// the complement keeps its digits), found by bisection on [0, 100].
// ---------------------------------------------------------------------------
static double gamma32_lower(double x) {
    double term = 1.0, sum = 1.0;
    for (int j = 1; j < 200; ++j) {
        term *= x / (1.5 + j);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return std::pow(x, 1.5) * std::exp(-x) / (0.75 * std::sqrt(PI)) * sum;
}

static double maxwell_x(double u) {
    const double c = 2.0 / std::sqrt(PI);
    const bool upper = u >= 0.5;
    const double target = upper ? 1.0 - u : u;
    auto f = [&](double x) {
        const double s = std::sqrt(x);
        return upper ? std::erfc(s) + c * s * std::exp(-x) : gamma32_lower(x);
    };
    double lo = 0.0, hi = 100.0;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        // G increases with x; 1 - G decreases
        const bool below = upper ? (f(mid) > target) : (f(mid) < target);
        if (below) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// Star instance.  The six differentiable parameters (B0, P, theta_m, M, R, m_a)
// are of type P (double, or a dual number for forward-mode derivatives).
// ---------------------------------------------------------------------------
template <class P>
struct Inst {
    P rs;      // Schwarzschild radius 2GM [km]
    P R;       // stellar radius [km]
    P Om;      // angular velocity / c [rad km^-1]
    P cm, sm;  // cos, sin of the magnetic inclination
    P B0;      // polar surface field [G]
    P Cwp;     // w_p^2 / w_inf^2 = Cwp * (density shape)
    P ma2;     // (m_a / w_inf)^2
    double kv2;  // (k0 / w_inf)^2 = v0^2 / (1 + v0^2) = 1 - ma2, formed without cancellation
    P w_inf;   // axion energy at infinity [eV]
    P n_inf;   // axion number density at infinity [eV^3]
    P k0;      // axion momentum at infinity [eV]
    P Period;  // [s]
    P kL;      // (hbar e / (m_e c) / w_inf)^2 [G^-2]: (w_L / w_inf)^2 = kL |B|^2, w_L the cyclotron frequency
    double g_eV;   // coupling [eV^-1]
    double Btest;  // constant |B_perp| of the zero-variance test [G]
    int plasma, density, weights, kdir, speeds, flags;
    // GJ density only: 0 = the density itself, |g|; +1 or -1 = the smooth piece s g of it
    // that forward tracing integrates between crossings of the null surface g = 0
    double gj_branch;
};

template <class P>
static Inst<P> make_inst(const orc_star& s, const P p[6]) {
    Inst<P> I;
    const P& B0 = p[0]; const P& Ps = p[1]; const P& th = p[2];
    const P& M = p[3]; const P& R = p[4]; const P& ma = p[5];
    I.rs = 2.0 * GM_SUN_KM * M;
    I.R = R;
    P Om_s = 2.0 * PI / Ps;                 // rad/s
    I.Om = Om_s / C_KMS;                    // rad/km
    I.cm = cos(th); I.sm = sin(th);
    I.B0 = B0;
    I.Period = Ps;
    double v0 = s.v0_kms / C_KMS;
    I.w_inf = ma * std::sqrt(1.0 + v0 * v0);  // w_inf^2 = m_a^2 + k0^2 with k0 = m_a v0
    I.k0 = ma * v0;
    I.ma2 = P(1.0 / (1.0 + v0 * v0)) + 0.0 * ma;  // (m_a/w_inf)^2 does not depend on m_a
    I.kv2 = v0 * v0 / (1.0 + v0 * v0);
    P Cp = wp2_per_ne() / (I.w_inf * I.w_inf);   // [cm^3]
    // Goldreich-Julian: n = 2 Omega.B / e (Heaviside-Lorentz) = Omega B0/(4 pi e c) (R/r)^3 |...| (Gaussian)
    P n0 = Om_s * B0 / (4.0 * PI * E_STATC * C_CMS);
    switch (s.density) {
        case DEN_GJ: I.Cwp = Cp * s.multiplicity * n0; break;
        // twisted magnetar: n_e = lambda psi B0 (R/r)^3 sin^2 / (4 pi e r), r in cm (= 1e5 r_km)
        case DEN_MAG: I.Cwp = Cp * s.multiplicity * s.psi_twist * B0 / (4.0 * PI * E_STATC * 1.0e5); break;
        case DEN_SPH: I.Cwp = Cp * s.multiplicity * n0; break;
        default: I.Cwp = P(0.0); break;
    }
    double rho_eV4 = s.rho_GeVcm3 * 1.0e9 * HBARC_EVCM * HBARC_EVCM * HBARC_EVCM;
    I.n_inf = rho_eV4 / ma;
    // electron cyclotron energy per gauss, hbar e B / (m_e c) with e in statC and m_e c^2 in erg
    const double hwc = HBARC_EVCM * E_STATC / (M_E_EV / EV_PER_ERG);  // [eV / G]
    I.kL = (hwc / I.w_inf) * (hwc / I.w_inf);
    I.g_eV = s.g_agg_GeV * 1.0e-9;
    I.Btest = s.B_test_G;
    I.plasma = s.plasma; I.density = s.density; I.weights = s.weights; I.kdir = s.kdir;
    I.speeds = s.speeds;
    I.flags = s.flags;
    I.gj_branch = 0.0;
    return I;
}

static Inst<double> make_inst_d(const orc_star& s) {
    double p[6] = {s.B0_G, s.P_s, s.theta_m, s.M_Msun, s.R_km, s.m_a_eV};
    return make_inst<double>(s, p);
}

template <class A, class B> static auto dot3(const A a[3], const B b[3]) -> decltype(a[0] * b[0]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Magnetic axis at time t: it rotates about z (the rotation axis) with
// inclination theta_m.  The paper's m.r lacks the azimuth; the reading taken
// is cos(phi - Omega t), i.e. the axis rotates rigidly about z.
template <class S, class P>
static void mhat_at(const Inst<P>& I, const S& t, S m[3]) {
    S ph = I.Om * t;
    m[0] = I.sm * cos(ph);
    m[1] = I.sm * sin(ph);
    m[2] = S(0.0) + I.cm;
}

// Plasma frequency squared in units of w_inf^2 at position x, time t.
template <class S, class P>
static S wp2_tilde(const Inst<P>& I, const S x[3], const S& t) {
    if (I.density == DEN_NONE) return S(0.0);
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S n[3] = {x[0] / r, x[1] / r, x[2] / r};
    S m[3];
    mhat_at(I, t, m);
    S mu = dot3(m, n);
    S Rr = I.R / r;
    S Rr3 = Rr * Rr * Rr;
    if (I.density == DEN_GJ) {
        // |2 Omega.B| with the dipole field below: Omega.B ~ 3 cos(theta) (m.n) - cos(theta_m)
        const S g = 3.0 * n[2] * mu - I.cm;
        return I.Cwp * Rr3 * ((I.gj_branch != 0.0) ? I.gj_branch * g : fabs(g));
    }
    if (I.density == DEN_MAG) {
        // sin^2 of the magnetic colatitude
        return I.Cwp * Rr3 * (1.0 - mu * mu) / r;
    }
    return I.Cwp * Rr3;  // spherical test profile
}

// The GJ factor g = 3 cos(theta) (m.n) - cos(theta_m) at a point (its sign picks the
// smooth piece of the density; the null surface is g = 0).
template <class P>
static double gj_factor(const Inst<P>& I, const double x[3], double t) {
    const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double n[3] = {x[0] / r, x[1] / r, x[2] / r};
    const double ph = val(I.Om) * t;
    const double m[3] = {val(I.sm) * std::cos(ph), val(I.sm) * std::sin(ph), val(I.cm)};
    return 3.0 * n[2] * (m[0] * n[0] + m[1] * n[1] + m[2] * n[2]) - val(I.cm);
}

// g and its derivative along a curve with tangent (dx, dt), in any scalar type (the implicit
// derivative of a null-surface crossing): dg = 3 (dn_z mu + n_z dmu), dn = (dx - n (n.dx))/r,
// dmu = (dm/dt . n) dt + m.dn, dm/dt = Omega e_z x m.
template <class S, class P>
static S gj_factor_t(const Inst<P>& I, const S x[3], const S& t, const S dx[3], const S& dt, S* dg) {
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S n[3] = {x[0] / r, x[1] / r, x[2] / r};
    S m[3];
    mhat_at(I, t, m);
    S mu = dot3(m, n);
    S ndx = dot3(n, dx);
    S dn[3] = {(dx[0] - n[0] * ndx) / r, (dx[1] - n[1] * ndx) / r, (dx[2] - n[2] * ndx) / r};
    S mdot[3] = {(S(0.0) - I.Om) * m[1], I.Om * m[0], S(0.0)};
    S dmu = dot3(mdot, n) * dt + dot3(m, dn);
    *dg = 3.0 * (dn[2] * mu + n[2] * dmu);
    return 3.0 * n[2] * mu - I.cm;
}

// Radial profiles of the static vacuum dipole in Schwarzschild, x = r_s / r: the vector
// potential is A_phi = (mu sin^2 theta / r) G(x) with
//   G(x) = -3 [ln(1 - x) + x + x^2/2] / x^3 = 3 sum_{j>=0} x^j / (j + 3)   (G(0) = 1),
// so that, in the static orthonormal frame,
//   B_rhat = (2 mu cos theta / r^3) G,   B_thetahat = (mu sin theta / r^3) F,
//   F = sqrt(1 - x) (G + x G')   (F follows from div B = 0, G from curl(sqrt(A) B) = 0).
// The power series converges for x < 1 and has no cancellation.
template <class S>
static void gr_dipole_profiles(const S& x, S& G, S& F) {
    S g = S(0.0), gp = S(0.0), xp = S(1.0);
    for (int j = 0; j < 400; ++j) {
        g = g + xp * (3.0 / (j + 3.0));
        if (j >= 1) gp = gp + (3.0 * j / (j + 3.0)) * (xp / x);
        xp = xp * x;
        if (val(xp) < 1e-19) break;
    }
    G = g;
    F = sqrt(1.0 - x) * (g + x * gp);
}

// Dipole field of polar surface strength B0 [G], components in the static orthonormal frame:
// the flat-space dipole placed in that frame (identical at M = 0), or with the GR flag the
// Schwarzschild vacuum dipole above, normalised to B0 at the surface pole.
template <class S, class P>
static void bfield_t(const Inst<P>& I, const S x[3], const S& t, S B[3]) {
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S n[3] = {x[0] / r, x[1] / r, x[2] / r};
    S m[3];
    mhat_at(I, t, m);
    S mu = dot3(m, n);
    S Rr = I.R / r;
    S amp = 0.5 * I.B0 * Rr * Rr * Rr;
    if ((I.flags & ORC_FLAG_GR_DIPOLE) && val(I.rs) > 0.0) {
        S G, F, GR, FR;
        gr_dipole_profiles(S(0.0) + I.rs / r, G, F);
        gr_dipole_profiles(S(0.0) + I.rs / I.R, GR, FR);
        // B = (mu_B / r^3) [(2G + F) mu n - F m], mu_B = B0 R^3 / (2 G(r_s/R))
        for (int i = 0; i < 3; ++i) B[i] = (amp / GR) * ((2.0 * G + F) * mu * n[i] - F * m[i]);
        return;
    }
    for (int i = 0; i < 3; ++i) B[i] = amp * (3.0 * mu * n[i] - m[i]);
}

// Inverse metric of the Schwarzschild line element in the Cartesian chart
// x = r n (r the areal radius): g^tt = -1/A, g^ij = delta^ij - (r_s/r) n^i n^j.
template <class S, class P>
static void inverse_metric(const Inst<P>& I, const S x[3], S& gtt, S gij[3][3]) {
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S n[3] = {x[0] / r, x[1] / r, x[2] / r};
    S A = 1.0 - I.rs / r;
    gtt = -1.0 / A;
    S s = I.rs / r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gij[i][j] = ((i == j) ? 1.0 : 0.0) - s * n[i] * n[j];
}

// Orthonormal static-frame components of a spatial covector k at x:
// radial e_r = sqrt(A) d_r, tangential components unchanged.
template <class S, class P, class K>
static void ortho_components(const Inst<P>& I, const S x[3], const K k[3], S ko[3]) {
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S n[3] = {x[0] / r, x[1] / r, x[2] / r};
    S A = 1.0 - I.rs / r;
    S nk = n[0] * k[0] + n[1] * k[1] + n[2] * k[2];
    S rad = sqrt(A) * nk;
    for (int i = 0; i < 3; ++i) ko[i] = (k[i] - nk * n[i]) + rad * n[i];
}

// Finite magnetisation (Sec. 4.1): eq. (DisRel) in its rewritten form, with p^2 = k^2 + w^2
// and w_L.p = w_L.k,
//   H_L = k^2 [w^2 w_L^2 (k^2 + w_p^2) - w_p^2 (w_L.k)^2] - w^2 (w^2 - w_p^2)(k^2 + w_p^2)^2,
// where k^2 = g^{mu nu} k_mu k_nu, w^2 the frequency in the static plasma frame and (w_L.k)^2 =
// w_L^2 k_par^2.  By eq. (Larmor) w_L is the electron cyclotron frequency e|B|/(m_e c) (the
// Levi-Civita contraction of the projected field tensor gives twice the field vector).  The
// ray Hamiltonian is H_L / (w_L^2 w^2 k^2): same rays on H_L = 0 away from k^2 = 0, and as
// w_L -> infinity it becomes eq. (StrongBHam), k^2 + (w^2 - k_par^2) w_p^2 / w^2, term for term.
// Arguments: k2 = k^2, w2 = w^2, wp2 = w_p^2, kp2 = k_par^2, wL2 = w_L^2 (units of w_inf).
template <class S>
static S finite_larmor_h(const S& k2, const S& w2, const S& wp2, const S& kp2, const S& wL2) {
    S q = k2 + wp2;
    S HL = k2 * (w2 * wL2 * q - wp2 * wL2 * kp2) - w2 * (w2 - wp2) * q * q;
    return HL / (wL2 * w2 * k2);
}

// Hamiltonian, eq. (StrongBHam): H = g^{mu nu} k_mu k_nu + (w^2 - k_par^2) w_p^2 / w^2,
// with w^2 = -g^{tt} k_t^2 the frequency seen by the static plasma and k_par the
// component of k along B in that frame.  The isotropic plasma, eq. (DispIsotropic),
// is H = g^{mu nu} k_mu k_nu + w_p^2.
template <class S, class P>
static S hamiltonian_t(const Inst<P>& I, const S y[8]) {
    S x[3] = {y[0], y[1], y[2]};
    const S& t = y[3];
    S k[3] = {y[4], y[5], y[6]};
    const S& kt = y[7];
    S gtt, gij[3][3];
    inverse_metric(I, x, gtt, gij);
    S kk = S(0.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) kk = kk + gij[i][j] * k[i] * k[j];
    S gkk = gtt * kt * kt + kk;
    S wp2 = wp2_tilde(I, x, t);
    if (I.plasma == PL_ISO) return gkk + wp2;
    S w2 = -gtt * kt * kt;
    S ko[3];
    ortho_components(I, x, k, ko);
    S B[3];
    bfield_t(I, x, t, B);
    S Bmag = sqrt(dot3(B, B));
    S kpar = dot3(ko, B) / Bmag;
    if (I.flags & ORC_FLAG_FINITE_LARMOR) return finite_larmor_h(gkk, w2, wp2, kpar * kpar, I.kL * dot3(B, B));
    return gkk + (w2 - kpar * kpar) * wp2 / w2;
}

// Gradient of H with respect to the 8 phase-space coordinates, by forward-mode AD.
template <class S, class P>
static void grad_h_t(const Inst<P>& I, const S y[8], S g[8]) {
    using D = Dual<8, S>;
    D yd[8];
    for (int i = 0; i < 8; ++i) yd[i] = D::var(y[i], i);
    D H = hamiltonian_t<D, P>(I, yd);
    for (int i = 0; i < 8; ++i) g[i] = H.d[i];
}

// Hamilton's equations, eq. (Hamilton): dx^mu/dl = dH/dk_mu, dk_mu/dl = -dH/dx^mu.
template <class S, class P>
static void rhs_t(const Inst<P>& I, const S y[8], S f[8], double sign) {
    S g[8];
    grad_h_t(I, y, g);
    for (int i = 0; i < 4; ++i) { f[i] = sign * g[4 + i]; f[4 + i] = -sign * g[i]; }
}

// LO-mode energy at fixed covariant spatial momentum k, eq. (AnisotropicDisp)
// with the '+' sign; |k|^2 = g^{ij} k_i k_j.  In units of w_inf.
template <class S, class P, class K>
static S energy_t(const Inst<P>& I, const S x[3], const P& t, const K k[3]) {
    S gtt, gij[3][3];
    inverse_metric(I, x, gtt, gij);
    S kk = S(0.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) kk = kk + gij[i][j] * k[i] * k[j];
    S tt = S(0.0) + t;
    S wp2 = wp2_tilde(I, x, tt);
    if (I.plasma == PL_ISO) return sqrt(kk + wp2);
    S ko[3];
    ortho_components(I, x, k, ko);
    S B[3];
    bfield_t(I, x, tt, B);
    S c = dot3(ko, B) / sqrt(dot3(B, B) * kk);
    S disc = kk * kk + wp2 * wp2 + 2.0 * kk * wp2 * (1.0 - 2.0 * c * c);
    S E0 = sqrt(0.5 * (kk + wp2 + sqrt(disc)));
    if (!(I.flags & ORC_FLAG_FINITE_LARMOR)) return E0;
    // finite magnetisation: the root w^2 of H_L / (w_L^2 w^2 k^2) = 0 at this covariant k,
    // k^2 = |k|^2 - w^2, that continues the strong-field LO root E0^2 (Newton's method from
    // it; the tangents of S converge with the value to the implicit derivative)
    using D1 = Dual<1, S>;
    const S wL2 = I.kL * dot3(B, B);
    const S kp2 = kk * c * c;
    S W = E0 * E0;
    int extra = -1;
    for (int it = 0; it < 100 && extra != 0; ++it) {
        D1 Wd = D1::var(W, 0);
        D1 h = finite_larmor_h<D1>(D1(kk) - Wd, Wd, D1(wp2), D1(kp2), D1(wL2));
        S step = h.v / h.d[0];
        W = W - step;
        if (extra > 0) --extra;
        else if (std::fabs(val(step)) <= 1e-15 * std::fabs(val(W))) extra = 2;
    }
    return sqrt(W);
}

// ---------------------------------------------------------------------------
// Magnetar options of Sec. 6.
// Open field lines: the dipole's field lines are r = L sin^2 theta_mag; a line is open when
// its apex L reaches the light cylinder r_LC = c/Omega, so a point is on an open line when
// r / sin^2 theta_mag >= r_LC, written r >= r_LC sin^2 theta_mag (true on the magnetic axis).
// ---------------------------------------------------------------------------
template <class P>
static bool on_open_field_line(const Inst<P>& I, const double x[3], double t) {
    const double r = std::sqrt(dot3(x, x));
    const double ph = val(I.Om) * t;
    const double m[3] = {val(I.sm) * std::cos(ph), val(I.sm) * std::sin(ph), val(I.cm)};
    const double mu = dot3(m, x) / r;
    const double rLC = 1.0 / val(I.Om);  // [km]
    return r >= rLC * (1.0 - mu * mu);
}

// Resonant cyclotron absorption (Sec. 6): with the trajectory taken radial along the ray's
// asymptotic direction nhat, the photon is at radius r at time t(r) = t_f + (r - r_f) and has
// local frequency w(r) = w_f / sqrt(A(r)); the resonance is the radius where the electron
// cyclotron frequency hbar e |B| / (m_e c) equals w (dipole |B|), and there
//   tau = (pi/3) (w_p^2 / w) r.
// No absorption when the resonance lies inside the emission radius or w exceeds the cyclotron
// frequency at the surface.  The root is bracketed by doubling and bisected.
static double hbar_omega_c_per_gauss() {  // [eV / G]: hbar e B/(m_e c) in Gaussian units
    return HBARC_EVCM * E_STATC / (M_E_EV / EV_PER_ERG);
}

static double cyclotron_tau(const Inst<double>& I, const double fin[ORC_NFIN], double r_emit, double* r_res) {
    const double th = fin[8], ph = fin[9];
    const double nh[3] = {std::sin(th) * std::cos(ph), std::sin(th) * std::sin(ph), std::cos(th)};
    const double tf = fin[3], rf = fin[14];
    const double wf = fin[11] * I.w_inf;  // energy at infinity [eV]
    const double kc = hbar_omega_c_per_gauss();
    auto g = [&](double r) {
        const double x[3] = {r * nh[0], r * nh[1], r * nh[2]};
        double B[3];
        bfield_t(I, x, tf + (r - rf), B);
        return kc * std::sqrt(dot3(B, B)) - wf / std::sqrt(1.0 - I.rs / r);
    };
    *r_res = -1.0;
    const double R = I.R;
    if (!(g(R) > 0.0)) return 0.0;
    double lo = R, hi = 2.0 * R;
    for (int j = 0; j < 200 && !(g(hi) < 0.0); ++j) { lo = hi; hi *= 2.0; }
    if (!(g(hi) < 0.0)) return 0.0;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (g(mid) > 0.0) lo = mid; else hi = mid;
    }
    const double rc = 0.5 * (lo + hi);
    *r_res = rc;
    if (rc < r_emit) return 0.0;
    const double x[3] = {rc * nh[0], rc * nh[1], rc * nh[2]};
    const double tc = tf + (rc - rf);
    const double wp2 = wp2_tilde(I, x, tc) * I.w_inf * I.w_inf;  // [eV^2]
    const double w = wf / std::sqrt(1.0 - I.rs / rc);
    return (PI / 3.0) * (wp2 / w) * (rc / HBARC_EVKM);
}

// ---------------------------------------------------------------------------
// Resonance foliation (Sec. 3 eq. (Hypersurfaces), Sec. 4 kinematic matching
// k^a_mu = k^gamma_mu).  The axion has conserved k_t = -w_inf and is on shell,
// so in the static frame w^2 = w_inf^2/A and |k_a|^2 = w^2 - m_a^2.  Putting
// that momentum into the photon dispersion relation (AnisotrpoicDisp) gives
//   F = w_p^2 (w^2 - |k_a|^2 cos^2 theta_B) - m_a^2 w^2 = 0
// (isotropic plasma: F = w_p^2 - m_a^2).  k-hat is held fixed as a direction in
// the static orthonormal frame, and the emission time t0 is held fixed.  om2 is
// the square of the axion's energy at infinity in units of w_inf (1 for the
// monochromatic distribution).
// ---------------------------------------------------------------------------
template <class S, class P>
static S resonance_F(const Inst<P>& I, const S x[3], const P& t0, const double khat[3], double om2 = 1.0,
                     bool thin = false) {
    S tt = S(0.0) + t0;
    S wp2 = wp2_tilde(I, x, tt);
    if (I.plasma == PL_ISO || thin) return wp2 - I.ma2;
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S A = 1.0 - I.rs / r;
    S w2 = om2 / A;
    S ka2 = w2 - I.ma2;
    S B[3];
    bfield_t(I, x, tt, B);
    S cB = (khat[0] * B[0] + khat[1] * B[1] + khat[2] * B[2]) / sqrt(dot3(B, B));
    if (I.flags & ORC_FLAG_FINITE_LARMOR) {
        // the same matching in the finite-magnetisation Hamiltonian: w^2 H at k^2 = -m_a^2
        S ma2 = S(0.0) + I.ma2;
        return w2 * finite_larmor_h(S(0.0) - ma2, w2, wp2, ka2 * cB * cB, I.kL * dot3(B, B));
    }
    return wp2 * (w2 - ka2 * cB * cB) - I.ma2 * w2;
}

template <class P>
static P F_on_ray(const Inst<P>& I, const P& r, const double n[3], const P& t0, const double khat[3],
                  double om2, bool thin) {
    P x[3] = {r * n[0], r * n[1], r * n[2]};
    return resonance_F(I, x, t0, khat, om2, thin);
}

// Root of F along the radial line through n, above the stellar surface.
// Returns -1 when F(R) <= 0 (no resonance).  Plain bisection on a bracket
// [R, R 2^j]; for dual parameters a final Newton correction carries the
// implicit-function derivative dr/dp = -(dF/dp)/(dF/dr).
template <class P>
static P resonance_radius_t(const Inst<P>& I, const double n[3], const P& t0, const double khat[3],
                            double om2 = 1.0, bool thin = false) {
    double R = val(I.R);
    Inst<double> Id;  // value copy for the bracketing
    auto Fval = [&](double r) { return val(F_on_ray(I, P(0.0) + r, n, t0, khat, om2, thin)); };
    if (!(Fval(R) > 0.0)) return P(-1.0);
    double lo = R, hi = 2.0 * R;
    int j = 0;
    while (!(Fval(hi) < 0.0) && j < 80) { lo = hi; hi *= 2.0; ++j; }
    if (!(Fval(hi) < 0.0)) return P(-1.0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (Fval(mid) > 0.0) lo = mid; else hi = mid;
    }
    double rc = 0.5 * (lo + hi);
    if constexpr (is_dual<P>::value) {
        using D1 = Dual<1, P>;
        D1 rd = D1::var(P(0.0) + rc, 0);
        D1 xd[3] = {rd * n[0], rd * n[1], rd * n[2]};
        D1 Fd = resonance_F(I, xd, t0, khat, om2, thin);
        P corr = Fd.v / Fd.d[0];
        P out = (P(0.0) + rc) - corr;
        out.v = rc;
        return out;
    } else {
        (void)Id;
        return rc;
    }
}

// ---------------------------------------------------------------------------
// Seeding (forward tracing, Sec. 2.2 and Sec. 4.2-4.4).
//
// The estimator of the power, eq. (PowerCurved) with the monochromatic axion
// distribution of eq. (fa_approx) (int d^3k f_a = n_c dOmega_k / 4 pi), is
//   P ~ (1/N) sum_i w_i,  w = C_k n_c Vt Q,
// for emission directions uniform in (cos theta, phi) and axion directions
// uniform over a solid angle C_k (4 pi, or 2 pi for the outward hemisphere):
//   Vt = sqrt|g_tt| sqrt|h_k| / sin(theta) = A r^2 sqrt(1 + |grad_perp F|^2/(A F_r^2)),
//        the area element of r = r_k(theta, phi), eqs. (RaidalHypersurface)-(redshift),
//        written with the gradient of F: the printed sqrt|h_k|, which carries a factor
//        A^{1/2}, times the sqrt|g_tt| of the time element (Sec. 4.2).  With both
//        factors the total power of a spherical isotropic conversion surface in
//        Schwarzschild equals the backward image sum of eq. (BackPower), the
//        equality Sec. 2.4 reports;
//   Q  = |cos theta_n| v_a w P_ag, where the 1/|k.dE| of P_ag cancels the
//        projection cos theta_n exactly, eqs. (CosIso), (AngleDefAniso):
//        isotropic   Q = pi g^2 |B_perp|^2 E^2 / |d w_p^2|        (eq. ProbIsoCurved, read
//                    with E^2 so that P_ag is dimensionless; the 1-D limit agrees)
//        anisotropic Q = (pi/2) g^2 |B_perp|^2 E^5 / (D |dE|),     eq. (CPAnisoCurved)
//                    D = cos^2 w_p^2 (w_p^2 - 2E^2) + E^4, rewritten as
//                    (E^2 - cos^2 w_p^2)^2 + cos^2 sin^2 w_p^4;
//   n_c = n_inf |k_a| / k0 (gravitational focusing; the general-relativistic
//        on-shell |k_a| = sqrt(w_inf^2/A - m_a^2) instead of the Newtonian k_c).
// Gradients are spatial, at fixed covariant k, with norms |v|^2 = g^{ij} v_i v_j.
// ---------------------------------------------------------------------------
template <class P>
struct SeedOut;

// flat-propagation variant (App. B): the photon leaves with its local (static-frame)
// frequency and momentum, to be traced with M = 0
template <class P>
static void finish_flat(const Inst<P>& I, SeedOut<P>& o, const P ko[3], double om, const P& sA);

template <class P>
struct SeedOut {
    P y[8];
    P w;
    P rc;
    int status;
};

template <class P>
static SeedOut<P> seed_ray(const Inst<P>& I, uint64_t seed, int32_t instance, int64_t i) {
    SeedOut<P> o;
    double u[6];
    ray_uniforms(seed, instance, i, u);
    // emission direction, uniform in (cos theta, phi)
    double ct = 2.0 * u[0] - 1.0, st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    double ph = 2.0 * PI * u[1];
    double n[3] = {st * std::cos(ph), st * std::sin(ph), ct};
    // axion direction in the static orthonormal frame
    double kh[3];
    if (I.kdir == KD_ISO) {
        double c = 2.0 * u[2] - 1.0, s = std::sqrt(std::max(0.0, 1.0 - c * c)), a = 2.0 * PI * u[3];
        kh[0] = s * std::cos(a); kh[1] = s * std::sin(a); kh[2] = c;
    } else {
        double c = u[2], s = std::sqrt(std::max(0.0, 1.0 - c * c)), a = 2.0 * PI * u[3];
        double th_hat[3] = {ct * std::cos(ph), ct * std::sin(ph), -st};
        double ph_hat[3] = {-std::sin(ph), std::cos(ph), 0.0};
        for (int d = 0; d < 3; ++d)
            kh[d] = c * n[d] + s * (std::cos(a) * th_hat[d] + std::sin(a) * ph_hat[d]);
    }
    // emission time uniform over one period [km]
    P t0 = u[4] * I.Period * C_KMS;
    // the axion's momentum at infinity: k0 = m_a v0 for every axion (eq. (fa_approx)), or
    // drawn from the Maxwellian of eq. (GaussianDist) with the sixth uniform; its energy at
    // infinity in units of w_inf is om, with om^2 = (1 + x v0^2) / (1 + v0^2), x = (k/k0)^2
    double x2 = 1.0;
    if (I.speeds == SP_MAXWELL) x2 = maxwell_x(u[5]);
    const double ma2v = val(I.ma2);
    const double om2 = ma2v + x2 * I.kv2;
    const double om = std::sqrt(om2);
    // thin-surface variant (App. B): the resonance is taken on w_p = m_a alone
    const bool thin = (I.flags & ORC_FLAG_THIN_SURFACE) != 0;
    P rc = resonance_radius_t(I, n, t0, kh, om2, thin);
    o.rc = rc;
    if (val(rc) < 0.0) {
        for (int d = 0; d < 8; ++d) o.y[d] = P(0.0);
        o.w = P(0.0);
        o.status = ORC_NO_RESONANCE;
        return o;
    }
    o.status = ORC_OK;
    P A = 1.0 - I.rs / rc;
    P sA = sqrt(A);
    // |k_a| / w_inf in the static frame: |k_a|^2 = om^2/A - m~^2 = (x kv2 + m~^2 rs/r) / A,
    // the second form without the cancellation of the first (|k_a| << w_inf far from the star)
    P ka = sqrt((x2 * I.kv2 + I.ma2 * (I.rs / rc)) / A);
    P x[3] = {rc * n[0], rc * n[1], rc * n[2]};
    if (I.flags & ORC_FLAG_EXCISE_OPEN) {
        const double xv[3] = {val(x[0]), val(x[1]), val(x[2])};
        if (on_open_field_line(I, xv, val(t0))) {
            for (int d = 0; d < 8; ++d) o.y[d] = P(0.0);
            o.w = P(0.0);
            o.status = ORC_EXCISED;
            return o;
        }
    }
    // photon momentum = axion momentum (kinematic matching), orthonormal |k| khat -> Cartesian
    // covariant.  On the thin surface the photon keeps the axion's frequency and direction and
    // takes |k| from the LO dispersion relation there, |k|^2 = E^2 (E^2 - w_p^2)/(E^2 - w_p^2 cos^2).
    P kg = ka;
    if (thin && I.plasma == PL_ANISO) {
        P Bt[3];
        bfield_t(I, x, t0, Bt);
        P cBt = dot3(kh, Bt) / sqrt(dot3(Bt, Bt));
        P E2 = om2 / A;
        P wpt = wp2_tilde(I, x, t0);
        kg = sqrt(E2 * (E2 - wpt) / (E2 - wpt * cBt * cBt));
    }
    P ko[3] = {kg * kh[0], kg * kh[1], kg * kh[2]};
    P nko = dot3(n, ko);
    P k[3];
    for (int d = 0; d < 3; ++d) k[d] = (ko[d] - nko * n[d]) + (nko / sA) * n[d];
    for (int d = 0; d < 3; ++d) { o.y[d] = x[d]; o.y[4 + d] = k[d]; }
    o.y[3] = t0;
    o.y[7] = P(-om);

    if (I.weights == W_UNIT) { o.w = P(1.0); return o; }

    // ---- weight ----
    const double Ck = (I.kdir == KD_ISO) ? 4.0 * PI : 2.0 * PI;
    P n_c = I.n_inf * ka * I.w_inf / (I.k0 * std::sqrt(x2));  // n_inf |k_a| / |k_inf|
    // surface element from the gradient of F at fixed khat and t0
    using D3 = Dual<3, P>;
    D3 xd[3] = {D3::var(x[0], 0), D3::var(x[1], 1), D3::var(x[2], 2)};
    D3 Fd = resonance_F(I, xd, t0, kh, om2, thin);
    P gF[3] = {Fd.d[0], Fd.d[1], Fd.d[2]};
    P Fr = dot3(n, gF);
    P gp2 = P(0.0);
    for (int d = 0; d < 3; ++d) { P gp = gF[d] - Fr * n[d]; gp2 = gp2 + gp * gp; }
    P Vt = A * rc * rc * sqrt(1.0 + gp2 / (A * Fr * Fr));     // km^2
    Vt = Vt / (HBARC_EVKM * HBARC_EVKM);                      // eV^-2
    // cos theta_n of eq. (AngleDef): the axion direction against the unit normal of the
    // surface in the static orthonormal frame (radial covector component times sqrt(A))
    P gFo[3];
    for (int d = 0; d < 3; ++d) gFo[d] = (gF[d] - Fr * n[d]) + sA * Fr * n[d];
    P cos_n = dot3(kh, gFo) / sqrt(dot3(gFo, gFo));
    if (I.flags & ORC_FLAG_RENORM_WEIGHTS) {
        // Sec. 6 eq. (reweight): P_ag = 1 and each ray rescaled by
        // R = (1 cm^-3 / n_a(r)) (m_a / |k_a|) / sqrt(1 - r_s/r), which leaves
        // w = C_k Vt |cos theta_n| m_a (1 cm^-3) / sqrt(A)
        const double n1 = HBARC_EVCM * HBARC_EVCM * HBARC_EVCM;  // 1 cm^-3 [eV^3]
        P m_a = I.w_inf * sqrt(I.ma2);
        o.w = Ck * Vt * fabs(cos_n) * m_a * n1 / sA;
        finish_flat(I, o, ko, om, sA);
        return o;
    }
    P E = om * I.w_inf / sA;                                  // local photon energy [eV]
    P Bv[3];
    bfield_t(I, x, t0, Bv);
    P B2 = dot3(Bv, Bv);
    P cB = dot3(ko, Bv) / sqrt(B2 * dot3(ko, ko));
    P Bperp2;
    const double G2 = gauss_in_eV2();
    if (I.weights == W_CONV_CONSTB) Bperp2 = P(I.Btest * G2 * I.Btest * G2);
    else Bperp2 = B2 * G2 * G2 * (1.0 - cB * cB);
    P gtt, gij[3][3];
    inverse_metric(I, x, gtt, gij);
    P Q;
    if (I.plasma == PL_ISO) {
        D3 wd = wp2_tilde(I, xd, D3(0.0) + t0);
        P gw2 = P(0.0);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) gw2 = gw2 + gij[a][b] * wd.d[a] * wd.d[b];
        P dwp2 = HBARC_EVKM * I.w_inf * I.w_inf * sqrt(gw2);  // |d w_p^2| [eV^3]
        Q = PI * I.g_eV * I.g_eV * Bperp2 * E * E / dwp2;
    } else {
        D3 Ed = energy_t(I, xd, t0, k);
        P gE2 = P(0.0);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) gE2 = gE2 + gij[a][b] * Ed.d[a] * Ed.d[b];
        P dE = HBARC_EVKM * I.w_inf * sqrt(gE2);              // |dE| [eV^2]
        P wp2 = wp2_tilde(I, x, t0) * I.w_inf * I.w_inf;      // [eV^2]
        P c2 = cB * cB, s2 = 1.0 - c2;
        P Dd = (E * E - c2 * wp2) * (E * E - c2 * wp2) + c2 * s2 * wp2 * wp2;
        if (thin) {
            // the surface is no level set of the photon energy, so cos theta_n and the
            // 1/|k.dE| of P_ag do not cancel: Q = |cos theta_n| v_a E P_ag with the photon's
            // k.dE = k^a d_a E (contravariant k)
            P kc[3];
            for (int a = 0; a < 3; ++a) kc[a] = gij[a][0] * k[0] + gij[a][1] * k[1] + gij[a][2] * k[2];
            P kdE = HBARC_EVKM * I.w_inf * I.w_inf * (kc[0] * Ed.d[0] + kc[1] * Ed.d[1] + kc[2] * Ed.d[2]);
            P Pag = 0.5 * PI * I.g_eV * I.g_eV * Bperp2 * E * E * E * E * E / (Dd * fabs(kdE));
            Q = fabs(cos_n) * (ka * I.w_inf) * Pag;  // |cos theta_n| v_a E P with v_a E = |k_a|
        } else {
            Q = 0.5 * PI * I.g_eV * I.g_eV * Bperp2 * E * E * E * E * E / (Dd * dE);
        }
    }
    o.w = Ck * n_c * Vt * Q;
    finish_flat(I, o, ko, om, sA);
    return o;
}

template <class P>
static void finish_flat(const Inst<P>& I, SeedOut<P>& o, const P ko[3], double om, const P& sA) {
    if (!(I.flags & ORC_FLAG_FLAT_PROPAGATION)) return;
    for (int d = 0; d < 3; ++d) o.y[4 + d] = ko[d];
    o.y[7] = -om / sA;
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) with FSAL and the 4th-order continuous extension.
// ---------------------------------------------------------------------------
namespace dp {
static const double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
static const double a21 = 1.0 / 5;
static const double a31 = 3.0 / 40, a32 = 9.0 / 40;
static const double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
static const double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
static const double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                    a65 = -5103.0 / 18656;
static const double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784, b6 = 11.0 / 84;
// 5th minus 4th order weights
static const double e1 = 71.0 / 57600, e3 = -71.0 / 16695, e4 = 71.0 / 1920, e5 = -17253.0 / 339200,
                    e6 = 22.0 / 525, e7 = -1.0 / 40;
// continuous extension
static const double d1 = -12715105075.0 / 11282082432.0, d3 = 87487479700.0 / 32700410799.0,
                    d4 = -10690763975.0 / 1880347072.0, d5 = 701980252875.0 / 199316789632.0,
                    d6 = -1453857185.0 / 822651844.0, d7 = 69997945.0 / 29380423.0;
}  // namespace dp

template <class S>
struct Step {
    S K[7][8];
    S ynew[8];
    S yerr[8];
};

template <class S, class F>
static void dopri_step(F& f, const S y[8], const S k1[8], double h, Step<S>& st) {
    using namespace dp;
    S tmp[8];
    for (int i = 0; i < 8; ++i) st.K[0][i] = k1[i];
    for (int i = 0; i < 8; ++i) tmp[i] = y[i] + h * (a21 * st.K[0][i]);
    f(tmp, st.K[1]);
    for (int i = 0; i < 8; ++i) tmp[i] = y[i] + h * (a31 * st.K[0][i] + a32 * st.K[1][i]);
    f(tmp, st.K[2]);
    for (int i = 0; i < 8; ++i) tmp[i] = y[i] + h * (a41 * st.K[0][i] + a42 * st.K[1][i] + a43 * st.K[2][i]);
    f(tmp, st.K[3]);
    for (int i = 0; i < 8; ++i)
        tmp[i] = y[i] + h * (a51 * st.K[0][i] + a52 * st.K[1][i] + a53 * st.K[2][i] + a54 * st.K[3][i]);
    f(tmp, st.K[4]);
    for (int i = 0; i < 8; ++i)
        tmp[i] = y[i] + h * (a61 * st.K[0][i] + a62 * st.K[1][i] + a63 * st.K[2][i] + a64 * st.K[3][i] +
                             a65 * st.K[4][i]);
    f(tmp, st.K[5]);
    for (int i = 0; i < 8; ++i)
        st.ynew[i] = y[i] + h * (b1 * st.K[0][i] + b3 * st.K[2][i] + b4 * st.K[3][i] + b5 * st.K[4][i] +
                                 b6 * st.K[5][i]);
    f(st.ynew, st.K[6]);
    for (int i = 0; i < 8; ++i)
        st.yerr[i] = h * (e1 * st.K[0][i] + e3 * st.K[2][i] + e4 * st.K[3][i] + e5 * st.K[4][i] +
                          e6 * st.K[5][i] + e7 * st.K[6][i]);
}

// RMS error norm with scale atol + rtol max(|y|, |y_new|) over all 8 components.
template <class S>
static double err_norm(const S y[8], const Step<S>& st, double rtol, double atol) {
    double acc = 0.0;
    for (int i = 0; i < 8; ++i) {
        double sc = atol + rtol * std::max(std::fabs(val(y[i])), std::fabs(val(st.ynew[i])));
        double q = val(st.yerr[i]) / sc;
        acc += q * q;
    }
    return std::sqrt(acc / 8.0);
}

// Continuous extension of the accepted step at theta in [0, 1].
template <class S, class TH>
static void dense_eval(const S y[8], const Step<S>& st, double h, const TH& th, S out[8]) {
    using namespace dp;
    for (int i = 0; i < 8; ++i) {
        S ydiff = st.ynew[i] - y[i];
        S r3 = h * st.K[0][i] - ydiff;
        S r4 = ydiff - h * st.K[6][i] - r3;
        S r5 = h * (d1 * st.K[0][i] + d3 * st.K[2][i] + d4 * st.K[3][i] + d5 * st.K[4][i] + d6 * st.K[5][i] +
                    d7 * st.K[6][i]);
        TH om = 1.0 - th;
        out[i] = y[i] + th * (ydiff + om * (r3 + th * (r4 + om * r5)));
    }
}

// d/dtheta of the continuous extension
template <class S>
static void dense_deriv(const S y[8], const Step<S>& st, double h, double th, S out[8]) {
    using namespace dp;
    for (int i = 0; i < 8; ++i) {
        S ydiff = st.ynew[i] - y[i];
        S r3 = h * st.K[0][i] - ydiff;
        S r4 = ydiff - h * st.K[6][i] - r3;
        S r5 = h * (d1 * st.K[0][i] + d3 * st.K[2][i] + d4 * st.K[3][i] + d5 * st.K[4][i] + d6 * st.K[5][i] +
                    d7 * st.K[6][i]);
        double om = 1.0 - th;
        S Q = r3 + th * (r4 + om * r5);
        S Pp = ydiff + om * Q;
        S dP = -1.0 * Q + om * (r4 + (1.0 - 2.0 * th) * r5);
        out[i] = Pp + th * dP;
    }
}

// Starting step, Hairer-Norsett-Wanner Sec. II.4 (order 5).
template <class S, class F>
static double initial_step(F& f, const S y0[8], const S f0[8], double rtol, double atol) {
    double d0 = 0, d1 = 0;
    for (int i = 0; i < 8; ++i) {
        double sc = atol + rtol * std::fabs(val(y0[i]));
        d0 += (val(y0[i]) / sc) * (val(y0[i]) / sc);
        d1 += (val(f0[i]) / sc) * (val(f0[i]) / sc);
    }
    d0 = std::sqrt(d0 / 8.0); d1 = std::sqrt(d1 / 8.0);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    S y1[8], f1[8];
    for (int i = 0; i < 8; ++i) y1[i] = y0[i] + h0 * f0[i];
    f(y1, f1);
    double d2 = 0;
    for (int i = 0; i < 8; ++i) {
        double sc = atol + rtol * std::fabs(val(y0[i]));
        double q = (val(f1[i]) - val(f0[i])) / sc;
        d2 += q * q;
    }
    d2 = std::sqrt(d2 / 8.0) / h0;
    double m = std::max(d1, d2);
    double h1 = (m <= 1e-15) ? std::max(1e-6, h0 * 1e-3) : std::pow(0.01 / m, 1.0 / 5.0);
    return std::min(100.0 * h0, h1);
}

static bool all_finite8(const double* y) {
    for (int i = 0; i < 8; ++i) if (!std::isfinite(y[i])) return false;
    return true;
}

// ---------------------------------------------------------------------------
// Observables at the r = r_max crossing (Sec. 2.2: the asymptotic direction
// of each ray is binned on the sky).  The direction is that of the static-frame
// momentum; psi is the azimuth in the frame co-rotating with the star at the
// arrival time t - r; w_f = -k_t is the energy at infinity in units of w_inf.
// ---------------------------------------------------------------------------
template <class S, class P>
static void observables(const Inst<P>& I, const S y[8], S& theta, S& phi, S& psi, S v[3]) {
    S x[3] = {y[0], y[1], y[2]};
    S k[3] = {y[4], y[5], y[6]};
    S ko[3];
    ortho_components(I, x, k, ko);
    S kn = sqrt(dot3(ko, ko));
    for (int d = 0; d < 3; ++d) v[d] = ko[d] / kn;
    theta = atan2(sqrt(v[0] * v[0] + v[1] * v[1]), v[2]);
    phi = atan2(v[1], v[0]);
    S r = sqrt(dot3(x, x));
    S p = phi - I.Om * (y[3] - r);
    // reduce to [0, 2 pi) on the value; the derivative is unaffected
    double pv = val(p);
    double red = std::fmod(pv, 2.0 * PI);
    if (red < 0) red += 2.0 * PI;
    if (red >= 2.0 * PI) red -= 2.0 * PI;
    psi = p + (red - pv);
}

// Result of tracing one ray.
template <class S>
struct TraceOut {
    S yf[8];
    double lam;
    double h;
    int64_t nacc, nrej;
    int status;
};

// One forward ray from y0 to r = r_max (or another terminal condition).
// hfix != nullptr replays a recorded sequence of accepted steps (frozen steps).
// kinks: for the GJ density, integrate one smooth piece s g of |g| at a time.  The
// density has a kink on the null surface g = 0, where the right-hand side jumps; an
// accepted step whose end lies on the other side is cut at the crossing, located by 60
// bisections on its continuous extension (the first point past it), and the ray restarts
// there on the other piece with a fresh derivative (the treatment of a discontinuity
// in Hairer, Norsett & Wanner I, Sec. II.6).  Without it the step size collapses at every
// crossing and the error control loses accuracy there.
template <class S, class P>
static TraceOut<S> trace_one(const Inst<P>& I, const orc_tol& tol, const S y0[8], double sign,
                             std::vector<double>* hrec, const double* hfix, int64_t nfix, bool kinks = false) {
    TraceOut<S> o;
    Inst<P> J = I;  // J.gj_branch: the piece being integrated
    const bool kinky = kinks && I.density == DEN_GJ;
    if (kinky) {
        const double x0[3] = {val(y0[0]), val(y0[1]), val(y0[2])};
        J.gj_branch = (gj_factor(I, x0, val(y0[3])) < 0.0) ? -1.0 : 1.0;
    }
    auto f = [&](const S* yy, S* ff) { rhs_t(J, yy, ff, sign); };
    S y[8], k1[8];
    for (int i = 0; i < 8; ++i) y[i] = y0[i];
    f(y, k1);
    double h = (hfix != nullptr) ? (nfix > 0 ? hfix[0] : 0.0) : initial_step(f, y, k1, tol.rtol, tol.atol);
    double lam = 0.0;
    double facmax = 10.0;
    int64_t nacc = 0, nrej = 0;
    const double R = val(I.R);
    Step<S> st;
    o.status = ORC_OK;
    while (true) {
        if (hfix != nullptr) {
            if (nacc >= nfix) { o.status = ORC_MAX_STEPS; break; }
            h = hfix[nacc];
        }
        dopri_step(f, y, k1, h, st);
        double err = err_norm(y, st, tol.rtol, tol.atol);
        if (!std::isfinite(err)) err = 1e300;
        if (hfix == nullptr && err > 1.0) {
            ++nrej;
            h *= std::max(0.2, 0.9 * std::pow(err, -0.2));
            facmax = 1.0;
            if (!(std::fabs(h) >= 1e-14 * (1.0 + std::fabs(lam)))) { o.status = ORC_STEP_UNDERFLOW; break; }
            continue;
        }
        // accepted
        ++nacc;
        if (hrec) hrec->push_back(h);
        double yv[8];
        for (int i = 0; i < 8; ++i) yv[i] = val(st.ynew[i]);
        double rnew = std::sqrt(yv[0] * yv[0] + yv[1] * yv[1] + yv[2] * yv[2]);
        if (!all_finite8(yv)) {
            for (int i = 0; i < 8; ++i) o.yf[i] = st.ynew[i];
            o.status = ORC_NONFINITE; lam += h; break;
        }
        if (rnew <= R) {
            for (int i = 0; i < 8; ++i) o.yf[i] = st.ynew[i];
            o.status = ORC_HIT_STAR; lam += h; break;
        }
        // crossing of the null surface inside the step (none: thk > 1)
        double thk = 2.0;
        if (kinky && J.gj_branch * gj_factor(I, yv, yv[3]) < 0.0) {
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 60; ++it) {
                double mid = 0.5 * (lo + hi);
                S ym[8];
                dense_eval(y, st, h, mid, ym);
                const double xm[3] = {val(ym[0]), val(ym[1]), val(ym[2])};
                if (J.gj_branch * gj_factor(I, xm, val(ym[3])) > 0.0) lo = mid; else hi = mid;
            }
            thk = hi;
        }
        double th = 2.0;
        if (rnew >= tol.r_max_km) {
            // locate r(theta) = r_max on the continuous extension: 60 bisections
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 60; ++it) {
                double mid = 0.5 * (lo + hi);
                S ym[8];
                dense_eval(y, st, h, mid, ym);
                double rm = std::sqrt(val(ym[0]) * val(ym[0]) + val(ym[1]) * val(ym[1]) + val(ym[2]) * val(ym[2]));
                if (rm >= tol.r_max_km) hi = mid; else lo = mid;
            }
            th = hi;
        }
        if (th <= 1.0 && th <= thk) {
            if constexpr (is_dual<S>::value) {
                // implicit derivative of the crossing: r(y(theta)) = r_max
                S yth[8], dy[8];
                dense_eval(y, st, h, th, yth);
                dense_deriv(y, st, h, th, dy);
                S r = sqrt(yth[0] * yth[0] + yth[1] * yth[1] + yth[2] * yth[2]);
                S drdth = (yth[0] * dy[0] + yth[1] * dy[1] + yth[2] * dy[2]) / r;
                S thd = (S(0.0) + th) - (r - tol.r_max_km) / drdth;
                thd.v = th;
                dense_eval(y, st, h, thd, o.yf);
            } else {
                dense_eval(y, st, h, th, o.yf);
            }
            o.status = ORC_ESCAPED;
            lam += th * h;
            break;
        }
        if (thk <= 1.0) {
            // restart at the first point past the null surface, on the other piece; for dual
            // parameters the location carries the implicit derivative of g(y(theta)) = 0
            S yk[8];
            if constexpr (is_dual<S>::value) {
                S yth[8], dy[8], dg;
                dense_eval(y, st, h, thk, yth);
                dense_deriv(y, st, h, thk, dy);
                const S g = gj_factor_t(I, yth, yth[3], dy, dy[3], &dg);
                S thd = (S(0.0) + thk) - g / dg;
                thd.v = thk;
                dense_eval(y, st, h, thd, yk);
            } else {
                dense_eval(y, st, h, thk, yk);
            }
            for (int i = 0; i < 8; ++i) y[i] = yk[i];
            lam += thk * h;
            J.gj_branch = -J.gj_branch;
            f(y, k1);
        } else {
            lam += h;
            for (int i = 0; i < 8; ++i) { y[i] = st.ynew[i]; k1[i] = st.K[6][i]; }
        }
        if (hfix == nullptr) {
            double fac = (err == 0.0) ? facmax : std::min(facmax, std::max(0.2, 0.9 * std::pow(err, -0.2)));
            h *= fac;
            facmax = 10.0;
            if (nacc >= tol.max_steps) {
                for (int i = 0; i < 8; ++i) o.yf[i] = y[i];
                o.status = ORC_MAX_STEPS;
                break;
            }
            if (!(std::fabs(h) >= 1e-14 * (1.0 + std::fabs(lam)))) {
                for (int i = 0; i < 8; ++i) o.yf[i] = y[i];
                o.status = ORC_STEP_UNDERFLOW;
                break;
            }
        }
    }
    o.lam = lam; o.h = h; o.nacc = nacc; o.nrej = nrej;
    return o;
}

static void store_final(const Inst<double>& I, const TraceOut<double>& o, int64_t i, int64_t n, double* fin,
                        int32_t* ifin) {
    for (int d = 0; d < 8; ++d) fin[d * n + i] = o.yf[d];
    double th, ph, ps, v[3];
    observables(I, o.yf, th, ph, ps, v);
    fin[8 * n + i] = th;
    fin[9 * n + i] = ph;
    fin[10 * n + i] = ps;
    fin[11 * n + i] = -o.yf[7];
    fin[12 * n + i] = hamiltonian_t(I, o.yf);
    fin[13 * n + i] = o.lam;
    fin[14 * n + i] = std::sqrt(o.yf[0] * o.yf[0] + o.yf[1] * o.yf[1] + o.yf[2] * o.yf[2]);
    fin[15 * n + i] = o.h;
    ifin[0 * n + i] = (int32_t)std::min<int64_t>(o.nacc, INT32_MAX);
    ifin[1 * n + i] = (int32_t)std::min<int64_t>(o.nrej, INT32_MAX);
    ifin[2 * n + i] = o.status;
}

// ---------------------------------------------------------------------------
// Backward tracing from an image plane (Sec. 2.1) with production events at
// every sign change of G = g^{mu nu} k_mu k_nu + m_a^2 (the photon momentum on
// the axion mass shell, k^gamma = k^a; Sec. 2.4 and Sec. 3: every level
// crossing along the ray contributes).
// ---------------------------------------------------------------------------
static double event_G(const Inst<double>& I, const double y[8]) {
    double x[3] = {y[0], y[1], y[2]};
    double k[3] = {y[4], y[5], y[6]};
    double gtt, gij[3][3];
    inverse_metric(I, x, gtt, gij);
    double kk = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) kk += gij[i][j] * k[i] * k[j];
    return gtt * y[7] * y[7] + kk + I.ma2;
}

// One backward ray through the point (b1, b2) of the plane at distance D perpendicular
// to the line of sight (inclination incl, azimuth phio).
static void backward_ray(const Inst<double>& I, const orc_tol& tol, double D, double incl, double phio, double b1,
                         double b2, int32_t K, int64_t slot, int64_t n, double* ev, int32_t* nev, double* fin,
                         int32_t* ifin) {
    double no[3] = {std::sin(incl) * std::cos(phio), std::sin(incl) * std::sin(phio), std::cos(incl)};
    double e1[3] = {std::cos(incl) * std::cos(phio), std::cos(incl) * std::sin(phio), -std::sin(incl)};
    double e2[3] = {-std::sin(phio), std::cos(phio), 0.0};
    double y[8];
    for (int d = 0; d < 3; ++d) y[d] = D * no[d] + b1 * e1[d] + b2 * e2[d];
    y[3] = 0.0;
    // parallel rays along the line of sight; |k| from H = 0 on the LO branch,
    // eq. (AnisotropicDisp) solved for |k|^2 at w^2 = 1/A (units of w_inf)
    double r0 = std::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double A0 = 1.0 - I.rs / r0;
    double w2 = 1.0 / A0;
    double wp2 = wp2_tilde(I, y, y[3]);
    double kap2;
    if (I.plasma == PL_ISO) {
        kap2 = w2 - wp2;
    } else {
        double B[3];
        bfield_t(I, y, y[3], B);
        double cB = dot3(no, B) / std::sqrt(dot3(B, B));
        kap2 = w2 * (w2 - wp2) / (w2 - wp2 * cB * cB);
    }
    double kap = std::sqrt(kap2);
    double ko[3] = {kap * no[0], kap * no[1], kap * no[2]};
    double n0[3] = {y[0] / r0, y[1] / r0, y[2] / r0};
    double nko = dot3(n0, ko);
    for (int d = 0; d < 3; ++d) y[4 + d] = (ko[d] - nko * n0[d]) + (nko / std::sqrt(A0)) * n0[d];
    y[7] = -1.0;

    // the GJ density one smooth piece at a time, as in forward tracing (J.gj_branch: the
    // piece being integrated; a step that crosses the null surface is cut there)
    Inst<double> J = I;
    const bool kinky = I.density == DEN_GJ;
    if (kinky) J.gj_branch = (gj_factor(I, y, y[3]) < 0.0) ? -1.0 : 1.0;
    auto f = [&](const double* yy, double* ff) { rhs_t(J, yy, ff, -1.0); };
    // Backward rays start in near-vacuum far from the star, where the error
    // estimate vanishes and the step would grow without bound and could jump
    // across the whole plasma region.  A step therefore never moves the ray by
    // more than a tenth of its current radius.
    auto cap = [&](const double* yy, const double* ff, double hh) {
        double r = std::sqrt(yy[0] * yy[0] + yy[1] * yy[1] + yy[2] * yy[2]);
        double sp = std::sqrt(ff[0] * ff[0] + ff[1] * ff[1] + ff[2] * ff[2]);
        double hmax = 0.1 * r / sp;
        return std::min(hh, hmax);
    };
    double k1[8];
    f(y, k1);
    double h = cap(y, k1, initial_step(f, y, k1, tol.rtol, tol.atol));
    double lam = 0.0, facmax = 10.0;
    int64_t nacc = 0, nrej = 0;
    int32_t ne = 0;
    Step<double> st;
    int status = ORC_OK;
    double Gprev = event_G(I, y);
    double rprev = r0;
    const double R = I.R;
    double yend[8];
    for (int d = 0; d < 8; ++d) yend[d] = y[d];
    while (true) {
        dopri_step(f, y, k1, h, st);
        double err = err_norm(y, st, tol.rtol, tol.atol);
        if (!std::isfinite(err)) err = 1e300;
        if (err > 1.0) {
            ++nrej;
            h *= std::max(0.2, 0.9 * std::pow(err, -0.2));
            facmax = 1.0;
            if (!(std::fabs(h) >= 1e-14 * (1.0 + std::fabs(lam)))) { status = ORC_STEP_UNDERFLOW; break; }
            continue;
        }
        ++nacc;
        // crossing of the null surface inside the step (none: thk > 1): 60 bisections, the
        // first point past the surface
        double thk = 2.0;
        if (kinky && J.gj_branch * gj_factor(I, st.ynew, st.ynew[3]) < 0.0) {
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 60; ++it) {
                double mid = 0.5 * (lo + hi);
                double ym[8];
                dense_eval(y, st, h, mid, ym);
                if (J.gj_branch * gj_factor(I, ym, ym[3]) > 0.0) lo = mid; else hi = mid;
            }
            thk = hi;
        }
        const double tend = (thk <= 1.0) ? thk : 1.0;
        // events: G sampled at theta = 1/4, 1/2, 3/4, 1 of the part of the step taken
        double thp = 0.0, Gp = Gprev;
        for (int q = 1; q <= 4; ++q) {
            double thq = 0.25 * q * tend;
            double yq[8];
            if (q == 4 && thk > 1.0) { for (int d = 0; d < 8; ++d) yq[d] = st.ynew[d]; }
            else dense_eval(y, st, h, thq, yq);
            double Gq = event_G(I, yq);
            if ((Gp > 0.0 && Gq <= 0.0) || (Gp < 0.0 && Gq >= 0.0)) {
                double lo = thp, hi = thq;
                for (int it = 0; it < 60; ++it) {
                    double mid = 0.5 * (lo + hi);
                    double ym[8];
                    dense_eval(y, st, h, mid, ym);
                    double Gm = event_G(I, ym);
                    if ((Gp > 0.0) == (Gm > 0.0)) lo = mid; else hi = mid;
                }
                double the = 0.5 * (lo + hi);
                double ye[8];
                dense_eval(y, st, h, the, ye);
                if (ne < K) {
                    for (int d = 0; d < 8; ++d) ev[((int64_t)ne * ORC_NEV + d) * n + slot] = ye[d];
                    double re = std::sqrt(ye[0] * ye[0] + ye[1] * ye[1] + ye[2] * ye[2]);
                    ev[((int64_t)ne * ORC_NEV + 8) * n + slot] = -ye[7] - 1.0;
                    ev[((int64_t)ne * ORC_NEV + 9) * n + slot] = -ye[7] / std::sqrt(1.0 - I.rs / re);
                }
                ++ne;
            }
            thp = thq; Gp = Gq;
        }
        Gprev = Gp;
        if (thk <= 1.0) {
            // restart at the crossing on the other piece, with a fresh derivative
            double yk[8];
            dense_eval(y, st, h, thk, yk);
            for (int d = 0; d < 8; ++d) y[d] = yk[d];
            lam += thk * h;
            J.gj_branch = -J.gj_branch;
            f(y, k1);
        } else {
            lam += h;
            for (int d = 0; d < 8; ++d) { y[d] = st.ynew[d]; k1[d] = st.K[6][d]; }
        }
        double rnew = std::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
        if (!all_finite8(y)) { status = ORC_NONFINITE; break; }
        if (rnew <= R) { status = ORC_HIT_STAR; break; }
        if (rnew > 1.01 * D && rnew > rprev) { status = ORC_ESCAPED; break; }
        rprev = rnew;
        double fac = (err == 0.0) ? facmax : std::min(facmax, std::max(0.2, 0.9 * std::pow(err, -0.2)));
        h = cap(y, k1, h * fac);
        facmax = 10.0;
        if (nacc >= tol.max_steps) { status = ORC_MAX_STEPS; break; }
        if (!(std::fabs(h) >= 1e-14 * (1.0 + std::fabs(lam)))) { status = ORC_STEP_UNDERFLOW; break; }
    }
    for (int d = 0; d < 8; ++d) yend[d] = y[d];
    nev[slot] = ne;
    for (int d = 0; d < 8; ++d) fin[d * n + slot] = yend[d];
    for (int d = 8; d < ORC_NFIN; ++d) fin[d * n + slot] = 0.0;
    fin[12 * n + slot] = hamiltonian_t(I, yend);
    fin[13 * n + slot] = lam;
    fin[14 * n + slot] = std::sqrt(yend[0] * yend[0] + yend[1] * yend[1] + yend[2] * yend[2]);
    fin[15 * n + slot] = h;
    ifin[0 * n + slot] = (int32_t)nacc;
    ifin[1 * n + slot] = (int32_t)nrej;
    ifin[2 * n + slot] = status;
}

// pixel (pi, pj) of an nx x ny plane of half-width W: rays through the pixel centres
static void backward_pixel(const Inst<double>& I, const orc_tol& tol, double D, double incl, double phio, double W,
                           int32_t nx, int32_t ny, int32_t pi, int32_t pj, int32_t K, int64_t slot, int64_t n,
                           double* ev, int32_t* nev, double* fin, int32_t* ifin) {
    double db = 2.0 * W / nx;
    double b1 = (pi + 0.5 - 0.5 * nx) * db, b2 = (pj + 0.5 - 0.5 * ny) * db;
    backward_ray(I, tol, D, incl, phio, b1, b2, K, slot, n, ev, nev, fin, ifin);
}

// ---------------------------------------------------------------------------
// Backward power (Sec. 2.1 eq. (BackPower)): the image sums Delta b^2 w^3 f_gamma over
// pixels, and a ray's f_gamma is the sum over its production events of P_ag f_a
// (Sec. 3), with the focused monochromatic axions of Sec. 4.3,
//   f_a = v_a n_c delta(w - w_c) / (4 pi k^2)     (local static-frame quantities),
// and the conversion probabilities of Sec. 4.4,
//   isotropic   P = pi g^2 |B_perp|^2 E^2 / |k.d(w_p^2)|           eq. (ProbIsoCurved)
//   anisotropic P = (pi/2) g^2 |B_perp|^2 E^5 / (D |k.dE|)          eq. (CPAnisoCurved)
// (k.d = k^mu d_mu, spatial for the stationary plasma; read with E^2 resp. E^5 so that
// P is dimensionless: the same readings as the forward weights, whose Q is the
// cancelled product |cos theta_n| v_a E P).  Integrating the image sum over frequency,
// delta(w_inf / sqrt(A) - w_c) = sqrt(A) delta(w_inf - sqrt(A) w_c), so an event at a
// static star contributes
//   dP/dOmega += Delta b^2 w_inf^3 sqrt(A) P v_a n_c / (4 pi k^2).
// The paper's IR cutoff on the conversion length (Sec. 4.4) is read as
// L_c = sqrt(2 pi v_p / |khat.dE|) (a length); events with L_c > Lc_max are excluded
// when Lc_max > 0.  Returns the event's weight per unit image area [eV^4].
// ---------------------------------------------------------------------------
static double event_weight(const Inst<double>& I, const double y[8], double Lc_max_km, double* Lc_out) {
    const double x[3] = {y[0], y[1], y[2]};
    const double t = y[3];
    if ((I.flags & ORC_FLAG_EXCISE_OPEN) && on_open_field_line(I, x, t)) {
        if (Lc_out) *Lc_out = 0.0;
        return 0.0;
    }
    const double k[3] = {y[4], y[5], y[6]};
    const double r = std::sqrt(dot3(x, x));
    const double A = 1.0 - I.rs / r, sA = std::sqrt(A);
    const double E = -y[7] * I.w_inf / sA;  // local photon energy [eV]
    double ko[3];
    ortho_components(I, x, k, ko);
    const double kmag = std::sqrt(dot3(ko, ko)) * I.w_inf;  // [eV]
    const double va = kmag / E;
    const double n_c = I.n_inf * kmag / I.k0;  // on shell: |k_a| = |k_gamma| at the event
    double Bv[3];
    bfield_t(I, x, t, Bv);
    const double B2 = dot3(Bv, Bv);
    const double cB = dot3(ko, Bv) / std::sqrt(B2 * dot3(ko, ko));
    const double G2 = gauss_in_eV2();
    const double Bperp2 = (I.weights == W_CONV_CONSTB) ? (I.Btest * G2) * (I.Btest * G2)
                                                      : B2 * G2 * G2 * (1.0 - cB * cB);
    double gtt, gij[3][3];
    inverse_metric(I, x, gtt, gij);
    double kc[3];  // contravariant spatial components [units of w_inf]
    for (int a = 0; a < 3; ++a) kc[a] = gij[a][0] * k[0] + gij[a][1] * k[1] + gij[a][2] * k[2];
    using D3 = Dual<3, double>;
    D3 xd[3] = {D3::var(x[0], 0), D3::var(x[1], 1), D3::var(x[2], 2)};
    double P, kdE;  // kdE = k^a d_a E [eV^2 / km]
    if (I.plasma == PL_ISO) {
        D3 wd = wp2_tilde(I, xd, D3(0.0) + t);
        double kdw = 0.0;
        for (int a = 0; a < 3; ++a) kdw += kc[a] * wd.d[a];
        const double kdwp2 = HBARC_EVKM * I.w_inf * I.w_inf * I.w_inf * kdw;  // k.d(w_p^2) [eV^4]
        P = PI * I.g_eV * I.g_eV * Bperp2 * E * E / std::fabs(kdwp2);
        kdE = I.w_inf * I.w_inf * I.w_inf * kdw / (2.0 * E);  // d E = d(w_p^2) / (2 E)
    } else {
        D3 Ed = energy_t(I, xd, t, k);
        double kd = 0.0;
        for (int a = 0; a < 3; ++a) kd += kc[a] * Ed.d[a];
        const double kdEe = HBARC_EVKM * I.w_inf * I.w_inf * kd;  // k.dE [eV^3]
        const double wp2 = wp2_tilde(I, x, t) * I.w_inf * I.w_inf;
        const double c2 = cB * cB, s2 = 1.0 - c2;
        const double Dd = (E * E - c2 * wp2) * (E * E - c2 * wp2) + c2 * s2 * wp2 * wp2;
        P = 0.5 * PI * I.g_eV * I.g_eV * Bperp2 * E * E * E * E * E / (Dd * std::fabs(kdEe));
        kdE = I.w_inf * I.w_inf * kd;
    }
    const double khdE = std::fabs(kdE) / kmag;  // |khat.dE| [eV/km]
    const double Lc = std::sqrt(2.0 * PI * va * HBARC_EVKM / khdE);
    if (Lc_out) *Lc_out = Lc;
    if (Lc_max_km > 0.0 && Lc > Lc_max_km) return 0.0;
    const double w3 = I.w_inf * I.w_inf * I.w_inf;
    return w3 * sA * P * va * n_c / (4.0 * PI * kmag * kmag);
}

// ---------------------------------------------------------------------------
// Smoothed flux F_j = (1/N) sum_{escaped} w_i K(n_i . o_j), K(c) = exp((c-1)/s^2)/(2 pi s^2)
// ---------------------------------------------------------------------------
template <class S>
static S kernel_K(const S& c, double sigma) {
    return exp((c - 1.0) / (sigma * sigma)) / (2.0 * PI * sigma * sigma);
}

}  // namespace orc

using namespace orc;

static int nthreads_or_default(int nt) {
#ifdef _OPENMP
    return nt > 0 ? nt : omp_get_max_threads();
#else
    (void)nt;
    return 1;
#endif
}

extern "C" {

int orc_constants(double* out, int n) {
    double v[] = {C_KMS, HBARC_EVKM, ALPHA, M_E_EV, E_STATC, GM_SUN_KM, gauss_in_eV2(), wp2_per_ne(),
                  hbar_omega_c_per_gauss()};
    int m = (int)(sizeof(v) / sizeof(v[0]));
    for (int i = 0; i < n && i < m; ++i) out[i] = v[i];
    return m;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox(ctr, key, out); }

void orc_uniforms(uint64_t seed, int32_t instance, int64_t i, double u[6]) { ray_uniforms(seed, instance, i, u); }

double orc_wp2(const orc_star* s, const double x[3], double t) {
    Inst<double> I = make_inst_d(*s);
    return wp2_tilde(I, x, t);
}

void orc_bfield(const orc_star* s, const double x[3], double t, double B[3]) {
    Inst<double> I = make_inst_d(*s);
    bfield_t(I, x, t, B);
}

double orc_hamiltonian(const orc_star* s, const double y[8]) {
    Inst<double> I = make_inst_d(*s);
    return hamiltonian_t(I, y);
}

void orc_grad_h(const orc_star* s, const double y[8], double g[8]) {
    Inst<double> I = make_inst_d(*s);
    grad_h_t(I, y, g);
}

void orc_inverse_metric(const orc_star* s, const double x[3], double gi[9]) {
    Inst<double> I = make_inst_d(*s);
    double gtt, gij[3][3];
    inverse_metric(I, x, gtt, gij);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gi[3 * a + b] = gij[a][b];
}

double orc_resonance_radius(const orc_star* s, const double nhat[3], const double khat[3], double t0) {
    Inst<double> I = make_inst_d(*s);
    return resonance_radius_t(I, nhat, t0, khat);
}

double orc_energy_aniso(const orc_star* s, const double x[3], double t, const double k[3]) {
    Inst<double> I = make_inst_d(*s);
    return energy_t(I, x, t, k);
}

int orc_sample(const orc_star* s, uint64_t seed, int32_t instance, int64_t first, int64_t n, double* rays,
               int32_t* status, int nthreads) {
    Inst<double> I = make_inst_d(*s);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads_or_default(nthreads))
    for (int64_t j = 0; j < n; ++j) {
        SeedOut<double> o = seed_ray(I, seed, instance, first + j);
        for (int d = 0; d < 8; ++d) rays[d * n + j] = o.y[d];
        rays[8 * n + j] = o.w;
        rays[9 * n + j] = o.rc;
        status[j] = o.status;
    }
    return 0;
}

int orc_trace_forward(const orc_star* s, const orc_tol* tol, const double* rays, const int32_t* status_in, int64_t n,
                      double* fin, int32_t* ifin, int nthreads, int kinks) {
    Inst<double> I = make_inst_d(*s);
    // flat-propagation variant: the seeds carry curved initial conditions, Hamilton's
    // equations are integrated with M = 0
    if (I.flags & ORC_FLAG_FLAT_PROPAGATION) I.rs = 0.0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
    for (int64_t j = 0; j < n; ++j) {
        if (status_in && status_in[j] != ORC_OK) {
            for (int d = 0; d < ORC_NFIN; ++d) fin[d * n + j] = 0.0;
            ifin[j] = 0; ifin[n + j] = 0; ifin[2 * n + j] = status_in[j];
            continue;
        }
        double y0[8];
        for (int d = 0; d < 8; ++d) y0[d] = rays[d * n + j];
        TraceOut<double> o = trace_one<double, double>(I, *tol, y0, 1.0, nullptr, nullptr, 0, kinks != 0);
        store_final(I, o, j, n, fin, ifin);
    }
    return 0;
}

int orc_trace_reverse(const orc_star* s, const orc_tol* tol, const double* rays, int64_t n, double lam_stop_abs,
                      double* fin, int32_t* ifin, int nthreads) {
    // Integrate dy/dl = -f(y) from the given states for a parameter length
    // lam_stop_abs (used to send escaped rays back to their seeds).  The last
    // step is shortened to land on it.
    Inst<double> I = make_inst_d(*s);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
    for (int64_t j = 0; j < n; ++j) {
        double y[8], k1[8];
        for (int d = 0; d < 8; ++d) y[d] = rays[d * n + j];
        double stop = (lam_stop_abs > 0) ? lam_stop_abs : rays[8 * n + j];
        auto f = [&](const double* yy, double* ff) { rhs_t(I, yy, ff, -1.0); };
        f(y, k1);
        double h = initial_step(f, y, k1, tol->rtol, tol->atol);
        double lam = 0, facmax = 10;
        int64_t nacc = 0, nrej = 0;
        Step<double> st;
        int status = ORC_OK;
        while (lam < stop) {
            bool last = false;
            if (lam + h >= stop) { h = stop - lam; last = true; }
            dopri_step(f, y, k1, h, st);
            double err = err_norm(y, st, tol->rtol, tol->atol);
            if (!std::isfinite(err)) err = 1e300;
            if (err > 1.0) { ++nrej; h *= std::max(0.2, 0.9 * std::pow(err, -0.2)); facmax = 1.0; continue; }
            ++nacc;
            lam += h;
            for (int d = 0; d < 8; ++d) { y[d] = st.ynew[d]; k1[d] = st.K[6][d]; }
            if (last) { status = ORC_ESCAPED; break; }
            double fac = (err == 0.0) ? facmax : std::min(facmax, std::max(0.2, 0.9 * std::pow(err, -0.2)));
            h *= fac; facmax = 10.0;
            if (nacc >= tol->max_steps) { status = ORC_MAX_STEPS; break; }
        }
        for (int d = 0; d < 8; ++d) fin[d * n + j] = y[d];
        for (int d = 8; d < ORC_NFIN; ++d) fin[d * n + j] = 0.0;
        fin[13 * n + j] = lam;
        ifin[j] = (int32_t)nacc; ifin[n + j] = (int32_t)nrej; ifin[2 * n + j] = status;
    }
    return 0;
}

int orc_bin(const double* fin, const int32_t* ifin, const double* w, int64_t n, int32_t nt, int32_t np, int32_t nw,
            double dw, double* hist, double* cnt, double* over) {
    // top-hat window on the sky (Sec. 2.2): uniform bins in theta, in the
    // co-rotating azimuth psi, and in the frequency offset at infinity, the
    // line centre (w_f = 1) sitting at the centre of a frequency bin
    const double dth = PI / nt, dps = 2.0 * PI / np;
    std::memset(hist, 0, sizeof(double) * (size_t)nt * np * nw);
    std::memset(cnt, 0, sizeof(double) * (size_t)nt * np * nw);
    over[0] = over[1] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (ifin[2 * n + i] != ORC_ESCAPED) continue;
        double th = fin[8 * n + i], ps = fin[10 * n + i], om = fin[11 * n + i];
        int it = std::min((int)std::floor(th / dth), nt - 1);
        int ip = std::min((int)std::floor(ps / dps), np - 1);
        double iwf = std::floor((om - 1.0) / dw + 0.5) + (double)(nw / 2);
        if (it < 0) it = 0;
        if (ip < 0) ip = 0;
        if (!(iwf >= 0.0 && iwf < (double)nw)) { over[0] += w[i]; over[1] += 1.0; continue; }
        int iw = (int)iwf;
        size_t b = ((size_t)it * np + ip) * nw + iw;
        hist[b] += w[i];
        cnt[b] += 1.0;
    }
    return 0;
}

int orc_trace_backward(const orc_star* s, const orc_tol* tol, double D_km, double incl, double phi_o,
                       double half_width_km, int32_t nx, int32_t ny, int32_t i0, int32_t j0, int32_t stride,
                       int32_t ni, int32_t nj, int32_t K, double* ev, int32_t* nev, double* fin, int32_t* ifin,
                       int nthreads) {
    Inst<double> I = make_inst_d(*s);
    int64_t n = (int64_t)ni * nj;
    for (int64_t q = 0; q < (int64_t)K * ORC_NEV * n; ++q) ev[q] = 0.0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
    for (int64_t q = 0; q < n; ++q) {
        int32_t a = (int32_t)(q / nj), b = (int32_t)(q % nj);
        backward_pixel(I, *tol, D_km, incl, phi_o, half_width_km, nx, ny, i0 + a * stride, j0 + b * stride, K, q, n,
                       ev, nev, fin, ifin);
    }
    return 0;
}

int orc_backward_rays(const orc_star* s, const orc_tol* tol, double D_km, double incl, double phi_o,
                      const double* b1, const double* b2, int64_t n, int32_t K, double Lc_max_km, double* wsum,
                      double* ev, int32_t* nev, double* fin, int32_t* ifin, int nthreads) {
    Inst<double> I = make_inst_d(*s);
    for (int64_t q = 0; q < (int64_t)K * ORC_NEV * n; ++q) ev[q] = 0.0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
    for (int64_t q = 0; q < n; ++q) {
        backward_ray(I, *tol, D_km, incl, phi_o, b1[q], b2[q], K, q, n, ev, nev, fin, ifin);
        double acc = 0.0;
        const int m = std::min(nev[q], K);
        for (int e = 0; e < m; ++e) {
            double ye[8];
            for (int d = 0; d < 8; ++d) ye[d] = ev[((int64_t)e * ORC_NEV + d) * n + q];
            acc += event_weight(I, ye, Lc_max_km, nullptr);
        }
        wsum[q] = acc;
    }
    return 0;
}

double orc_maxwell_x(double u) { return maxwell_x(u); }

int orc_open_field(const orc_star* s, const double* x, double t) {
    Inst<double> I = make_inst_d(*s);
    return on_open_field_line(I, x, t) ? 1 : 0;
}

int orc_cyclotron_depth(const orc_star* s, const double* fin, const int32_t* ifin, const double* r_emit, int64_t n,
                        double* tau, double* r_cyc) {
    Inst<double> I = make_inst_d(*s);
    for (int64_t q = 0; q < n; ++q) {
        tau[q] = 0.0;
        r_cyc[q] = -1.0;
        if (ifin[2 * n + q] != ORC_ESCAPED) continue;
        double f[ORC_NFIN];
        for (int d = 0; d < ORC_NFIN; ++d) f[d] = fin[(int64_t)d * n + q];
        tau[q] = cyclotron_tau(I, f, r_emit[q], &r_cyc[q]);
    }
    return 0;
}

int orc_event_weight(const orc_star* s, const double* y, double Lc_max_km, double* w, double* Lc) {
    Inst<double> I = make_inst_d(*s);
    *w = event_weight(I, y, Lc_max_km, Lc);
    return 0;
}

int orc_dopri_test(int32_t problem, double rtol, double atol, double t_end, double* y_end, int64_t* n_acc,
                   int64_t* n_rej, double h_fixed, double* dense_err) {
    // problem 0: four harmonic oscillators q' = w p, p' = -w q (w = 1, 2, 3, 0.5)
    // problem 1: exponentials y_i' = c_i y_i (c = 1, -1, 0.5, -0.5, 2, -2, 0.25, 0)
    const double wq[4] = {1.0, 2.0, 3.0, 0.5};
    const double cc[8] = {1.0, -1.0, 0.5, -0.5, 2.0, -2.0, 0.25, 0.0};
    auto f = [&](const double* y, double* fo) {
        if (problem == 0) {
            for (int i = 0; i < 4; ++i) { fo[i] = wq[i] * y[4 + i]; fo[4 + i] = -wq[i] * y[i]; }
        } else {
            for (int i = 0; i < 8; ++i) fo[i] = cc[i] * y[i];
        }
    };
    auto exact = [&](double t, double* ye) {
        if (problem == 0) {
            for (int i = 0; i < 4; ++i) { ye[i] = std::sin(wq[i] * t); ye[4 + i] = std::cos(wq[i] * t); }
        } else {
            for (int i = 0; i < 8; ++i) ye[i] = std::exp(cc[i] * t);
        }
    };
    double y[8], k1[8];
    exact(0.0, y);
    f(y, k1);
    double h = (h_fixed > 0) ? h_fixed : initial_step(f, y, k1, rtol, atol);
    double t = 0, facmax = 10, dmax = 0;
    int64_t na = 0, nr = 0;
    Step<double> st;
    while (t < t_end * (1 - 1e-15)) {
        if (t + h > t_end) h = t_end - t;
        dopri_step(f, y, k1, h, st);
        double err = err_norm(y, st, rtol, atol);
        if (h_fixed <= 0 && err > 1.0) {
            ++nr; h *= std::max(0.2, 0.9 * std::pow(err, -0.2)); facmax = 1.0; continue;
        }
        ++na;
        if (h_fixed > 0) {
            // local error of the continuous extension: restart from the exact
            // solution so only the one-step error is measured
            double ys[8], k1s[8];
            exact(t, ys);
            f(ys, k1s);
            Step<double> s2;
            dopri_step(f, ys, k1s, h, s2);
            const double ths[3] = {0.3, 0.5, 0.7};
            for (double th : ths) {
                double yd[8], ye[8];
                dense_eval(ys, s2, h, th, yd);
                exact(t + th * h, ye);
                for (int d = 0; d < 8; ++d) dmax = std::max(dmax, std::fabs(yd[d] - ye[d]));
            }
        }
        t += h;
        for (int d = 0; d < 8; ++d) { y[d] = st.ynew[d]; k1[d] = st.K[6][d]; }
        if (h_fixed <= 0) {
            double fac = (err == 0.0) ? facmax : std::min(facmax, std::max(0.2, 0.9 * std::pow(err, -0.2)));
            h *= fac; facmax = 10.0;
        }
    }
    for (int d = 0; d < 8; ++d) y_end[d] = y[d];
    *n_acc = na; *n_rej = nr;
    if (dense_err) *dense_err = dmax;
    return 0;
}

int orc_flux_fwdmode(const orc_star* s, const orc_tol* tol, uint64_t seed, int64_t n, const double* obs,
                     int32_t n_obs, double sigma, double* flux, double* dflux, double* fray, double* dray,
                     int32_t* ray_status, int nthreads) {
    using D6 = Dual<6, double>;
    D6 p[6];
    double pv[6] = {s->B0_G, s->P_s, s->theta_m, s->M_Msun, s->R_km, s->m_a_eV};
    for (int q = 0; q < 6; ++q) p[q] = D6::var(pv[q], q);
    Inst<D6> I = make_inst<D6>(*s, p);
    std::vector<double> acc((size_t)n_obs * 7, 0.0);
#pragma omp parallel num_threads(nthreads_or_default(nthreads))
    {
        std::vector<double> loc((size_t)n_obs * 7, 0.0);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            if (fray)
                for (int j = 0; j < n_obs; ++j) fray[(size_t)i * n_obs + j] = 0.0;
            if (dray)
                for (int q = 0; q < n_obs * 6; ++q) dray[(size_t)i * n_obs * 6 + q] = 0.0;
            SeedOut<D6> so = seed_ray(I, seed, 0, i);
            if (ray_status) ray_status[i] = so.status;
            if (so.status != ORC_OK) continue;
            TraceOut<D6> o = trace_one<D6, D6>(I, *tol, so.y, 1.0, nullptr, nullptr, 0, true);
            if (ray_status) ray_status[i] = o.status;
            if (o.status != ORC_ESCAPED) continue;
            D6 th, ph, ps, v[3];
            observables(I, o.yf, th, ph, ps, v);
            D6 nh[3] = {sin(th) * cos(ps), sin(th) * sin(ps), cos(th)};
            for (int j = 0; j < n_obs; ++j) {
                D6 c = nh[0] * obs[3 * j] + nh[1] * obs[3 * j + 1] + nh[2] * obs[3 * j + 2];
                D6 contrib = so.w * kernel_K(c, sigma);
                loc[(size_t)j * 7] += contrib.v;
                for (int q = 0; q < 6; ++q) loc[(size_t)j * 7 + 1 + q] += contrib.d[q];
                if (fray) fray[(size_t)i * n_obs + j] = contrib.v / (double)n;
                if (dray)
                    for (int q = 0; q < 6; ++q) dray[((size_t)i * n_obs + j) * 6 + q] = contrib.d[q] / (double)n;
            }
        }
#pragma omp critical
        for (size_t q = 0; q < loc.size(); ++q) acc[q] += loc[q];
    }
    for (int j = 0; j < n_obs; ++j) {
        flux[j] = acc[(size_t)j * 7] / (double)n;
        for (int q = 0; q < 6; ++q) dflux[j * 6 + q] = acc[(size_t)j * 7 + 1 + q] / (double)n;
    }
    return 0;
}

int orc_flux_replay(const orc_star* s, const orc_tol* tol, uint64_t seed, int64_t n, const double* obs, int32_t n_obs,
                    double sigma, int32_t record, int32_t max_rec, double* hseq, int32_t* nseq, int32_t* stat,
                    double* flux, int nthreads) {
    Inst<double> I = make_inst_d(*s);
    std::vector<double> acc((size_t)n_obs, 0.0);
#pragma omp parallel num_threads(nthreads_or_default(nthreads))
    {
        std::vector<double> loc((size_t)n_obs, 0.0);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            SeedOut<double> so = seed_ray(I, seed, 0, i);
            TraceOut<double> o;
            if (record) {
                if (so.status != ORC_OK) { stat[i] = so.status; nseq[i] = 0; continue; }
                std::vector<double> hr;
                o = trace_one<double, double>(I, *tol, so.y, 1.0, &hr, nullptr, 0, true);
                int32_t m = (int32_t)std::min<size_t>(hr.size(), (size_t)max_rec);
                for (int32_t q = 0; q < m; ++q) hseq[(size_t)i * max_rec + q] = hr[q];
                nseq[i] = m;
                stat[i] = (hr.size() > (size_t)max_rec) ? ORC_MAX_STEPS : o.status;
                if (stat[i] != ORC_ESCAPED) continue;
            } else {
                if (stat[i] != ORC_ESCAPED || so.status != ORC_OK) continue;
                o = trace_one<double, double>(I, *tol, so.y, 1.0, nullptr, hseq + (size_t)i * max_rec, nseq[i], true);
                if (o.status != ORC_ESCAPED) {
                    // the replayed final step no longer reaches r_max: locate on its extension anyway
                    continue;
                }
            }
            double th, ph, ps, v[3];
            observables(I, o.yf, th, ph, ps, v);
            double nh[3] = {std::sin(th) * std::cos(ps), std::sin(th) * std::sin(ps), std::cos(th)};
            for (int j = 0; j < n_obs; ++j) {
                double c = nh[0] * obs[3 * j] + nh[1] * obs[3 * j + 1] + nh[2] * obs[3 * j + 2];
                loc[j] += so.w * kernel_K(c, sigma);
            }
        }
#pragma omp critical
        for (int j = 0; j < n_obs; ++j) acc[j] += loc[j];
    }
    for (int j = 0; j < n_obs; ++j) flux[j] = acc[j] / (double)n;
    return 0;
}

}  // extern "C"
