// Star constants and resonance seeding, generic in the scalar type so that the
// same code yields values (double) and their derivatives with respect to the six
// star parameters p = (B0, P, theta_m, M, R, m_a) (dual numbers), for the adjoint.
//
// McDonald & Witte, arXiv:2309.08655: Sec. 2.2 eq. (Power) (forward Monte Carlo),
// Sec. 3 eqs. (Hypersurfaces), (ForwardTracingEquation1) (resonance foliation),
// Sec. 4.2 eqs. (RaidalHypersurface)-(PowerCurved) (surface measure), Sec. 4.3
// eq. (fa_approx) (focused axion density), Sec. 4.4 eqs. (ProbIsoCurved),
// (CPAnisoCurved) (conversion probability times flux projection), Sec. 5 eq.
// (GJDensity) and Sec. 6 eq. (neMag) (densities).
#pragma once

#include "rt_device.hpp"

namespace rtd {

// CODATA 2018 / IAU 2015 constants used by the library
namespace phys {
constexpr double pi = 3.14159265358979323846;
constexpr double c_kms = 299792.458;
constexpr double c_cms = 2.99792458e10;
constexpr double hbarc_eVkm = 1.973269804e-10;
constexpr double hbarc_eVcm = 1.973269804e-5;
constexpr double alpha = 1.0 / 137.035999084;
constexpr double m_e_eV = 510998.95;
constexpr double e_statC = 4.803204712570263e-10;
constexpr double GMsun_km = 1.4766250;
constexpr double erg_per_eV = 1.602176634e-12;
// 1 G in eV^2 (Heaviside-Lorentz, hbar = c = 1): B^2/(8 pi) erg/cm^3 = B_HL^2 / 2
RT_HD double gauss_eV2() { return ::sqrt(hbarc_eVcm * hbarc_eVcm * hbarc_eVcm / (erg_per_eV * 4.0 * pi)); }
// w_p^2 = 4 pi alpha n_e / m_e  [eV^2 per cm^-3]
RT_HD double wp2_per_ne() { return 4.0 * pi * alpha * hbarc_eVcm * hbarc_eVcm * hbarc_eVcm / m_e_eV; }
// electron cyclotron energy per gauss, hbar e B / (m_e c)  [eV / G]
RT_HD double hbar_wc_per_G() { return hbarc_eVcm * e_statC / (m_e_eV * erg_per_eV); }
}  // namespace phys

// parameters of a star that are never differentiated
struct StarFixed {
    double g_agg_GeV, v0_kms, rho_GeVcm3, multiplicity, psi_twist, B_test_G;
    int plasma, density, weights, kdir, speeds, flags;
};

// seeding / weight constants
template <class T>
struct SeedT {
    T B0;          // polar surface field [G]
    T period_km;   // P c [km]
    T w_inf;       // axion energy at infinity [eV]
    T nc_per_ka;   // n_inf w_inf / k0 [eV^3], multiplies |k_a|/w_inf
    double g2;     // coupling^2 [eV^-2]
    double G2;     // 1 gauss in eV^2
    double Btest;  // constant |B_perp| [G] (zero-variance test)
    double hbarc;  // [eV km]
    double kv2;    // (k0 / w_inf)^2 = v0^2 / (1 + v0^2)
    int weights, kdir, speeds, flags;
};

template <class T>
RT_HD void sincos_any(const T& x, T* s, T* c) {
    sincos_t(x, s, c);
}

// integrator-unit constants of one star: p = (B0 [G], P [s], theta_m [rad], M [Msun], R [km], m_a [eV])
template <class T>
RT_HD InstT<T> make_inst_t(const T p[6], const StarFixed& f) {
    InstT<T> I;
    const T& B0 = p[0]; const T& Ps = p[1]; const T& th = p[2];
    const T& M = p[3]; const T& R = p[4]; const T& ma = p[5];
    I.rs = (2.0 * phys::GMsun_km) * M;
    I.R = R;
    I.R3 = R * R * R;
    T Om_s = (2.0 * phys::pi) * rcp(Ps);
    I.Om = Om_s * (1.0 / phys::c_kms);
    T s_, c_;
    sincos_any(th, &s_, &c_);
    I.cm = c_;
    I.sm = s_;
    I.oblique = (value(s_) != 0.0) ? 1 : 0;
    I.iOm = rcp(I.Om);
    I.Omsm = I.Om * I.sm;
    I.msm = T(0.0) - I.sm;
    // field shape: the Schwarzschild vacuum dipole, normalised to B0 at the surface pole
    I.gr_dipole = ((f.flags & FLAG_GR_DIPOLE) && value(I.rs) > 0.0) ? 1 : 0;
    I.bnorm = T(1.0);
    if (I.gr_dipole) {
        T G, G1, G2;
        gr_dipole_G(I.rs * rcp(R), G, G1, G2);
        I.bnorm = rcp(G);
    }
    double v0 = f.v0_kms / phys::c_kms;
    T w_inf = ma * ::sqrt(1.0 + v0 * v0);
    I.ma2 = T(1.0 / (1.0 + v0 * v0));
    T Cp = phys::wp2_per_ne() * rcp(w_inf * w_inf);
    // Goldreich-Julian number density scale Omega B0 / (4 pi e c) [cm^-3]
    T n0 = Om_s * B0 * (1.0 / (4.0 * phys::pi * phys::e_statC * phys::c_cms));
    if (f.density == DEN_GJ || f.density == DEN_SPH) {
        I.Cwp = (Cp * n0) * f.multiplicity;
    } else if (f.density == DEN_MAG) {
        // lambda psi B0 (R/r)^3 sin^2 / (4 pi e r_cm), r_cm = 1e5 r_km
        I.Cwp = Cp * B0 * (f.multiplicity * f.psi_twist / (4.0 * phys::pi * phys::e_statC * 1.0e5));
    } else {
        I.Cwp = T(0.0);
    }
    I.plasma = f.plasma;
    I.density = f.density;
    // finite magnetisation: (w_L / w_inf)^2 = kL r^-6 F^2 (1 + c mu^2), w_L = e|B|/(m_e c) the
    // cyclotron frequency of the dipole field B = (B0/2) bnorm (R/r)^3 F |g mu n - m|
    I.larmor = (f.flags & FLAG_FINITE_LARMOR) ? 1 : 0;
    const T bL = (0.5 * phys::hbar_wc_per_G()) * B0 * I.bnorm * rcp(w_inf);
    I.kL = (bL * bL) * (I.R3 * I.R3);
    I.CwpR3 = I.Cwp * I.R3;
    return I;
}

template <class T>
RT_HD SeedT<T> make_seed_t(const T p[6], const StarFixed& f) {
    SeedT<T> C;
    double v0 = f.v0_kms / phys::c_kms;
    C.B0 = p[0];
    C.period_km = p[1] * phys::c_kms;
    C.w_inf = p[5] * ::sqrt(1.0 + v0 * v0);
    double rho_eV4 = f.rho_GeVcm3 * 1.0e9 * phys::hbarc_eVcm * phys::hbarc_eVcm * phys::hbarc_eVcm;
    // n_inf w_inf / k0 = (rho / m_a) sqrt(1 + v0^2) / v0
    C.nc_per_ka = rho_eV4 * (::sqrt(1.0 + v0 * v0) / v0) * rcp(p[5]);
    double g = f.g_agg_GeV * 1.0e-9;
    C.g2 = g * g;
    C.G2 = phys::gauss_eV2();
    C.Btest = f.B_test_G;
    C.hbarc = phys::hbarc_eVkm;
    C.weights = f.weights;
    C.kdir = f.kdir;
    C.speeds = f.speeds;
    C.flags = f.flags;
    C.kv2 = v0 * v0 / (1.0 + v0 * v0);
    return C;
}

template <class S, class T>
RT_HD InstT<S> lift_inst(const InstT<T>& I) {
    InstT<S> J;
    J.rs = S(I.rs); J.R = S(I.R); J.Om = S(I.Om); J.cm = S(I.cm); J.sm = S(I.sm); J.Cwp = S(I.Cwp);
    J.R3 = S(I.R3); J.ma2 = S(I.ma2); J.bnorm = S(I.bnorm); J.kL = S(I.kL);
    J.iOm = S(I.iOm); J.Omsm = S(I.Omsm); J.msm = S(I.msm); J.CwpR3 = S(I.CwpR3);
    J.plasma = I.plasma; J.density = I.density; J.oblique = I.oblique; J.gr_dipole = I.gr_dipole;
    J.larmor = I.larmor;
    return J;
}

// Resonance function of the foliation (kinematic matching k^a = k^gamma at fixed axion
// direction kh in the static frame and fixed emission time):
//   F = P (w^2 - |k_a|^2 cos^2 theta_B) - m_a^2 w^2, w^2 = 1/A, |k_a|^2 = w^2 - m_a^2
// (isotropic plasma: F = P - m_a^2), at a general point x, for axis m.  It is w^2 H at the
// axion's momentum (k^2 = -m_a^2); with finite magnetisation H gains -a Q^2/(L k^2), so F
// gains w^2 (w^2 - P)(P - m_a^2)^2 / (L m_a^2), L = (w_L / w_inf)^2.
template <class S, class T>
RT_HD S resonance_point(const InstT<T>& I, const S x[3], const T m[3], const double kh[3], double om2, bool thin) {
    InstT<S> J = lift_inst<S>(I);
    S r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    S ir = rcp(r);
    S n[3] = {x[0] * ir, x[1] * ir, x[2] * ir};
    S mm[3] = {S(m[0]), S(m[1]), S(m[2])};
    S mu = mm[0] * n[0] + mm[1] * n[1] + mm[2] * n[2];
    Plasma<S> pl = plasma_eval(J, n, ir, mm, mu, S(0.0));
    if (I.plasma == PL_ISO || thin) return pl.P - J.ma2;
    S gsh = S(3.0), csh = S(3.0);
    if (I.gr_dipole) {
        const DipoleShape<S> sh = dipole_shape(J, ir);
        gsh = sh.g;
        csh = sh.c;
    }
    S u[3];
    for (int i = 0; i < 3; ++i) u[i] = gsh * mu * n[i] - mm[i];
    S ku = kh[0] * u[0] + kh[1] * u[1] + kh[2] * u[2];
    S cB2 = ku * ku * rcp(1.0 + csh * mu * mu);
    S w2 = om2 * rcp(1.0 - J.rs * ir);
    S F = pl.P * (w2 - (w2 - J.ma2) * cB2) - J.ma2 * w2;
    if (I.larmor) {
        S fsh = S(1.0);
        if (I.gr_dipole) fsh = dipole_shape(J, ir).F;
        const S ir2 = ir * ir;
        const S L = J.kL * (ir2 * ir2 * ir2) * (fsh * fsh) * (1.0 + csh * mu * mu);
        const S Qv = pl.P - J.ma2;
        F = F + w2 * (w2 - pl.P) * Qv * Qv * rcp(L * J.ma2);
    }
    return F;
}

// F along the radial line through n at radius r (values only: the bisection)
template <class T>
RT_HD double resonance_line(const InstT<T>& I, const double n[3], const double m[3], double mu, double cB2,
                            double om2, bool thin, double r, const double kh[3]) {
    InstT<double> J;
    J.rs = value(I.rs); J.R = value(I.R); J.Om = value(I.Om); J.cm = value(I.cm); J.sm = value(I.sm);
    J.Cwp = value(I.Cwp); J.R3 = value(I.R3); J.ma2 = value(I.ma2); J.bnorm = value(I.bnorm);
    J.iOm = value(I.iOm); J.Omsm = value(I.Omsm); J.msm = value(I.msm); J.CwpR3 = value(I.CwpR3);
    J.plasma = I.plasma; J.density = I.density; J.oblique = I.oblique; J.gr_dipole = I.gr_dipole;
    J.kL = value(I.kL); J.larmor = I.larmor;
    double ir = 1.0 / r;
    Plasma<double> pl = plasma_eval(J, n, ir, m, mu, 0.0);
    if (I.plasma == PL_ISO || thin) return pl.P - J.ma2;
    double fsh = 1.0, csh = 3.0;
    if (I.gr_dipole) {  // the field direction along the line changes with r
        const DipoleShape<double> sh = dipole_shape(J, ir);
        double ku = 0.0;
        for (int i = 0; i < 3; ++i) ku += kh[i] * (sh.g * mu * n[i] - m[i]);
        cB2 = ku * ku / (1.0 + sh.c * mu * mu);
        fsh = sh.F;
        csh = sh.c;
    }
    double w2 = om2 / (1.0 - J.rs * ir);
    double F = pl.P * (w2 - (w2 - J.ma2) * cB2) - J.ma2 * w2;
    if (I.larmor) {
        const double ir2 = ir * ir;
        const double L = J.kL * (ir2 * ir2 * ir2) * (fsh * fsh) * (1.0 + csh * mu * mu);
        const double Qv = pl.P - J.ma2;
        F = F + w2 * (w2 - pl.P) * Qv * Qv / (L * J.ma2);
    }
    return F;
}

// Root of F along the radial line through n above the surface; -1 when F(R) <= 0 or F
// stays non-negative up to R 2^80.  The bracket [R 2^(j-1), R 2^j] is shrunk to adjacent
// doubles lo < hi with F(lo) > 0 and F(hi) <= 0 (or not a number), the pair a bisection
// reaches, and the midpoint returned.  The shrinking takes Illinois false-position points
// (the value at the end kept twice in a row is halved), which reach that pair in about a
// dozen evaluations instead of the ~55 of bisection.  Where the false-position point rounds
// onto an end (the root within rounding of it, or F exactly zero there), points 1, 2, 4, ...
// ulp inside that end close the bracket instead.  A midpoint replaces
// any point that is not strictly inside the bracket or whose end values are not finite
// with opposite signs, and after 40 points only midpoints are taken.  nevals, when given,
// counts evaluations.
template <class T>
RT_HD double resonance_radius(const InstT<T>& I, const double n[3], const double m[3], double mu, double cB2,
                              double om2, bool thin, const double kh[3], int* nevals = nullptr) {
    int ne = 1;
    const double R = value(I.R);
    double rcv = -1.0;
    const double fR = resonance_line(I, n, m, mu, cB2, om2, thin, R, kh);
    if (fR > 0.0) {
        double lo = R, hi = 2.0 * R, flo = fR;
        double fhi = resonance_line(I, n, m, mu, cB2, om2, thin, hi, kh);
        ++ne;
        int j = 0;
        while (!(fhi < 0.0) && j < 80) {
            lo = hi; flo = fhi; hi *= 2.0; ++j;
            fhi = resonance_line(I, n, m, mu, cB2, om2, thin, hi, kh);
            ++ne;
        }
        if (fhi < 0.0) {
            int kept = 0;               // +1: lo moved last, -1: hi moved last
            double dlo = 0.0, dhi = 0.0;  // probe offsets inside an end
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double x = mid;
                if (it < 40 && flo > 0.0 && fhi <= 0.0 && flo < 1e300 && fhi > -1e300) {
                    const double fp = lo + (hi - lo) * (flo / (flo - fhi));
                    if (fp > lo && fp < hi) {
                        x = fp;
                        dlo = dhi = 0.0;
                    } else if (fp >= hi) {
                        // the root is within rounding of hi (or F is zero there): probe
                        // 1, 2, 4, ... ulp below hi; bisect once the bracket is that narrow
                        dhi = (dhi == 0.0) ? hi * 0x1p-52 : 2.0 * dhi;
                        if (hi - lo > 4.0 * dhi) x = hi - dhi;
                    } else {
                        dlo = (dlo == 0.0) ? lo * 0x1p-52 : 2.0 * dlo;
                        if (hi - lo > 4.0 * dlo) x = lo + dlo;
                    }
                }
                const double f = resonance_line(I, n, m, mu, cB2, om2, thin, x, kh);
                ++ne;
                if (f > 0.0) {
                    lo = x; flo = f;
                    if (kept > 0) fhi *= 0.5;
                    kept = 1;
                } else {
                    hi = x; fhi = f;
                    if (kept < 0) flo *= 0.5;
                    kept = -1;
                }
            }
            rcv = 0.5 * (lo + hi);
        }
    }
    if (nevals) *nevals = ne;
    return rcv;
}

// Maxwellian momenta at infinity (Sec. 4.3 eq. (GaussianDist)): x = (|k_inf|/k0)^2 has the
// Gamma(3/2) distribution, density (2/sqrt pi) sqrt(x) e^{-x}.  maxwell_x(u) solves G(x) = u
// for its distribution function by Newton's method inside a shrinking bracket, with G from
// its power series x^{3/2} e^{-x}/Gamma(5/2) sum_j x^j/((5/2)...(3/2+j)) below the median and
// 1 - G = erfc(sqrt x) + (2/sqrt pi) sqrt(x) e^{-x} above it.
RT_HD double maxwell_x(double u) {
    const double c = 1.1283791670955126;  // 2/sqrt(pi)
    const bool upper = u >= 0.5;
    const double target = upper ? 1.0 - u : u;
    double lo = 0.0, hi = 100.0;
    // starting point: the leading term x^{3/2}/Gamma(5/2) below the median, the tail
    // c sqrt(x) e^{-x} ~ 1 - u above it
    double x = upper ? fmax(1.2, -::log(target)) : ::pow(1.3293403881791355 * target, 2.0 / 3.0);
    for (int it = 0; it < 100; ++it) {
        const double sx = ::sqrt(x), ex = ::exp(-x);
        double g;  // signed so that g increases with x
        if (upper) {
            g = target - (::erfc(sx) + c * sx * ex);
        } else {
            double term = 1.0, sum = 1.0;
            for (int j = 1; j < 60; ++j) {
                term *= x / (1.5 + j);
                sum += term;
                if (term < 1e-17 * sum) break;
            }
            g = x * sx * ex * (sum / 1.3293403881791355) - target;
        }
        if (g < 0.0) lo = x; else hi = x;
        const double dg = c * sx * ex;
        double xn = (dg > 0.0) ? x - g / dg : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (::fabs(xn - x) <= 2e-16 * xn || hi - lo <= 2e-16 * hi) { x = xn; break; }
        x = xn;
    }
    return x;
}

// Open field lines of the rotating dipole (Sec. 6): the line through x has apex
// L = r / sin^2 theta_mag; it is open when L >= r_LC = c / Omega, i.e. r >= r_LC sin^2 theta_mag.
template <class T>
RT_HD bool on_open_field_line(const InstT<T>& I, const double x[3], double t) {
    const double r = ::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double s, c;
    sincos_t(value(I.Om) * t, &s, &c);
    const double sm = value(I.sm);
    const double mu = (sm * c * x[0] + sm * s * x[1] + value(I.cm) * x[2]) / r;
    return r * value(I.Om) >= 1.0 - mu * mu;
}

// the six uniforms of ray gi (Philox4x32-10, key = seed, counter = (gi, instance, block))
RT_HD void ray_uniforms(uint64_t seed, int32_t instance, int64_t gi, double u[6]) {
    uint32_t o[4];
    for (uint32_t blk = 0; blk < 3; ++blk) {
        philox4x32_10((uint32_t)(uint64_t)gi, (uint32_t)((uint64_t)gi >> 32), (uint32_t)instance, blk,
                      (uint32_t)seed, (uint32_t)(seed >> 32), o);
        u[2 * blk] = unit_from_bits(o[0], o[1]);
        u[2 * blk + 1] = unit_from_bits(o[2], o[3]);
    }
}

// One seed: emission point on the resonance, photon momentum = axion momentum, weight.
// out = (x, y, z, t, k_x, k_y, k_z, k_t, w, r_c); returns the status.
template <class T>
RT_HD int seed_ray(const InstT<T>& I, const SeedT<T>& C, uint64_t seed, int32_t instance, int64_t gi, T out[10]) {
    double u[6];
    ray_uniforms(seed, instance, gi, u);
    // emission direction uniform in (cos theta, phi)
    double ct = 2.0 * u[0] - 1.0;
    double st = ::sqrt(fmax(0.0, 1.0 - ct * ct));
    double sp, cp;
    sincos_t(2.0 * phys::pi * u[1], &sp, &cp);
    double n[3] = {st * cp, st * sp, ct};
    double kh[3];
    {
        double sa, ca;
        sincos_t(2.0 * phys::pi * u[3], &sa, &ca);
        if (C.kdir == KD_ISO) {
            double c = 2.0 * u[2] - 1.0, s = ::sqrt(fmax(0.0, 1.0 - c * c));
            kh[0] = s * ca; kh[1] = s * sa; kh[2] = c;
        } else {
            // outward hemisphere about n: polar cosine u3, azimuth in the (theta-hat, phi-hat) basis
            double c = u[2], s = ::sqrt(fmax(0.0, 1.0 - c * c));
            double e1[3] = {ct * cp, ct * sp, -st};
            double e2[3] = {-sp, cp, 0.0};
            for (int d = 0; d < 3; ++d) kh[d] = c * n[d] + s * (ca * e1[d] + sa * e2[d]);
        }
    }
    T t0 = u[4] * C.period_km;
    T mT[3], mtT[3];
    magnetic_axis(I, t0, mT, mtT);
    double m[3] = {value(mT[0]), value(mT[1]), value(mT[2])};
    double mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
    double ud[3];
    for (int d = 0; d < 3; ++d) ud[d] = 3.0 * mu * n[d] - m[d];
    double ku = kh[0] * ud[0] + kh[1] * ud[1] + kh[2] * ud[2];
    double cB2 = ku * ku / (1.0 + 3.0 * mu * mu);
    // momentum at infinity: k0 = m_a v0, or Maxwellian (x = (k/k0)^2 from the sixth uniform);
    // energy at infinity om = sqrt(m~^2 + x kv2) in units of w_inf
    const double x2 = (C.speeds == SP_MAXWELL) ? maxwell_x(u[5]) : 1.0;
    const double om2 = value(I.ma2) + x2 * C.kv2;
    const double om = ::sqrt(om2);
    // thin-surface variant: the resonance on w_p = m_a alone
    const bool thin = (C.flags & FLAG_THIN_SURFACE) != 0;

    // root of F above the surface
    const double rcv = resonance_radius(I, n, m, mu, cB2, om2, thin, kh);
    if (rcv < 0.0) {
        for (int d = 0; d < 10; ++d) out[d] = T(0.0);
        out[9] = T(-1.0);
        return ST_NO_RESONANCE;
    }
    // r_c carries dr_c/dp = -(dF/dp)/(dF/dr) through one Newton correction (a no-op on the value)
    T rc = T(rcv);
    if constexpr (is_dual<T>::value) {
        typedef gdual<1, T> D1;
        D1 rd{T(rcv)};
        rd.d[0] = T(1.0);
        D1 xd[3] = {rd * n[0], rd * n[1], rd * n[2]};
        D1 Fd = resonance_point<D1, T>(I, xd, mT, kh, om2, thin);
        rc = T(rcv) - Fd.v * rcp(Fd.d[0]);
        set_value(rc, rcv);
    }
    T s = I.rs * rcp(rc);
    T A = 1.0 - s;
    T sA = sqrt(A);
    // |k_a|^2 = om^2/A - m~^2 = (x kv2 + m~^2 s)/A without the cancellation of the first form
    T ka = sqrt((x2 * C.kv2 + I.ma2 * s) * rcp(A));
    T x[3] = {rc * n[0], rc * n[1], rc * n[2]};
    if (C.flags & FLAG_EXCISE_OPEN) {
        const double xv[3] = {rcv * n[0], rcv * n[1], rcv * n[2]};
        if (on_open_field_line(I, xv, value(t0))) {
            for (int d = 0; d < 9; ++d) out[d] = T(0.0);
            out[9] = rc;
            return ST_EXCISED;
        }
    }
    // photon covariant momentum from the static-frame axion momentum |k_a| kh; on the thin
    // surface the photon keeps kh and the frequency, with |k|^2 = E^2 (E^2 - P)/(E^2 - P cos^2)
    // from the LO dispersion relation (P = w_p^2 there)
    T kg = ka;
    if (thin && I.plasma == PL_ANISO) {
        T ir0 = rcp(rc);
        T nT0[3] = {T(n[0]), T(n[1]), T(n[2])};
        T mu0 = mT[0] * nT0[0] + mT[1] * nT0[1] + mT[2] * nT0[2];
        Plasma<T> p0 = plasma_eval(I, nT0, ir0, mT, mu0, T(0.0));
        // cos^2 between kh and the dipole direction g mu n - m (the axis depends on theta_m, P)
        T g0 = T(3.0), c0 = T(3.0);
        if (I.gr_dipole) {
            const DipoleShape<T> sh0 = dipole_shape(I, ir0);
            g0 = sh0.g;
            c0 = sh0.c;
        }
        T ku0 = T(0.0);
        for (int d = 0; d < 3; ++d) ku0 = ku0 + kh[d] * (g0 * mu0 * n[d] - mT[d]);
        T cB20 = ku0 * ku0 * rcp(1.0 + c0 * mu0 * mu0);
        T E2 = om2 * rcp(A);
        kg = sqrt(E2 * (E2 - p0.P) * rcp(E2 - p0.P * cB20));
    }
    T ko[3] = {kg * kh[0], kg * kh[1], kg * kh[2]};
    T nko = n[0] * ko[0] + n[1] * ko[1] + n[2] * ko[2];
    T corr = nko * rcp(sA) - nko;
    T k[3] = {ko[0] + corr * n[0], ko[1] + corr * n[1], ko[2] + corr * n[2]};
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = t0;
    out[4] = k[0]; out[5] = k[1]; out[6] = k[2]; out[7] = T(-om);
    out[9] = rc;
    // flat-propagation variant: the photon leaves with its static-frame momentum and local
    // frequency (to be traced with M = 0); the weight below uses the curved state
    auto finish = [&]() {
        if (C.flags & FLAG_FLAT_PROPAGATION) {
            out[4] = ko[0]; out[5] = ko[1]; out[6] = ko[2];
            out[7] = -(om * rcp(sA));
        }
        return ST_OK;
    };
    if (C.weights == W_UNIT) { out[8] = T(1.0); return finish(); }

    // ---- weight w = C_k n_c Vt Q ----
    const double Ck = (C.kdir == KD_ISO) ? 4.0 * phys::pi : 2.0 * phys::pi;
    T n_c = C.nc_per_ka * ka * (1.0 / ::sqrt(x2));  // n_inf |k_a| / |k_inf|
    // surface element from grad F (dual numbers over x, 3 tangents)
    typedef gdual<3, T> D3;
    D3 xd[3];
    for (int d = 0; d < 3; ++d) { xd[d] = D3(x[d]); xd[d].d[d] = T(1.0); }
    D3 Fd = resonance_point<D3, T>(I, xd, mT, kh, om2, thin);
    T Fr = n[0] * Fd.d[0] + n[1] * Fd.d[1] + n[2] * Fd.d[2];
    T gp2 = T(0.0);
    for (int d = 0; d < 3; ++d) { T gp = Fd.d[d] - Fr * n[d]; gp2 = gp2 + gp * gp; }
    // sqrt|g_tt| times the printed sqrt|h_k| (which already carries A^{1/2})
    T Vt = A * rc * rc * sqrt(1.0 + gp2 * rcp(A * Fr * Fr)) * (1.0 / (C.hbarc * C.hbarc));
    // cos theta_n (eq. (AngleDef)): kh against the surface normal in the static orthonormal
    // frame, whose radial component is sqrt(A) F_r
    T khg = kh[0] * Fd.d[0] + kh[1] * Fd.d[1] + kh[2] * Fd.d[2];
    T khn = kh[0] * n[0] + kh[1] * n[1] + kh[2] * n[2];
    T cos_n = (khg - Fr * khn + sA * Fr * khn) * rcp(sqrt(gp2 + A * Fr * Fr));
    if (C.flags & FLAG_RENORM_WEIGHTS) {
        // Sec. 6 eq. (reweight): P_ag = 1, rescaled by (1 cm^-3/n_a)(m_a/|k_a|)/sqrt(A)
        const double n1 = phys::hbarc_eVcm * phys::hbarc_eVcm * phys::hbarc_eVcm;  // 1 cm^-3 [eV^3]
        T m_a = C.w_inf * sqrt(I.ma2);
        out[8] = Ck * Vt * fabs(cos_n) * m_a * n1 * rcp(sA);
        return finish();
    }
    T E = (C.w_inf * om) * rcp(sA);
    T ir = rcp(rc);
    T Rr = I.R * ir;
    T nT[3] = {T(n[0]), T(n[1]), T(n[2])};
    T muT = mT[0] * nT[0] + mT[1] * nT[1] + mT[2] * nT[2];
    T gT = T(3.0), cT = T(3.0), fT = T(1.0);
    if (I.gr_dipole) {
        const DipoleShape<T> shT = dipole_shape(I, ir);
        gT = shT.g;
        cT = shT.c;
        fT = I.bnorm * shT.F;
    }
    T Bmag = 0.5 * C.B0 * Rr * Rr * Rr * sqrt(1.0 + cT * muT * muT);
    if (I.gr_dipole) Bmag = Bmag * fT;
    T uT[3];
    for (int d = 0; d < 3; ++d) uT[d] = gT * muT * nT[d] - mT[d];
    T kuT = kh[0] * uT[0] + kh[1] * uT[1] + kh[2] * uT[2];
    T cB2T = kuT * kuT * rcp(1.0 + cT * muT * muT);
    T Bperp2 = (C.weights == W_CONV_CONSTB) ? T((C.Btest * C.G2) * (C.Btest * C.G2))
                                            : (Bmag * C.G2) * (Bmag * C.G2) * (1.0 - cB2T);
    T Q;
    Plasma<T> pl = plasma_eval(I, nT, ir, mT, muT, T(0.0));
    if (I.plasma == PL_ISO) {
        T gP[3];
        plasma_grad(pl, nT, mT, gP);
        T gn = n[0] * gP[0] + n[1] * gP[1] + n[2] * gP[2];
        T g2 = gP[0] * gP[0] + gP[1] * gP[1] + gP[2] * gP[2] - s * gn * gn;
        T dwp2 = C.hbarc * C.w_inf * C.w_inf * sqrt(g2);
        Q = (phys::pi * C.g2) * Bperp2 * E * E * rcp(dwp2);
    } else {
        // dE/dx at fixed covariant k from H(x, k_t, k) = 0 with w = -k_t/sqrt(A):
        //   dE/dx = (dH/dx) / (sqrt(A) dH/dk_t) - w s/(2 A r) n
        T y[8] = {x[0], x[1], x[2], t0, k[0], k[1], k[2], T(-om)};
        T g[8];
        grad_h(I, y, g);
        T w = om * rcp(sA);
        T c0 = rcp(sA * g[7]);
        T c1 = w * s * ir * rcp(2.0 * A);
        T dE[3] = {g[0] * c0 - c1 * n[0], g[1] * c0 - c1 * n[1], g[2] * c0 - c1 * n[2]};
        T dn = n[0] * dE[0] + n[1] * dE[1] + n[2] * dE[2];
        T dE2 = dE[0] * dE[0] + dE[1] * dE[1] + dE[2] * dE[2] - s * dn * dn;
        T dEn = C.hbarc * C.w_inf * sqrt(dE2);
        T wp2 = pl.P * C.w_inf * C.w_inf;
        T c2 = cB2T, s2 = 1.0 - cB2T;
        T Dd = (E * E - c2 * wp2) * (E * E - c2 * wp2) + c2 * s2 * wp2 * wp2;
        T E2 = E * E;
        if (thin) {
            // no cancellation on the thin surface: Q = |cos theta_n| v_a E P_ag, with the photon's
            // k.dE = k^a d_a E (contravariant k = k - s (n.k) n)
            T q = n[0] * k[0] + n[1] * k[1] + n[2] * k[2];
            T kdE = T(0.0);
            for (int a = 0; a < 3; ++a) kdE = kdE + (k[a] - s * q * n[a]) * dE[a];
            kdE = (C.hbarc * C.w_inf * C.w_inf) * kdE;
            T Pag = (0.5 * phys::pi * C.g2) * Bperp2 * E2 * E2 * E * rcp(Dd * fabs(kdE));
            Q = fabs(cos_n) * (ka * C.w_inf) * Pag;
        } else {
            Q = (0.5 * phys::pi * C.g2) * Bperp2 * E2 * E2 * E * rcp(Dd * dEn);
        }
    }
    out[8] = Ck * n_c * Vt * Q;
    return finish();
}

// Resonant cyclotron absorption (Sec. 6).  The escaped photon is taken to move radially along
// its asymptotic direction nhat: at radius r it is there at time t_f + (r - r_f) with local
// frequency w_f / sqrt(A(r)).  Its cyclotron resonance is where hbar e |B| / (m_e c) (dipole
// |B| = (B0/2)(R/r)^3 sqrt(1 + 3 mu^2)) equals that frequency, and there
//   tau = (pi/3) (w_p^2 / w) r.
// The root of ln(hbar w_c / w) is bracketed by doubling from R, then refined by the step
// r -> r exp(ln(hbar w_c / w)/3) (exact for the r^-3 falloff alone) inside the bracket, with
// geometric bisection whenever that step leaves it.  No absorption (tau = 0) without a
// resonance above the surface or with the emission point beyond it; *r_res = -1 when there
// is no resonance.
RT_HD double cyclotron_tau(const InstT<double>& I, const SeedT<double>& C, double th, double ph, double tf, double rf,
                           double omf, double r_emit, double* r_res) {
    double st, ct, sp, cp;
    sincos_t(th, &st, &ct);
    sincos_t(ph, &sp, &cp);
    const double nh[3] = {st * cp, st * sp, ct};
    const double wf = omf * value(C.w_inf);
    const double kc = phys::hbarc_eVcm * phys::e_statC / (phys::m_e_eV * phys::erg_per_eV);  // eV per gauss
    const double R = value(I.R);
    auto lng = [&](double r) {
        double m[3], mt[3];
        magnetic_axis(I, tf + (r - rf), m, mt);
        const double mu = m[0] * nh[0] + m[1] * nh[1] + m[2] * nh[2];
        const double Rr = R / r;
        const DipoleShape<double> sh = dipole_shape(I, 1.0 / r);
        const double B = 0.5 * value(C.B0) * value(I.bnorm) * sh.F * Rr * Rr * Rr * ::sqrt(1.0 + sh.c * mu * mu);
        return ::log(kc * B * ::sqrt(1.0 - value(I.rs) / r) / wf);
    };
    *r_res = -1.0;
    double glo = lng(R);
    if (!(glo > 0.0)) return 0.0;
    double lo = R, hi = 2.0 * R, ghi = lng(hi);
    for (int j = 0; j < 200 && !(ghi < 0.0); ++j) { lo = hi; glo = ghi; hi *= 2.0; ghi = lng(hi); }
    if (!(ghi < 0.0)) return 0.0;
    double r = lo * ::exp(glo / 3.0);
    if (!(r > lo && r < hi)) r = ::sqrt(lo * hi);
    for (int it = 0; it < 200; ++it) {
        const double g = lng(r);
        if (g > 0.0) lo = r; else hi = r;
        if (g == 0.0) break;
        double rn = r * ::exp(g / 3.0);
        if (!(rn > lo && rn < hi)) rn = ::sqrt(lo * hi);
        const bool done = ::fabs(rn - r) <= 1e-15 * r || hi - lo <= 1e-15 * hi;
        r = rn;
        if (done) break;
    }
    *r_res = r;
    if (r < r_emit) return 0.0;
    double m[3], mt[3];
    const double tc = tf + (r - rf);
    magnetic_axis(I, tc, m, mt);
    const double mu = m[0] * nh[0] + m[1] * nh[1] + m[2] * nh[2];
    const Plasma<double> pl = plasma_eval(I, nh, 1.0 / r, m, mu, 0.0);
    const double wp2 = pl.P * value(C.w_inf) * value(C.w_inf);
    const double w = wf / ::sqrt(1.0 - value(I.rs) / r);
    return (phys::pi / 3.0) * (wp2 / w) * (r / C.hbarc);
}

// Weight of one backward production event (Sec. 2.1 eq. (BackPower), Sec. 3): a ray's
// photon density is the sum over its events of P_ag f_a, with the focused monochromatic
// axion density f_a = v_a n_c delta(w - w_c)/(4 pi k^2) of Sec. 4.3 and P_ag of Sec. 4.4,
//   isotropic   P = pi g^2 |B_perp|^2 E^2 / |k.d(w_p^2)|,   eq. (ProbIsoCurved)
//   anisotropic P = (pi/2) g^2 |B_perp|^2 E^5 / (D |k.dE|),  eq. (CPAnisoCurved)
// with k.d = k^a d_a (contravariant spatial k; the plasma is quasi-stationary).  The
// frequency integral of w^3 f turns delta(w_inf/sqrt(A) - w_c) into sqrt(A), so the event
// adds w_inf^3 sqrt(A) P v_a n_c / (4 pi k^2) [eV^4] to dP/dOmega per unit image area.
// E is the event's own local frequency -k_t/sqrt(A); for the LO mode dE/dx at fixed
// covariant k follows from H(x, k_t, k) = 0:
//   dE/dx = (dH/dx)/(sqrt(A) dH/dk_t) - E s/(2 A r) n.
// The conversion length L_c = sqrt(2 pi v_a / |khat.dE|) [km] (isotropic: dE = d(w_p^2)/2E)
// is returned in *Lc; the event counts only if Lc_max <= 0 or L_c <= Lc_max (the IR
// cutoff of Sec. 4.4).
RT_HD double event_weight(const InstT<double>& I, const SeedT<double>& C, const double y[8], double Lc_max,
                          double* Lc) {
    if ((C.flags & FLAG_EXCISE_OPEN) && on_open_field_line(I, y, y[3])) {
        if (Lc) *Lc = 0.0;
        return 0.0;
    }
    const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    const double ir = rcp(::sqrt(r2));
    const double n[3] = {y[0] * ir, y[1] * ir, y[2] * ir};
    const double s = I.rs * ir;
    const double A = 1.0 - s;
    const double sA = ::sqrt(A);
    const double El = -y[7] * rcp(sA);  // local frequency [w_inf]
    const double q = n[0] * y[4] + n[1] * y[5] + n[2] * y[6];
    const double kk = y[4] * y[4] + y[5] * y[5] + y[6] * y[6];
    const double ku = ::sqrt(kk - s * q * q);  // static-frame |k| [w_inf]
    const double E = El * C.w_inf, kmag = ku * C.w_inf;
    const double va = ku * rcp(El);
    const double n_c = C.nc_per_ka * ku;
    // static-frame k = k + (sqrt(A) - 1) q n; contravariant k = k - s q n
    const double ko[3] = {y[4] + (sA - 1.0) * q * n[0], y[5] + (sA - 1.0) * q * n[1], y[6] + (sA - 1.0) * q * n[2]};
    const double kc[3] = {y[4] - s * q * n[0], y[5] - s * q * n[1], y[6] - s * q * n[2]};
    double m[3], mt[3];
    magnetic_axis(I, y[3], m, mt);
    const double mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
    const DipoleShape<double> sh = dipole_shape(I, ir);  // flat: g = c = 3, F = 1
    double u[3];
    dipole_dir(n, m, mu, u, sh.g);
    const double u2 = 1.0 + sh.c * mu * mu;
    const double ko_u = ko[0] * u[0] + ko[1] * u[1] + ko[2] * u[2];
    const double cB2 = ko_u * ko_u * rcp(ku * ku * u2);
    const double Rr = I.R * ir;
    const double Bmag = 0.5 * value(C.B0) * value(I.bnorm) * sh.F * Rr * Rr * Rr * ::sqrt(u2);
    const double Bperp2 = (C.weights == W_CONV_CONSTB) ? (C.Btest * C.G2) * (C.Btest * C.G2)
                                                       : (Bmag * C.G2) * (Bmag * C.G2) * (1.0 - cB2);
    const double w = value(C.w_inf);
    const Plasma<double> pl = plasma_eval(I, n, ir, m, mu, 0.0);
    double P, kdE;  // kdE = k^a d_a E [eV^2 / km]
    if (I.plasma == PL_ISO) {
        double gP[3];
        plasma_grad(pl, n, m, gP);
        const double kdw = kc[0] * gP[0] + kc[1] * gP[1] + kc[2] * gP[2];  // [w_inf^3 / km]
        P = (phys::pi * C.g2) * Bperp2 * E * E * rcp(::fabs(C.hbarc * w * w * w * kdw));
        kdE = w * w * w * kdw * rcp(2.0 * E);
    } else {
        double g[8];
        grad_h(I, y, g);
        const double c0 = rcp(sA * g[7]);
        const double c1 = El * s * ir * rcp(2.0 * A);
        const double kd = kc[0] * (g[0] * c0 - c1 * n[0]) + kc[1] * (g[1] * c0 - c1 * n[1]) +
                          kc[2] * (g[2] * c0 - c1 * n[2]);  // [w_inf^2 / km]
        const double wp2 = pl.P * w * w;
        const double s2 = 1.0 - cB2;
        const double D0 = E * E - cB2 * wp2;
        const double Dd = D0 * D0 + cB2 * s2 * wp2 * wp2;
        const double E2 = E * E;
        P = (0.5 * phys::pi * C.g2) * Bperp2 * E2 * E2 * E * rcp(Dd * ::fabs(C.hbarc * w * w * kd));
        kdE = w * w * kd;
    }
    const double Lcv = ::sqrt(2.0 * phys::pi * va * C.hbarc * kmag * rcp(::fabs(kdE)));
    if (Lc) *Lc = Lcv;
    if (Lc_max > 0.0 && Lcv > Lc_max) return 0.0;
    return w * w * w * sA * P * va * n_c * rcp(4.0 * phys::pi * kmag * kmag);
}

}  // namespace rtd
