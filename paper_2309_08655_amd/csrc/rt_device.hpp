// Device-side physics of the ray tracer (gfx950, FP64).
//
// Hamiltonian rays of McDonald & Witte, arXiv:2309.08655:
//   Sec. 2, eq. (Hamilton):           x' = dH/dk, k' = -dH/dx
//   Sec. 4.1, eqs. (StrongBHam), (SchwarzshildMetric1):
//       H = g^{mu nu} k_mu k_nu + (w^2 - k_par^2) w_p^2 / w^2  (strongly magnetised, LO mode)
//       H = g^{mu nu} k_mu k_nu + w_p^2                         (isotropic, eq. (DispIsotropic))
//   Sec. 5, eq. (GJDensity) and Sec. 6, eq. (neMag): plasma densities.
//
// State y = (x, y, z, t, k_x, k_y, k_z, k_t) in the Cartesian Schwarzschild chart
// (x = r n, r the areal radius; km), covariant momentum in units of the axion
// energy at infinity.  Inverse metric: g^tt = -1/A, g^ij = delta^ij - s n^i n^j,
// with A = 1 - s and s = r_s / r.  The static plasma frame sees w^2 = k_t^2 / A;
// its orthonormal components of k are sqrt(A)(n.k) radially, unchanged tangentially.
//
// The gradient of H is derived by hand (no automatic differentiation on the hot
// path).  Writing q = n.k, mu = m.n for the magnetic axis m(t), and
// N = (1 + 2 sqrt(A)) mu q - m.k, the dipole field direction gives
//   k_par^2 = N^2 / (1 + 3 mu^2),   K = k_par^2 / w^2 = A N^2 / (k_t^2 (1 + 3 mu^2)),
//   H_aniso = H_vac + P (1 - K),    H_vac = -k_t^2/A + |k|^2 - s q^2,  P = w_p^2 / w_inf^2.
// Every function is templated on the scalar so the same code runs in FP64 and
// in forward-mode dual numbers (Hessian-vector products of the adjoint).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rtd {

// ----------------------------------------------------------------------------
// scalar helpers (double)
// ----------------------------------------------------------------------------
#define RT_HD __host__ __device__ __forceinline__

using ::sqrt;
using ::fabs;
using ::exp;
using ::atan2;

RT_HD double rcp(double a) { return 1.0 / a; }
RT_HD double value(double a) { return a; }
RT_HD void sincos_t(double a, double* s, double* c) { ::sincos(a, s, c); }

// Reciprocal and reciprocal square root from the hardware estimates (v_rcp_f64,
// v_rsq_f64) refined by two Newton steps: within about one ulp for the normal,
// finite arguments that occur here, at a fraction of the cost of a correctly
// rounded division or square root.  Host builds use the exact operations.
RT_HD double frcp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}
// One Newton step only: about 1e-14 relative, for values that merely feed the step
// controller's accept test and step-size heuristic.
// A loop counter or index that has the same value in every lane of the wave, so held in a
// scalar register: its table look-ups become scalar loads and its tests scalar branches.
RT_HD int wave_uniform(int x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_readfirstlane(x);
#else
    return x;
#endif
}
RT_HD double frcp_coarse(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}
RT_HD double frsqrt(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double y = __builtin_amdgcn_rsq(x);
    double hx = 0.5 * x;
    double e = fma(-(hx * y), y, 0.5);
    y = fma(y, e, y);
    e = fma(-(hx * y), y, 0.5);
    return fma(y, e, y);
#else
    return 1.0 / ::sqrt(x);
#endif
}

// ----------------------------------------------------------------------------
// forward-mode dual number with N tangents of scalar type T (nestable:
// gdual<3, gdual<6>> carries mixed second derivatives), device and host
// ----------------------------------------------------------------------------
template <int N, class T = double>
struct gdual {
    T v;
    T d[N];
    __host__ __device__ gdual() : v(0.0) {
        for (int i = 0; i < N; ++i) d[i] = T(0.0);
    }
    __host__ __device__ gdual(double c) : v(c) {
        for (int i = 0; i < N; ++i) d[i] = T(0.0);
    }
    template <class U, class = typename std::enable_if<std::is_same<U, T>::value && !std::is_same<U, double>::value>::type>
    __host__ __device__ gdual(const U& c) : v(c) {
        for (int i = 0; i < N; ++i) d[i] = T(0.0);
    }
};

template <int N, class T> RT_HD double value(const gdual<N, T>& a) { return value(a.v); }

template <class X> struct is_dual { static const bool value = false; };
template <int N, class T> struct is_dual<gdual<N, T>> { static const bool value = true; };

// overwrite the value part, keeping every tangent
RT_HD void set_value(double& a, double v) { a = v; }
template <int N, class T> RT_HD void set_value(gdual<N, T>& a, double v) { set_value(a.v, v); }

template <int N, class T> RT_HD gdual<N, T> operator+(const gdual<N, T>& a, const gdual<N, T>& b) {
    gdual<N, T> r; r.v = a.v + b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N, class T> RT_HD gdual<N, T> operator-(const gdual<N, T>& a, const gdual<N, T>& b) {
    gdual<N, T> r; r.v = a.v - b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N, class T> RT_HD gdual<N, T> operator-(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = -a.v;
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N, class T> RT_HD gdual<N, T> operator*(const gdual<N, T>& a, const gdual<N, T>& b) {
    gdual<N, T> r; r.v = a.v * b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
// scalar (double, or the inner type T) on either side
template <int N, class T, class U>
using gd_scalar = typename std::enable_if<std::is_same<U, double>::value ||
                                              (std::is_same<U, T>::value && !std::is_same<T, double>::value),
                                          gdual<N, T>>::type;
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator*(const U& a, const gdual<N, T>& b) {
    gdual<N, T> r; r.v = a * b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a * b.d[i];
    return r;
}
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator*(const gdual<N, T>& b, const U& a) {
    return a * b;
}
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator+(const U& a, const gdual<N, T>& b) {
    gdual<N, T> r = b; r.v = a + b.v; return r;
}
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator+(const gdual<N, T>& b, const U& a) {
    gdual<N, T> r = b; r.v = b.v + a; return r;
}
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator-(const U& a, const gdual<N, T>& b) {
    return a + (-b);
}
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator-(const gdual<N, T>& b, const U& a) {
    gdual<N, T> r = b; r.v = b.v - a; return r;
}
template <int N, class T> RT_HD gdual<N, T> rcp(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = rcp(a.v);
    T g = -(r.v * r.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r;
}
template <int N, class T> RT_HD gdual<N, T> operator/(const gdual<N, T>& a, const gdual<N, T>& b) {
    return a * rcp(b);
}
template <int N, class T, class U> RT_HD gd_scalar<N, T, U> operator/(const U& a, const gdual<N, T>& b) {
    return a * rcp(b);
}
template <int N, class T> RT_HD gdual<N, T> operator/(const gdual<N, T>& a, double b) { return a * (1.0 / b); }
template <int N, class T> RT_HD gdual<N, T> sqrt(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = sqrt(a.v);
    T g = 0.5 * rcp(r.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r;
}
template <int N, class T> RT_HD void sincos_t(const gdual<N, T>& a, gdual<N, T>* s, gdual<N, T>* c) {
    T sv, cv;
    sincos_t(a.v, &sv, &cv);
    s->v = sv; c->v = cv;
    for (int i = 0; i < N; ++i) { s->d[i] = cv * a.d[i]; c->d[i] = -(sv * a.d[i]); }
}
template <int N, class T> RT_HD gdual<N, T> exp(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = exp(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = r.v * a.d[i];
    return r;
}
RT_HD double log1p_t(double a) { return ::log1p(a); }
template <int N, class T> RT_HD gdual<N, T> log1p_t(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = log1p_t(a.v);
    T g = rcp(1.0 + a.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r;
}
template <int N, class T> RT_HD gdual<N, T> atan2(const gdual<N, T>& y, const gdual<N, T>& x) {
    gdual<N, T> r; r.v = atan2(y.v, x.v);
    T den = rcp(x.v * x.v + y.v * y.v);
    for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) * den;
    return r;
}
template <int N, class T> RT_HD gdual<N, T> fabs(const gdual<N, T>& a) { return (value(a) < 0.0) ? -a : a; }
// the refined hardware estimates for the value, the exact derivative on top:
// d(1/a) = -(1/a)^2 da,  d(a^-1/2) = -(a^-1/2)^3 da / 2
template <int N, class T> RT_HD gdual<N, T> frcp(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = frcp(a.v);
    T g = -(r.v * r.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r;
}
template <int N, class T> RT_HD gdual<N, T> frsqrt(const gdual<N, T>& a) {
    gdual<N, T> r; r.v = frsqrt(a.v);
    T g = (-0.5 * r.v) * (r.v * r.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r;
}

// ----------------------------------------------------------------------------
// instance constants (integrator units: km, k in units of w_inf)
// ----------------------------------------------------------------------------
enum { PL_ISO = 0, PL_ANISO = 1 };
enum { DEN_GJ = 0, DEN_MAG = 1, DEN_SPH = 2, DEN_NONE = 3 };
enum { W_UNIT = 0, W_CONV = 1, W_CONV_CONSTB = 2 };
enum { KD_ISO = 0, KD_OUT = 1 };
enum { SP_MONO = 0, SP_MAXWELL = 1 };
enum { ST_OK = 0, ST_ESCAPED = 1, ST_HIT_STAR = 2, ST_NO_RESONANCE = 3, ST_MAX_STEPS = 4,
       ST_STEP_UNDERFLOW = 5, ST_NONFINITE = 6, ST_EXCISED = 7 };
enum { FLAG_EXCISE_OPEN = 1, FLAG_FLAT_PROPAGATION = 2, FLAG_RENORM_WEIGHTS = 4, FLAG_THIN_SURFACE = 8,
       FLAG_GR_DIPOLE = 16, FLAG_FINITE_LARMOR = 32 };

template <class T>
struct InstT {
    T rs;      // Schwarzschild radius [km]
    T R;       // stellar radius [km]
    T Om;      // rotation rate / c [rad/km]
    T cm, sm;  // cos / sin of the magnetic inclination
    T Cwp;     // plasma coefficient: P = Cwp * shape
    T R3;      // R^3
    T ma2;     // (m_a / w_inf)^2
    int plasma, density;
    int oblique;    // sm != 0
    int gr_dipole;  // the Schwarzschild vacuum dipole instead of the flat one
    T bnorm;        // field-strength factor: 1, or 1 / G(r_s/R) for the GR dipole (B0 at the pole)
    int larmor;     // finite magnetisation: the plasma response at the cyclotron frequency w_L
    T kL;           // (w_L / w_inf)^2 = kL r^-6 F^2 (1 + c mu^2): (hbar e B0 bnorm / (2 m_e c w_inf))^2 R^6
    // Products of the constants above, formed once by whoever builds the instance: a product
    // of two star constants formed in a kernel is hoisted out of its loops into a vector
    // register held (or spilled) for the whole launch, while these arrive with the other
    // constants in scalar registers.  Values only: dual-number code forms the products
    // itself where derivatives must flow through them.
    T iOm;    // 1 / Om
    T Omsm;   // Om sin theta_m
    T msm;    // -sin theta_m
    T CwpR3;  // Cwp R^3
};

// ----------------------------------------------------------------------------
// Dipole field shape.  The field is B = (B0/2) bnorm (R/r)^3 F (g mu n - m), mu = m.n, with
// |g mu n - m|^2 = 1 + c mu^2, c = g^2 - 2g.  Flat dipole: g = 3, c = 3, F = 1.  Schwarzschild
// vacuum dipole (x = r_s/r): the vector potential (mu sin^2/r) G(x),
//   G(x) = -3 [ln(1 - x) + x + x^2/2] / x^3,  F = sqrt(1 - x) (G + x G'),  g = 1 + 2G/F,
// with G from its power series 3 sum_j x^j/(j + 3) below x = 1/8 (no cancellation) and the
// logarithm above.  dg and dc are the radial derivatives of g and c.
// ----------------------------------------------------------------------------
template <class T>
struct DipoleShape {
    T g, c, F, dg, dc, dF;  // dg, dc, dF: radial derivatives
};

template <class T>
RT_HD void gr_dipole_G(const T& x, T& G, T& G1, T& G2) {
    if (value(x) < 0.125) {
        G = T(0.0); G1 = T(0.0); G2 = T(0.0);
        T xp = T(1.0), xm1 = T(0.0), xm2 = T(0.0);  // x^j, x^(j-1), x^(j-2)
        for (int j = 0; j < 26; ++j) {
            const double a = 3.0 / (j + 3.0);
            G = G + a * xp;
            if (j >= 1) G1 = G1 + (a * j) * xm1;
            if (j >= 2) G2 = G2 + (a * j * (j - 1)) * xm2;
            xm2 = xm1;
            xm1 = xp;
            xp = xp * x;
        }
    } else {
        const T ix = rcp(x), ix1 = rcp(1.0 - x);
        const T S = log1p_t(T(0.0) - x) + x + 0.5 * x * x;
        G = -3.0 * S * ix * ix * ix;
        G1 = 3.0 * ix * ix1 - 3.0 * G * ix;          // G' = 3/(x(1-x)) - 3G/x
        G2 = 3.0 * (2.0 * x - 1.0) * (ix * ix1) * (ix * ix1) - 3.0 * G1 * ix + 3.0 * G * ix * ix;
    }
}

template <class T>
RT_HD DipoleShape<T> dipole_shape(const InstT<T>& I, const T& ir) {
    DipoleShape<T> d;
    if (!I.gr_dipole) {
        d.g = T(3.0); d.c = T(3.0); d.F = T(1.0); d.dg = T(0.0); d.dc = T(0.0); d.dF = T(0.0);
        return d;
    }
    const T x = I.rs * ir;
    T G, G1, G2;
    gr_dipole_G(x, G, G1, G2);
    const T sq = sqrt(1.0 - x);
    const T H = G + x * G1;
    d.F = sq * H;
    const T dF = (0.0 - 0.5) * H * rcp(sq) + sq * (2.0 * G1 + x * G2);  // dF/dx
    const T iF = rcp(d.F);
    d.g = 1.0 + 2.0 * G * iF;
    const T dgdx = 2.0 * (G1 * d.F - G * dF) * iF * iF;
    d.dg = (0.0 - x * ir) * dgdx;  // dx/dr = -x/r
    d.c = d.g * d.g - 2.0 * d.g;
    d.dc = (2.0 * d.g - 2.0) * d.dg;
    d.dF = (0.0 - x * ir) * dF;
    return d;
}

// ----------------------------------------------------------------------------
// plasma: P = w_p^2 / w_inf^2, its spatial gradient and time derivative
// ----------------------------------------------------------------------------
template <class T>
struct Plasma {
    // P and its derivatives: grad_x P = pn n + pm m + pz e_z, dP/dt = pt
    T P, pn, pm, pz, pt;
    T g;  // GJ density: the factor g = 3 n_z mu - cos(theta_m) itself (0 for the others)
};

// the Cartesian components of grad_x P
template <class T>
RT_HD void plasma_grad(const Plasma<T>& p, const T n[3], const T m[3], T g[3]) {
    g[0] = p.pn * n[0] + p.pm * m[0];
    g[1] = p.pn * n[1] + p.pm * m[1];
    g[2] = p.pn * n[2] + p.pm * m[2] + p.pz;
}

// sin and cos of a rotation angle from Taylor polynomials: for |x| <= 1/32 the
// series truncated after x^7 and x^8; otherwise after x^13 and x^14 (error below
// 3e-17 for |x| <= 1/2), after halving the angle until |x| <= 1/2 and doubling back.
// No table, no library call.
template <class T>
RT_HD void small_angle_sincos(T x, T* s, T* c) {
    if (fabs(value(x)) <= 0.03125) {
        // the angles of the tracing kernels' stages: the series to x^7 and x^8 is exact to
        // below 3e-18 relative for |x| <= 1/32.  In nested form,
        //   sin x = x (1 - x^2/6 (1 - x^2/20 (1 - x^2/42))),
        //   cos x = 1 - x^2/2 (1 - x^2/12 (1 - x^2/30 (1 - x^2/56))),
        // every factor is one FMA onto the inline constant 1 (a Horner chain would need each
        // coefficient moved into the accumulator first).
        const T x2 = x * x;
        T ps = 1.0 + x2 * (-1.0 / 42.0);
        ps = 1.0 + (x2 * (-1.0 / 20.0)) * ps;
        ps = 1.0 + (x2 * (-1.0 / 6.0)) * ps;
        *s = x * ps;
        T pc = 1.0 + x2 * (-1.0 / 56.0);
        pc = 1.0 + (x2 * (-1.0 / 30.0)) * pc;
        pc = 1.0 + (x2 * (-1.0 / 12.0)) * pc;
        *c = 1.0 + (x2 * -0.5) * pc;
        return;
    }
    int k = 0;
    while (!(fabs(value(x)) <= 0.5) && k < 64) { x = 0.5 * x; ++k; }
    T x2 = x * x;
    T ps = 1.0 / 6227020800.0;
    ps = -1.0 / 39916800.0 + x2 * ps;
    ps = 1.0 / 362880.0 + x2 * ps;
    ps = -1.0 / 5040.0 + x2 * ps;
    ps = 1.0 / 120.0 + x2 * ps;
    ps = -1.0 / 6.0 + x2 * ps;
    T sn = x + (x * x2) * ps;
    T pc = -1.0 / 87178291200.0;
    pc = 1.0 / 479001600.0 + x2 * pc;
    pc = -1.0 / 3628800.0 + x2 * pc;
    pc = 1.0 / 40320.0 + x2 * pc;
    pc = -1.0 / 720.0 + x2 * pc;
    pc = 1.0 / 24.0 + x2 * pc;
    pc = -0.5 + x2 * pc;
    T cs = 1.0 + x2 * pc;
    for (; k > 0; --k) {
        T s2 = 2.0 * (sn * cs);
        T c2 = cs * cs - sn * sn;
        sn = s2;
        cs = c2;
    }
    *s = sn;
    *c = cs;
}

// Rotation phase of the magnetic axis relative to a reference time t0 at which
// (cos, sin)(Omega t0) = (c0, s0) are known; the tracing kernels keep the
// reference at the start of the current step, so the per-stage angle is small.
struct AxisRef {
    double t0, c0, s0;
};

// reference phase at time t (angle reduced to [-pi, pi] first)
template <class T>
RT_HD AxisRef axis_ref_at(const InstT<T>& I, double t) {
    AxisRef r;
    r.t0 = t;
    double x = value(I.Om) * t;
    x -= 6.283185307179586 * rint(x * 0.15915494309189535);
    double s, c;
    small_angle_sincos(x, &s, &c);
    r.c0 = c;
    r.s0 = s;
    return r;
}

// move the reference to time t (rotation by the small step angle, renormalised)
template <class T>
RT_HD void axis_ref_advance(const InstT<T>& I, AxisRef& r, double t) {
    double sd, cd;
    small_angle_sincos(value(I.Om) * (t - r.t0), &sd, &cd);
    double c = r.c0 * cd - r.s0 * sd;
    double s = r.s0 * cd + r.c0 * sd;
    double nrm = frsqrt(c * c + s * s);
    r.c0 = c * nrm;
    r.s0 = s * nrm;
    r.t0 = t;
}

// magnetic axis m(t) and its time derivative
template <class T>
RT_HD void magnetic_axis(const InstT<T>& I, const T& t, T m[3], T mt[3], const AxisRef* ref = nullptr) {
    if (I.oblique) {
        T s, c;
        if (ref != nullptr) {
            T sd, cd;
            small_angle_sincos(I.Om * (t - ref->t0), &sd, &cd);
            c = ref->c0 * cd - ref->s0 * sd;
            s = ref->s0 * cd + ref->c0 * sd;
        } else {
            sincos_t(I.Om * t, &s, &c);
        }
        m[0] = I.sm * c; m[1] = I.sm * s; m[2] = I.cm;
        T w;
        if constexpr (std::is_same<T, double>::value)
            w = I.Omsm;
        else
            w = I.Om * I.sm;
        mt[0] = -(w * s); mt[1] = w * c; mt[2] = T(0.0);
    } else {
        m[0] = T(0.0); m[1] = T(0.0); m[2] = I.cm;
        mt[0] = T(0.0); mt[1] = T(0.0); mt[2] = T(0.0);
    }
}

// n = unit position, ir = 1/r, m = axis, mu = m.n, dmu = dm/dt . n.  gjs (GJ density only):
// 0 = the density D3 |g| itself; +1 or -1 = its smooth piece D3 gjs g, which forward
// tracing integrates between crossings of the null surface g = 0.
template <class T>
RT_HD Plasma<T> plasma_eval(const InstT<T>& I, const T n[3], const T& ir, const T m[3], const T& mu,
                            const T& dmu, double gjs = 0.0) {
    Plasma<T> p;
    if (I.density == DEN_NONE) {
        p.P = T(0.0); p.pn = T(0.0); p.pm = T(0.0); p.pz = T(0.0); p.pt = T(0.0); p.g = T(0.0);
        return p;
    }
    T ir3 = ir * ir * ir;
    // Cwp (R/r)^3 = (Cwp R^3) r^-3; in dual numbers grouped so that no product of two star
    // constants is formed (the derivatives by Cwp flow through it)
    T D3;
    if constexpr (std::is_same<T, double>::value)
        D3 = I.CwpR3 * ir3;
    else
        D3 = I.Cwp * (I.R3 * ir3);
    p.g = T(0.0);
    if (I.density == DEN_GJ) {
        // P = D3 |g|, g = 3 n_z mu - cos(theta_m); with a = 3 sign(g),
        // grad P = (D3/r) [a (n_z m + mu e_z) - (2 a n_z mu + 3 |g|) n],  dP/dt = D3 a n_z dmu
        T g = 3.0 * n[2] * mu - I.cm;
        p.g = g;
        double sg = (gjs != 0.0) ? gjs : ((value(g) < 0.0) ? -1.0 : 1.0);
        T ag = sg * g;
        p.P = D3 * ag;
        T c = D3 * ir;
        T ca = (3.0 * sg) * c;
        T nzmu = n[2] * mu;
        p.pn = T(0.0) - (2.0 * ca * nzmu + 3.0 * c * ag);
        p.pm = ca * n[2];
        p.pz = ca * mu;
        p.pt = ((3.0 * sg) * D3) * (n[2] * dmu);
    } else if (I.density == DEN_MAG) {
        // P = D3 (1 - mu^2) / r; grad P = (D3/r^2)(-4 (1 - mu^2) n - 2 mu (m - mu n))
        T s2 = 1.0 - mu * mu;
        T D4 = D3 * ir;
        p.P = D4 * s2;
        T c = D4 * ir;
        p.pn = T(0.0) - c * (4.0 * s2 - 2.0 * mu * mu);
        p.pm = (-2.0 * c) * mu;
        p.pz = T(0.0);
        p.pt = (-2.0 * D4) * (mu * dmu);
    } else {
        // spherical test profile P = D3
        p.P = D3;
        p.pn = -3.0 * D3 * ir;
        p.pm = T(0.0);
        p.pz = T(0.0);
        p.pt = T(0.0);
    }
    return p;
}

// ----------------------------------------------------------------------------
// gradient of H: g = (dH/dx, dH/dy, dH/dz, dH/dt, dH/dk_x, dH/dk_y, dH/dk_z, dH/dk_t)
// ----------------------------------------------------------------------------
template <class T>
RT_HD void grad_h(const InstT<T>& I, const T y[8], T g[8], const AxisRef* ref = nullptr, double gjs = 0.0,
                  T* gfac = nullptr) {
    const T& kx = y[4]; const T& ky = y[5]; const T& kz = y[6]; const T& kt = y[7];
    T r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    T ir = frsqrt(r2);
    T n[3] = {y[0] * ir, y[1] * ir, y[2] * ir};
    T s = I.rs * ir;
    T A = 1.0 - s;
    // 1/sqrt(A) serves the anisotropic term; 1/A follows from it
    const bool aniso = (I.plasma == PL_ANISO) && (I.density != DEN_NONE);
    T ia = aniso ? frsqrt(A) : T(0.0);
    T iA = aniso ? ia * ia : frcp(A);
    T q = n[0] * kx + n[1] * ky + n[2] * kz;
    T sr = s * ir;
    // vacuum: dH/dk = 2k - 2 s q n; dH/dk_t = -2 k_t / A;
    //         dH/dx = (s/r) [(k_t^2/A^2 + 3 q^2) n - 2 q k]
    // Each spatial part is assembled below as Cn n + Cm m + Ck k (+ Cz e_z).
    T kti = kt * iA;
    T q3 = 3.0 * q;
    T kn = -2.0 * s * q;                    // n coefficient of dH/dk
    T Cn = sr * (kti * kti + q3 * q);       // n coefficient of dH/dx
    T Ck = kn * ir;                         // k coefficient of dH/dx (-2 s q / r)
    g[7] = -2.0 * kti;
    if (I.density == DEN_NONE) {
        for (int i = 0; i < 3; ++i) {
            g[4 + i] = kn * n[i] + 2.0 * y[4 + i];
            g[i] = Cn * n[i] + Ck * y[4 + i];
        }
        g[3] = T(0.0);
        return;
    }

    T m[3], mt[3];
    magnetic_axis(I, y[3], m, mt, ref);
    T mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
    // dm/dt = Omega e_z x m, so (dm/dt).v = Omega (m_x v_y - m_y v_x)
    T dmu = I.oblique ? I.Om * (m[0] * n[1] - m[1] * n[0]) : T(0.0);
    Plasma<T> p = plasma_eval(I, n, ir, m, mu, dmu, gjs);
    if (gfac) *gfac = p.g;  // the same bits as gj_factor at y
    if (I.plasma == PL_ISO) {
        const T Cn2 = Cn + p.pn;
        for (int i = 0; i < 3; ++i) {
            g[4 + i] = kn * n[i] + 2.0 * y[4 + i];
            g[i] = Cn2 * n[i] + p.pm * m[i] + Ck * y[4 + i];
        }
        g[2] = g[2] + p.pz;
        g[3] = p.pt;
        return;
    }
    // anisotropic (strong-B LO mode): H += P (1 - K), K = A N^2 / (k_t^2 (1 + c mu^2)),
    // N = (static-frame k).(g mu n - m) = b mu q - m.k with b = 1 + (g - 1) sqrt(A)
    // (flat dipole: g = c = 3)
    T a = A * ia;
    DipoleShape<T> sh;
    if (I.gr_dipole) sh = dipole_shape(I, ir);
    T b = I.gr_dipole ? 1.0 + (sh.g - 1.0) * a : 1.0 + 2.0 * a;
    T mk = m[0] * kx + m[1] * ky + m[2] * kz;
    T bmu = b * mu;
    T muq = mu * q;
    T Nn = b * muq - mk;
    T cc = I.gr_dipole ? sh.c : T(3.0);
    T den = frcp(1.0 + cc * mu * mu);
    T ikt = frcp(kt);
    T Nd = Nn * (ikt * ikt) * den;  // N / (k_t^2 (1 + c mu^2))
    T N2d = Nn * Nd;                // N^2 / (k_t^2 (1 + c mu^2))
    T K = A * N2d;
    T c1 = 2.0 * A * Nd;            // dK/dN
    // dK/dk = c1 (b mu n - m);  dK/dk_t = -2 K / k_t
    T PK = p.P * c1;
    T kn2 = kn - PK * bmu;
    for (int i = 0; i < 3; ++i) g[4 + i] = kn2 * n[i] + (PK * m[i] + 2.0 * y[4 + i]);
    g[7] = g[7] + 2.0 * p.P * K * ikt;
    // dK/dx = e_n n + e_m m + e_k k with
    //   dN/dx = mu q (db/dr) n + b [q (m - mu n) + mu (k - q n)] / r   (flat: db/dr = s / (sqrt(A) r))
    //   dD/dx = c' mu^2 n + 2 c mu (m - mu n) / r,  D = 1 + c mu^2
    //   dK/dx = N2d (s/r) n + c1 dN/dx - K den dD/dx
    T cbi = c1 * b * ir;
    T e_k = cbi * mu;
    T KDt = 2.0 * cc * K * den * mu;  // 2 c K mu den
    T KD = KDt * ir;                  // 2 c K mu den / r
    T e_m = cbi * q - KD;
    T e_n;
    if (I.gr_dipole) {
        T dbdr = sh.dg * a + (sh.g - 1.0) * (0.5 * s * ir * ia);
        e_n = N2d * sr + muq * (c1 * dbdr - 2.0 * cbi) + KD * mu - K * den * sh.dc * mu * mu;
    } else {
        e_n = N2d * sr + muq * (c1 * (sr * ia) - 2.0 * cbi) + KD * mu;
    }
    // dH/dx = vacuum + (1 - K) grad P - P dK/dx
    T omK = 1.0 - K;
    T Cn2 = Cn + (omK * p.pn - p.P * e_n);
    T Cm = omK * p.pm - p.P * e_m;
    T Ck2 = Ck - p.P * e_k;
    for (int i = 0; i < 3; ++i) g[i] = Cn2 * n[i] + (Cm * m[i] + Ck2 * y[4 + i]);
    g[2] = g[2] + omK * p.pz;
    // time: dN/dt = b q dmu - mt.k ; dK/dt = c1 dN/dt - 2 c K mu den dmu
    g[3] = T(0.0);
    if (I.oblique) {
        T mtk = I.Om * (m[0] * ky - m[1] * kx);
        T dKdt = c1 * (b * q * dmu - mtk) - KDt * dmu;
        g[3] = omK * p.pt - p.P * dKdt;
    }
    if (I.larmor) {
        // finite magnetisation (Sec. 4.1 eq. (DisRel) over w_L^2 w^2 k^2): H += C with
        //   C = -a Q^2 / (L k2),  k2 = H_vac, a = w^2 - P, Q = k2 + P, L = (w_L / w_inf)^2,
        //   dC = al da + be dQ - C dlog(L) + de dk2,  al = -Q^2/(L k2), be = -2 a Q/(L k2), de = -C/k2,
        // with da = d(w^2) - dP, dQ = dk2 + dP and dk2 the vacuum gradient (Cn n + Ck k,
        // kn n + 2 k, -2 k_t/A); dlog L = (-6/r + 2 F'/F + c' mu^2/D) n + 2 c mu (m - mu n)/(r D),
        // D = 1 + c mu^2, and 2 c mu dmu / D in time
        const T kk = kx * kx + ky * ky + kz * kz;
        const T w2 = kt * kti;
        const T k2 = kk - s * q * q - w2;
        const T av = w2 - p.P;
        const T Qv = k2 + p.P;
        const T ir2 = ir * ir;
        const T Fb2 = I.gr_dipole ? sh.F * sh.F : T(1.0);
        const T L = I.kL * (ir2 * ir2 * ir2) * Fb2 * (1.0 + cc * mu * mu);
        const T iLk = frcp(L * k2);
        const T C = (0.0 - av) * Qv * Qv * iLk;
        const T al = (0.0 - Qv) * Qv * iLk;
        const T be = -2.0 * av * Qv * iLk;
        const T de = (0.0 - C) * L * iLk;
        const T bd = be + de;   // coefficient of the vacuum gradient
        const T bma = be - al;  // coefficient of grad P
        const T lm = 2.0 * cc * mu * ir * den;
        T ln = -6.0 * ir - lm * mu;
        if (I.gr_dipole) ln = ln + 2.0 * sh.dF * rcp(sh.F) + sh.dc * mu * mu * den;
        const T xn = bd * Cn - al * (kti * kti) * sr + bma * p.pn - C * ln;
        const T xm = bma * p.pm - C * lm;
        const T xk = bd * Ck;
        const T kn3 = bd * kn;
        const T k2c = 2.0 * bd;
        for (int i = 0; i < 3; ++i) {
            g[i] = g[i] + (xn * n[i] + (xm * m[i] + xk * y[4 + i]));
            g[4 + i] = g[4 + i] + (kn3 * n[i] + k2c * y[4 + i]);
        }
        g[2] = g[2] + bma * p.pz;
        g[7] = g[7] + 2.0 * kti * (al - bd);
        if (I.oblique) g[3] = g[3] + (bma * p.pt - C * (2.0 * cc * mu * dmu * den));
    }
}

// Hamilton's equations, eq. (Hamilton); sign = -1 integrates backwards in the worldline parameter.
// gjs selects the piece of the GJ density (see plasma_eval); *gfac, if given, receives the GJ
// factor at y for a density with one (left as it was for the others).
template <class T>
RT_HD void rhs(const InstT<T>& I, const T y[8], T f[8], double sign, const AxisRef* ref = nullptr,
               double gjs = 0.0, T* gfac = nullptr) {
    T g[8];
    grad_h(I, y, g, ref, gjs, gfac);
    for (int i = 0; i < 4; ++i) {
        f[i] = sign * g[4 + i];
        f[4 + i] = -sign * g[i];
    }
}

// H itself (health checks and the backward event function)
template <class T>
RT_HD T hamiltonian(const InstT<T>& I, const T y[8], const AxisRef* ref = nullptr) {
    T r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    T r = sqrt(r2);
    T ir = rcp(r);
    T n[3] = {y[0] * ir, y[1] * ir, y[2] * ir};
    T s = I.rs * ir;
    T A = 1.0 - s;
    T q = n[0] * y[4] + n[1] * y[5] + n[2] * y[6];
    T kk = y[4] * y[4] + y[5] * y[5] + y[6] * y[6];
    T Hv = -(y[7] * y[7]) * rcp(A) + kk - s * q * q;
    if (I.density == DEN_NONE) return Hv;
    T m[3], mt[3];
    magnetic_axis(I, y[3], m, mt, ref);
    T mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
    T dmu = T(0.0);
    Plasma<T> p = plasma_eval(I, n, ir, m, mu, dmu);
    if (I.plasma == PL_ISO) return Hv + p.P;
    T a = sqrt(A);
    DipoleShape<T> sh;
    if (I.gr_dipole) sh = dipole_shape(I, ir);
    T mk = m[0] * y[4] + m[1] * y[5] + m[2] * y[6];
    T Nn = (I.gr_dipole ? 1.0 + (sh.g - 1.0) * a : 1.0 + 2.0 * a) * mu * q - mk;
    const T Dsh = 1.0 + (I.gr_dipole ? sh.c : T(3.0)) * mu * mu;
    T K = A * Nn * Nn * rcp(y[7] * y[7] * Dsh);
    T H = Hv + p.P * (1.0 - K);
    if (I.larmor) {
        // finite magnetisation: - (w^2 - P) (Hv + P)^2 / (L Hv), L = (w_L / w_inf)^2
        const T ir2 = ir * ir;
        const T L = I.kL * (ir2 * ir2 * ir2) * (I.gr_dipole ? sh.F * sh.F : T(1.0)) * Dsh;
        const T Qv = Hv + p.P;
        H = H - (y[7] * y[7] * rcp(A) - p.P) * Qv * Qv * rcp(L * Hv);
    }
    return H;
}

// g^{mu nu} k_mu k_nu (vacuum part of H)
template <class T>
RT_HD T g_kk(const InstT<T>& I, const T y[8]) {
    T ir = frsqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    T s = I.rs * ir;
    T q = (y[0] * y[4] + y[1] * y[5] + y[2] * y[6]) * ir;
    T kk = y[4] * y[4] + y[5] * y[5] + y[6] * y[6];
    return -(y[7] * y[7]) * frcp(1.0 - s) + kk - s * q * q;
}

// The GJ factor g = 3 n_z (m.n) - cos(theta_m) at the state y (the density is
// proportional to |g|; the null surface is g = 0)
template <class T>
RT_HD double gj_factor(const InstT<T>& I, const double y[8], const AxisRef* ref = nullptr) {
    const double ir = frsqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    const double n[3] = {y[0] * ir, y[1] * ir, y[2] * ir};
    double m[3], mt[3];
    magnetic_axis(I, y[3], m, mt, ref);
    return 3.0 * n[2] * (m[0] * n[0] + m[1] * n[1] + m[2] * n[2]) - value(I.cm);
}

// dipole field direction u = 3 mu n - m (|u|^2 = 1 + 3 mu^2) and magnitude factor
template <class T>
RT_HD void dipole_dir(const T n[3], const T m[3], const T& mu, T u[3], const T& g = T(3.0)) {
    for (int i = 0; i < 3; ++i) u[i] = g * mu * n[i] - m[i];
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al. 2011)
// ----------------------------------------------------------------------------
RT_HD void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                         uint32_t out[4]) {
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// 52 random bits -> (m + 1/2) 2^-52 in (0, 1)
RT_HD double unit_from_bits(uint32_t hi, uint32_t lo) {
    uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)m + 0.5) * 2.220446049250313e-16;
}

}  // namespace rtd
