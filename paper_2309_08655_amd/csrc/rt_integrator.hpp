// Dormand-Prince 5(4) step with FSAL, its error norm and its continuous
// extension, one ray per lane in registers (FP64).
//
// Tableau: Dormand & Prince (1980).  Error norm, step-size controller, starting
// step and 4th-order continuous extension: Hairer, Norsett & Wanner, "Solving
// Ordinary Differential Equations I", Sec. II.4-II.6.
#pragma once

#include "rt_device.hpp"

namespace rtd {
namespace dp5 {
constexpr double a21 = 1.0 / 5;
constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                 a65 = -5103.0 / 18656;
constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784, b6 = 11.0 / 84;
constexpr double e1 = 71.0 / 57600, e3 = -71.0 / 16695, e4 = 71.0 / 1920, e5 = -17253.0 / 339200,
                 e6 = 22.0 / 525, e7 = -1.0 / 40;
constexpr double d1 = -12715105075.0 / 11282082432.0, d3 = 87487479700.0 / 32700410799.0,
                 d4 = -10690763975.0 / 1880347072.0, d5 = 701980252875.0 / 199316789632.0,
                 d6 = -1453857185.0 / 822651844.0, d7 = 69997945.0 / 29380423.0;
}  // namespace dp5

// tolerances and limits of one trace in integrator units (km)
struct TolC {
    double rtol, atol, rmax;
    long long max_steps;
};

// Stage derivatives of one attempted step.  K[0] is the FSAL derivative at y.
template <class T>
struct StagesT {
    T K[7][8];
};
using Stages = StagesT<double>;

RT_HD bool finite_value(double x) { return __builtin_isfinite(x); }

// One attempted step of length h from y with K[0] = f(y) already set.
// Fills K[1..6], ynew, and returns the square of the RMS error ratio (not yet checked;
// the step is accepted when it is <= 1, and non-finite values arrive as 1e300).
template <class T, class RHS>
RT_HD T dopri_attempt(RHS&& f, const T y[8], StagesT<T>& S, T h, T ynew[8], double rtol, double atol) {
    using namespace dp5;
    // h folded into the tableau once per attempt: each stage state is then an FMA chain
    const T h21 = h * a21, h31 = h * a31, h32 = h * a32, h41 = h * a41, h42 = h * a42, h43 = h * a43;
    const T h51 = h * a51, h52 = h * a52, h53 = h * a53, h54 = h * a54;
    const T h61 = h * a61, h62 = h * a62, h63 = h * a63, h64 = h * a64, h65 = h * a65;
    const T hb1 = h * b1, hb3 = h * b3, hb4 = h * b4, hb5 = h * b5, hb6 = h * b6;
    T tmp[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) tmp[i] = y[i] + h21 * S.K[0][i];
    f(tmp, S.K[1]);
#pragma unroll
    for (int i = 0; i < 8; ++i) tmp[i] = y[i] + h31 * S.K[0][i] + h32 * S.K[1][i];
    f(tmp, S.K[2]);
#pragma unroll
    for (int i = 0; i < 8; ++i) tmp[i] = y[i] + h41 * S.K[0][i] + h42 * S.K[1][i] + h43 * S.K[2][i];
    f(tmp, S.K[3]);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        tmp[i] = y[i] + h51 * S.K[0][i] + h52 * S.K[1][i] + h53 * S.K[2][i] + h54 * S.K[3][i];
    f(tmp, S.K[4]);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        tmp[i] = y[i] + h61 * S.K[0][i] + h62 * S.K[1][i] + h63 * S.K[2][i] + h64 * S.K[3][i] + h65 * S.K[4][i];
    f(tmp, S.K[5]);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        ynew[i] = y[i] + hb1 * S.K[0][i] + hb3 * S.K[2][i] + hb4 * S.K[3][i] + hb5 * S.K[4][i] + hb6 * S.K[5][i];
    f(ynew, S.K[6]);
    const T he1 = h * e1, he3 = h * e3, he4 = h * e4, he5 = h * e5, he6 = h * e6, he7 = h * e7;
    T acc = T(0.0);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        T e = he1 * S.K[0][i] + he3 * S.K[2][i] + he4 * S.K[3][i] + he5 * S.K[4][i] + he6 * S.K[5][i] +
              he7 * S.K[6][i];
        T sc = atol + rtol * fmax(fabs(y[i]), fabs(ynew[i]));
        T qq = e * frcp_coarse(sc);
        acc = acc + qq * qq;
    }
    T err2 = acc * 0.125;
    return finite_value(err2) ? err2 : T(1e300);
}

// Coefficients of the continuous extension of components [c0, c1) of an accepted step:
// y(theta) = y + theta (a + om (b + theta (c + om d))), om = 1 - theta.
RT_HD void dense_coeffs(const double y[8], const double ynew[8], const Stages& S, double h, int c0, int c1,
                        double* a, double* b, double* c, double* d) {
    using namespace dp5;
    for (int i = c0; i < c1; ++i) {
        const double ydiff = ynew[i] - y[i];
        const double r3 = h * S.K[0][i] - ydiff;
        const double r4 = ydiff - h * S.K[6][i] - r3;
        const double r5 = h * (d1 * S.K[0][i] + d3 * S.K[2][i] + d4 * S.K[3][i] + d5 * S.K[4][i] + d6 * S.K[5][i] +
                               d7 * S.K[6][i]);
        a[i - c0] = ydiff; b[i - c0] = r3; c[i - c0] = r4; d[i - c0] = r5;
    }
}
RT_HD double dense_value(double y, double a, double b, double c, double d, double th) {
    const double om = 1.0 - th;
    return y + th * (a + om * (b + th * (c + om * d)));
}

// Continuous extension at theta of components [c0, c1) (accepted step y -> ynew).
template <class T>
RT_HD void dense_at(const T y[8], const T ynew[8], const StagesT<T>& S, T h, T th, T out[8], int c0, int c1) {
    using namespace dp5;
    T om = 1.0 - th;
    for (int i = c0; i < c1; ++i) {
        T ydiff = ynew[i] - y[i];
        T r3 = h * S.K[0][i] - ydiff;
        T r4 = ydiff - h * S.K[6][i] - r3;
        T r5 = h * (d1 * S.K[0][i] + d3 * S.K[2][i] + d4 * S.K[3][i] + d5 * S.K[4][i] + d6 * S.K[5][i] +
                    d7 * S.K[6][i]);
        out[i] = y[i] + th * (ydiff + om * (r3 + th * (r4 + om * r5)));
    }
}

// Location theta in (0, 1] of the crossing |x(theta)| = rmax on the continuous extension
// of an accepted step that starts inside (|y| < rmax) and ends outside (|ynew| >= rmax):
// Newton's method on phi(theta) = x.x - rmax^2 from the linear interpolation of r,
// safeguarded by the bracket [lo, hi] (a step leaving it bisects instead).  Converges
// to the root to about an ulp in a few iterations, where plain bisection to the same
// precision takes 60 evaluations.
// (from the coefficients a..d of components 0..2, see dense_coeffs, and r1 = |x(1)|)
RT_HD double locate_crossing_c(const double y[3], const double a[3], const double b[3], const double c[3],
                               const double d[3], double r1, double rmax) {
    const double r0 = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    const double R2 = rmax * rmax;
    double lo = 0.0, hi = 1.0;
    double th = (r1 > r0) ? (rmax - r0) / (r1 - r0) : 1.0;
    if (!(th > 0.0 && th <= 1.0)) th = 0.5;
    for (int it = 0; it < 16; ++it) {
        const double om = 1.0 - th;
        double x2 = 0.0, xdx = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double q = b[i] + th * (c[i] + om * d[i]);
            const double p = a[i] + om * q;
            const double xi = y[i] + th * p;
            const double dxi = p + th * (-q + om * (c[i] + (1.0 - 2.0 * th) * d[i]));
            x2 += xi * xi;
            xdx += xi * dxi;
        }
        const double phi = x2 - R2;
        if (phi == 0.0) break;  // th is the root
        if (phi > 0.0) hi = th; else lo = th;
        const double step = phi / (2.0 * xdx);
        double tn = th - step;
        if (tn > lo && tn < hi) {
            if (fabs(step) <= 4.0e-16 * th) {  // converged to about an ulp
                th = tn;
                break;
            }
        } else {
            if (hi - lo <= 4.0e-16 * hi) break;  // the bracket is down to an ulp
            tn = 0.5 * (lo + hi);
        }
        th = tn;
    }
    return th;
}

RT_HD double locate_crossing(const double y[8], const double ynew[8], const Stages& S, double h, double rmax) {
    double a[3], b[3], c[3], d[3];
    dense_coeffs(y, ynew, S, h, 0, 3, a, b, c, d);
    const double r1 = sqrt(ynew[0] * ynew[0] + ynew[1] * ynew[1] + ynew[2] * ynew[2]);
    return locate_crossing_c(y, a, b, c, d, r1, rmax);
}

// Location theta of the crossing of the GJ density's null surface g = 0 on the continuous
// extension of an accepted step: phi(theta) = sg g(x(theta), t(theta)) with phi0 = phi(0) >= 0
// > phi1 = phi(1) (sg: the piece being integrated).  Newton's method from the linear
// interpolation of phi, with dphi/dtheta from the extension's derivative, safeguarded by
// the bracket [lo, hi] (a step leaving it bisects), converges to the root to about an ulp
// in a few iterations; the result is then moved forward by 1, 2, 4, ... ulp to the first
// point strictly past the surface (phi < 0), where the ray restarts on the other piece,
// so that the next step starts strictly inside it.  *phi_past = phi there.
RT_HD double locate_null_crossing_c(const InstT<double>& I, const double y[4], const double a[4], const double b[4],
                                    const double c[4], const double d[4], double sg, double phi0, double phi1,
                                    const AxisRef* ref, double* phi_past) {
    // phi and dphi/dtheta on the extension
    auto eval = [&](double th, double* dphi) {
        const double om = 1.0 - th;
        double x[4], dx[4];
        for (int i = 0; i < 4; ++i) {
            const double q = b[i] + th * (c[i] + om * d[i]);
            const double p = a[i] + om * q;
            x[i] = y[i] + th * p;
            dx[i] = p + th * (-q + om * (c[i] + (1.0 - 2.0 * th) * d[i]));
        }
        const double ir = frsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double n[3] = {x[0] * ir, x[1] * ir, x[2] * ir};
        double m[3], mt[3];
        magnetic_axis(I, x[3], m, mt, ref);
        const double mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
        const double ndx = n[0] * dx[0] + n[1] * dx[1] + n[2] * dx[2];
        double dn[3], mdn = 0.0;
        for (int i = 0; i < 3; ++i) {
            dn[i] = (dx[i] - n[i] * ndx) * ir;
            mdn += m[i] * dn[i];
        }
        const double dmu = (mt[0] * n[0] + mt[1] * n[1] + mt[2] * n[2]) * dx[3] + mdn;
        *dphi = sg * 3.0 * (dn[2] * mu + n[2] * dmu);
        return sg * (3.0 * n[2] * mu - I.cm);
    };
    double lo = 0.0, hi = 1.0, fhi = phi1;
    double th = (phi0 > 0.0 && phi1 < 0.0) ? phi0 / (phi0 - phi1) : 0.5;
    if (!(th > 0.0 && th < 1.0)) th = 0.5;
    double ph = 0.0;
    for (int it = 0; it < 24; ++it) {
        double dph;
        ph = eval(th, &dph);
        if (ph > 0.0) lo = th; else { hi = th; fhi = ph; }
        if (ph == 0.0) break;  // th is the root
        const double step = ph / dph;
        double tn = th - step;
        if (tn > lo && tn < hi) {
            if (fabs(step) <= 4.0e-16 * th) {  // converged to about an ulp
                th = tn;
                double dd;
                ph = eval(th, &dd);
                if (ph > 0.0) lo = th; else { hi = th; fhi = ph; }
                break;
            }
        } else {
            if (hi - lo <= 4.0e-16 * hi) break;  // the bracket is down to an ulp
            tn = 0.5 * (lo + hi);
        }
        th = tn;
    }
    // the first point strictly past the surface (hi is always past or on it)
    double dz = th * 0x1p-52;
    for (int k = 0; k < 64 && !(ph < 0.0); ++k) {
        double tn = th + dz;
        if (!(tn < hi)) {
            th = hi;
            ph = fhi;
            break;
        }
        double dd;
        th = tn;
        ph = eval(th, &dd);
        dz *= 2.0;
    }
    *phi_past = ph;
    return th;
}

// the same from an accepted step's stages
RT_HD double locate_null_crossing(const InstT<double>& I, const double y[8], const double ynew[8], const Stages& S,
                                  double h, double sg, double phi0, double phi1, const AxisRef* ref,
                                  double* phi_past) {
    double a[4], b[4], c[4], d[4];
    dense_coeffs(y, ynew, S, h, 0, 4, a, b, c, d);
    return locate_null_crossing_c(I, y, a, b, c, d, sg, phi0, phi1, ref, phi_past);
}

// Step-size update after an attempt (HNW I-controller, order 5), from err2 = err^2:
// accepted: h *= min(facmax, max(0.2, 0.9 err^-1/5)) (err = 0 -> facmax);
// rejected: h *= max(0.2, 0.9 err^-1/5) and facmax = 1 for the next accepted step.
// err^(-1/5) = err2^(-1/10): a single-precision estimate refined by two Newton steps in
// double on u = x^10 err2 = 1, x <- x (1 - (u - 1)/(10 u)), with 1/u replaced by 2 - u
// (u is within ~1e-6 of 1 after the estimate, so the replacement costs nothing in
// accuracy): a few ulp, no division.  err2 is clamped to [1e-30, 1e30] (single-precision
// range for the estimate), outside which the factor saturates at facmax or 0.2 anyway.
RT_HD double inv_tenth_root(double err2) {
    const double e = fmin(fmax(err2, 1e-30), 1e30);
    double x = (double)exp2f(-0.1f * log2f((float)e));
    for (int it = 0; it < 2; ++it) {
        const double x2 = x * x;
        const double x4 = x2 * x2;
        const double u = (x4 * x4) * x2 * e;
        x = x - (x * (u - 1.0)) * (0.1 * (2.0 - u));
    }
    return x;
}

RT_HD double step_factor(double err2, double facmax, bool accepted) {
    if (accepted) {
        if (err2 == 0.0) return facmax;
        return fmin(facmax, fmax(0.2, 0.9 * inv_tenth_root(err2)));
    }
    return fmax(0.2, 0.9 * inv_tenth_root(err2));
}

// Starting step (HNW Sec. II.4, order 5), norm scale atol + rtol |y0|.
template <class RHS>
RT_HD double initial_step(RHS&& f, const double y0[8], const double f0[8], double rtol,
                                               double atol) {
    double d0 = 0.0, d1 = 0.0;
    for (int i = 0; i < 8; ++i) {
        double sc = atol + rtol * fabs(y0[i]);
        d0 += (y0[i] / sc) * (y0[i] / sc);
        d1 += (f0[i] / sc) * (f0[i] / sc);
    }
    d0 = sqrt(d0 * 0.125);
    d1 = sqrt(d1 * 0.125);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    double y1[8], f1[8];
    for (int i = 0; i < 8; ++i) y1[i] = y0[i] + h0 * f0[i];
    f(y1, f1);
    double d2 = 0.0;
    for (int i = 0; i < 8; ++i) {
        double sc = atol + rtol * fabs(y0[i]);
        double qq = (f1[i] - f0[i]) / sc;
        d2 += qq * qq;
    }
    d2 = sqrt(d2 * 0.125) / h0;
    double m = fmax(d1, d2);
    double h1 = (m <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / m, 0.2);
    return fmin(100.0 * h0, h1);
}

}  // namespace rtd
