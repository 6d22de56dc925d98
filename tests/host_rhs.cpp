// Test-only host build of the device templates (hand-derived gradient of H and
// one DOPRI5 attempt), so that the CPU test suite can compare them with the
// oracle without a GPU.  Not part of the library.
#include <cmath>

#include "../paper_2309_08655_amd/csrc/rt_device.hpp"
#include "../paper_2309_08655_amd/csrc/rt_integrator.hpp"

using namespace rtd;

static InstT<double> inst_from(const double* c, const int* e) {
    InstT<double> I;
    I.rs = c[0]; I.R = c[1]; I.Om = c[2]; I.cm = c[3]; I.sm = c[4]; I.Cwp = c[5]; I.R3 = c[1] * c[1] * c[1];
    I.iOm = 1.0 / I.Om; I.Omsm = I.Om * I.sm; I.msm = -I.sm; I.CwpR3 = I.Cwp * I.R3;
    I.ma2 = c[6];
    I.plasma = e[0]; I.density = e[1]; I.oblique = (I.sm != 0.0) ? 1 : 0;
    I.gr_dipole = e[2]; I.bnorm = c[7];
    I.kL = c[8]; I.larmor = e[3];
    return I;
}

extern "C" {
// c = (rs, R, Om, cos theta_m, sin theta_m, Cwp, ma2, bnorm, kL); e = (plasma, density, gr_dipole, larmor)
void host_grad_h(const double* c, const int* e, const double* y, double* g) {
    InstT<double> I = inst_from(c, e);
    grad_h(I, y, g);
}
double host_hamiltonian(const double* c, const int* e, const double* y) {
    InstT<double> I = inst_from(c, e);
    return hamiltonian(I, y);
}
// one attempted step: returns err^2, writes ynew
double host_attempt(const double* c, const int* e, const double* y, double h, double* ynew, double rtol,
                    double atol) {
    InstT<double> I = inst_from(c, e);
    Stages S;
    auto f = [&](const double* yy, double* ff) { rhs(I, yy, ff, 1.0); };
    f(y, S.K[0]);
    return dopri_attempt(f, y, S, h, ynew, rtol, atol);
}
}

extern "C" {
// host run of the tracing loop of the persistent kernel for one ray (same decisions)
// locate = 0: the kernels' Newton locators of the r = rmax and null-surface crossings;
// 1: 60 bisections for both (the oracle's definition)
int host_trace(const double* c, const int* e, const double* y0, double rtol, double atol, double rmax,
               long long max_steps, double* yf, int* nacc_out, int* nrej_out, int locate) {
    InstT<double> I = inst_from(c, e);
    double gjs = 0.0, phi = 0.0;
    auto f = [&](const double* yy, double* ff) { rhs(I, yy, ff, 1.0, nullptr, gjs); };
    Stages S;
    double y[8], ynew[8];
    for (int d = 0; d < 8; ++d) y[d] = y0[d];
    if (I.density == DEN_GJ) {
        const double g0 = gj_factor(I, y);
        gjs = (g0 < 0.0) ? -1.0 : 1.0;
        phi = gjs * g0;
    }
    f(y, S.K[0]);
    double h = initial_step(f, y, S.K[0], rtol, atol);
    double lam = 0.0, facmax = 10.0;
    int nacc = 0, nrej = 0, status = 0;
    auto bisect = [&](auto&& inside) {  // first theta of the extension with !inside(theta)
        double lo = 0.0, hi = 1.0, yt[8];
        for (int it = 0; it < 60; ++it) {
            double mid = 0.5 * (lo + hi);
            dense_at(y, ynew, S, h, mid, yt, 0, 8);
            if (inside(yt)) lo = mid; else hi = mid;
        }
        return hi;
    };
    while (status == 0) {
        double err2 = dopri_attempt(f, y, S, h, ynew, rtol, atol);
        if (!(err2 <= 1.0)) {
            ++nrej;
            h *= step_factor(err2, facmax, false);
            facmax = 1.0;
            if (!(fabs(h) >= 1e-14 * (1.0 + fabs(lam)))) status = 5;
            continue;
        }
        ++nacc;
        double rnew = sqrt(ynew[0] * ynew[0] + ynew[1] * ynew[1] + ynew[2] * ynew[2]);
        if (rnew <= I.R) { status = 2; for (int d = 0; d < 8; ++d) yf[d] = ynew[d]; break; }
        double g1 = 0.0, thk = 2.0;
        bool cross = false;
        if (I.density == DEN_GJ) {
            g1 = gj_factor(I, ynew);
            cross = gjs * g1 < 0.0;
        }
        double phik = 0.0;
        if (cross) {
            if (locate == 0) {
                thk = locate_null_crossing(I, y, ynew, S, h, gjs, phi, gjs * g1, nullptr, &phik);
            } else {
                thk = bisect([&](const double* yt) { return gjs * gj_factor(I, yt) > 0.0; });
                double yt[8];
                dense_at(y, ynew, S, h, thk, yt, 0, 8);
                phik = gjs * gj_factor(I, yt);
            }
        }
        if (rnew >= rmax) {
            double th = (locate == 0) ? locate_crossing(y, ynew, S, h, rmax) : bisect([&](const double* yt) {
                return sqrt(yt[0] * yt[0] + yt[1] * yt[1] + yt[2] * yt[2]) < rmax;
            });
            if (th <= thk) {
                dense_at(y, ynew, S, h, th, yf, 0, 8);
                status = 1;
                break;
            }
        }
        if (cross) {
            double yt[8];
            dense_at(y, ynew, S, h, thk, yt, 0, 8);
            for (int d = 0; d < 8; ++d) y[d] = yt[d];
            lam += thk * h;
            gjs = -gjs;
            phi = -phik;
            f(y, S.K[0]);
        } else {
            lam += h;
            for (int d = 0; d < 8; ++d) { y[d] = ynew[d]; S.K[0][d] = S.K[6][d]; }
            phi = gjs * g1;
        }
        h *= step_factor(err2, facmax, true);
        facmax = 10.0;
        if (nacc >= max_steps) status = 4;
    }
    *nacc_out = nacc; *nrej_out = nrej;
    return status;
}
}

extern "C" {
// the controller's err^(-1/5) = err2^(-1/10) and step factor, from err2 = err^2
double host_inv_tenth_root(double err2) { return inv_tenth_root(err2); }
double host_step_factor(double err2, double facmax, int accepted) { return step_factor(err2, facmax, accepted != 0); }
}

#include "../paper_2309_08655_amd/csrc/rt_seed.hpp"

extern "C" {
// root of F along the radial line through n (the seeding's search, and a plain bisection on
// the same bracket for comparison); d = (mu, cB2) as the seeding forms them from n, m, kh
double host_resonance_radius(const double* c, const int* e, const double* n, const double* m, const double* kh,
                             double om2, int thin, int bisect, int* nevals) {
    InstT<double> I = inst_from(c, e);
    double mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
    double ku = 0.0;
    for (int d = 0; d < 3; ++d) ku += kh[d] * (3.0 * mu * n[d] - m[d]);
    const double cB2 = ku * ku / (1.0 + 3.0 * mu * mu);
    if (!bisect) return resonance_radius(I, n, m, mu, cB2, om2, thin != 0, kh, nevals);
    auto F = [&](double r) { return resonance_line(I, n, m, mu, cB2, om2, thin != 0, r, kh); };
    int ne = 1;
    const double R = I.R;
    if (!(F(R) > 0.0)) { *nevals = ne; return -1.0; }
    double lo = R, hi = 2.0 * R;
    int j = 0;
    while (!(F(hi) < 0.0) && j < 80) { lo = hi; hi *= 2.0; ++j; ++ne; }
    ++ne;
    if (!(F(hi) < 0.0)) { *nevals = ne; return -1.0; }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        ++ne;
        if (F(mid) > 0.0) lo = mid; else hi = mid;
    }
    *nevals = ne;
    return 0.5 * (lo + hi);
}
}
