// Test-only host build of the per-ray adjoint (paper_2309_08655_amd/csrc/rt_adjoint.hpp):
// seed, forward pass with checkpoints, smoothed flux and the reverse sweep, ray by
// ray on the CPU, so the CPU test suite can compare the hand-written adjoint with
// the oracle's forward-mode derivatives without a GPU.  Not part of the library.
#include <cmath>
#include <vector>

#include "../paper_2309_08655_amd/csrc/rt_adjoint.hpp"

using namespace rtd;

extern "C" {
// p = (B0, P, theta_m, M, R, m_a); fd = (g_agg, v0, rho, multiplicity, psi, B_test);
// fi = (plasma, density, weights, kdir, speeds, flags); tl = (rtol, atol, r_max).
// Writes flux[n_obs], grad[6] = sum_j gbar_j dF_j/dp, per-ray status/n_acc and
// per-ray gradients gray[n][6]; returns the number of steps the recompute missed.
long long host_flux_grad(const double* p, const double* fd, const int* fi, const double* tl, long long max_steps,
                         unsigned long long seed, long long n, const double* obs, int n_obs, double sigma,
                         const double* gbar, int C, int Kc, double* flux, double* grad, int* status, int* nacc,
                         double* gray) {
    StarFixed fx;
    fx.g_agg_GeV = fd[0];
    fx.v0_kms = fd[1];
    fx.rho_GeVcm3 = fd[2];
    fx.multiplicity = fd[3];
    fx.psi_twist = fd[4];
    fx.B_test_G = fd[5];
    fx.plasma = fi[0];
    fx.density = fi[1];
    fx.weights = fi[2];
    fx.kdir = fi[3];
    fx.speeds = fi[4];
    fx.flags = fi[5];
    InstT<double> I = make_inst_t<double>(p, fx);
    I.oblique = 1;
    SeedT<double> Cs = make_seed_t<double>(p, fx);
    TolC tol{tl[0], tl[1], tl[2], max_steps};
    AdjParams A;
    make_adj_params(p, fx, A);
    for (int q = 0; q < n_obs; ++q) flux[q] = 0.0;
    for (int q = 0; q < 6; ++q) grad[q] = 0.0;
    long long missing = 0;
    std::vector<double> ck((size_t)Kc * 11), rbuf((size_t)C * 11), rows(LR_SLOTS);
    for (long long i = 0; i < n; ++i) {
        for (int q = 0; q < 6; ++q) gray[i * 6 + q] = 0.0;
        double seedv[10];
        int st = seed_ray<double>(I, Cs, seed, 0, i, seedv);
        nacc[i] = 0;
        if (st != ST_OK) {
            status[i] = st;
            continue;
        }
        double f0[8];
        adj_rhs(I, seedv, f0);
        auto f = [&](const double* yy, double* ff) { adj_rhs(I, yy, ff); };
        const double h0 = initial_step(f, seedv, f0, tol.rtol, tol.atol);
        auto store = [&](int s, const double* y, double h, double facmax, double gjs) {
            for (int d = 0; d < 8; ++d) ck[(size_t)s * 11 + d] = y[d];
            ck[(size_t)s * 11 + 8] = h;
            ck[(size_t)s * 11 + 9] = facmax;
            ck[(size_t)s * 11 + 10] = gjs;
        };
        AdjRay R;
        adj_ray_start(I, seedv, h0, R, store);
        double yf[8], th = 0.0;
        int s = ST_OK;
        while (s == ST_OK) s = adj_ray_step(I, tol, C, Kc, R, store, yf, &th);
        status[i] = s;
        nacc[i] = R.nacc;
        if (s != ST_ESCAPED) continue;
        double nh[3];
        arrival_direction(I, yf, nh);
        for (int o = 0; o < n_obs; ++o) {
            const double c = nh[0] * obs[3 * o] + nh[1] * obs[3 * o + 1] + nh[2] * obs[3 * o + 2];
            flux[o] += seedv[8] * smoothing_kernel(c, sigma);
        }
        auto load = [&](int sg, double* y, double* h, double* facmax, double* gjs) {
            for (int d = 0; d < 8; ++d) y[d] = ck[(size_t)sg * 11 + d];
            *h = ck[(size_t)sg * 11 + 8];
            *facmax = ck[(size_t)sg * 11 + 9];
            *gjs = ck[(size_t)sg * 11 + 10];
        };
        auto rb = [&](int idx, int d) -> double& { return rbuf[(size_t)idx * 11 + d]; };
        auto lr = [&](int r) { return LaneRow<double, 1>{rows.data() + 8 * r}; };
        double pb[6] = {0, 0, 0, 0, 0, 0};
        missing += adj_reverse_ray(I, A, tol, seed, i, R.nacc, R.nseg, th, seedv[8], C, load, rb, lr, obs, gbar, n_obs,
                                   sigma, pb);
        for (int q = 0; q < 6; ++q) {
            gray[i * 6 + q] = pb[q] / (double)n;
            grad[q] += pb[q];
        }
    }
    for (int q = 0; q < n_obs; ++q) flux[q] /= (double)n;
    for (int q = 0; q < 6; ++q) grad[q] /= (double)n;
    return missing;
}
}
