// Test-only host build of the library's backward event weight
// (paper_2309_08655_amd/csrc/rt_seed.hpp, event_weight), so the CPU test suite can
// compare it with the oracle's on the same events without a GPU.  Not part of the library.
#include <cmath>

#include "../paper_2309_08655_amd/csrc/rt_seed.hpp"

using namespace rtd;

extern "C" {
// p = (B0, P, theta_m, M, R, m_a); fd = (g_agg, v0, rho, multiplicity, psi, B_test);
// fi = (plasma, density, weights, kdir, speeds, flags)
double host_event_weight(const double* p, const double* fd, const int* fi, const double* y, double Lc_max,
                         double* Lc) {
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
    SeedT<double> C = make_seed_t<double>(p, fx);
    return event_weight(I, C, y, Lc_max, Lc);
}

// cyclotron depth of one escaped ray from its final state f[16] and emission radius
double host_cyclotron_tau(const double* p, const double* fd, const int* fi, const double* f, double r_emit,
                          double* r_res) {
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
    SeedT<double> C = make_seed_t<double>(p, fx);
    return cyclotron_tau(I, C, f[8], f[9], f[3], f[14], f[11], r_emit, r_res);
}
}
