// Static FP64 operation count of the tracer's arithmetic, obtained by running
// the device templates (gradient of H, one DOPRI5 attempt, the adjoint's stage
// products in dual numbers) on the host with a counting scalar.
// Convention: +, -, x each 1; fused multiply-add 2; division, reciprocal,
// square root, pow 1 each; sin and cos 1 each; negation, |.|, max/min,
// comparisons 0.  Prints one JSON object keyed by the physics variant.
#include <cmath>
#include <cstdio>

static long long g_flops = 0;

struct FC {
    double v;
    FC() : v(0.0) {}
    FC(double x) : v(x) {}
};
inline FC operator+(FC a, FC b) { ++g_flops; return FC(a.v + b.v); }
inline FC operator-(FC a, FC b) { ++g_flops; return FC(a.v - b.v); }
inline FC operator*(FC a, FC b) { ++g_flops; return FC(a.v * b.v); }
inline FC operator/(FC a, FC b) { ++g_flops; return FC(a.v / b.v); }
inline FC operator+(double a, FC b) { ++g_flops; return FC(a + b.v); }
inline FC operator+(FC a, double b) { ++g_flops; return FC(a.v + b); }
inline FC operator-(double a, FC b) { ++g_flops; return FC(a - b.v); }
inline FC operator-(FC a, double b) { ++g_flops; return FC(a.v - b); }
inline FC operator*(double a, FC b) { ++g_flops; return FC(a * b.v); }
inline FC operator*(FC a, double b) { ++g_flops; return FC(a.v * b); }
inline FC operator/(FC a, double b) { ++g_flops; return FC(a.v / b); }
inline FC operator/(double a, FC b) { ++g_flops; return FC(a / b.v); }
inline FC operator-(FC a) { return FC(-a.v); }
inline FC sqrt(FC a) { ++g_flops; return FC(std::sqrt(a.v)); }
inline FC rcp(FC a) { ++g_flops; return FC(1.0 / a.v); }
inline FC frcp(FC a) { ++g_flops; return FC(1.0 / a.v); }
inline FC frcp_coarse(FC a) { ++g_flops; return FC(1.0 / a.v); }
inline FC frsqrt(FC a) { ++g_flops; return FC(1.0 / std::sqrt(a.v)); }
inline FC log1p_t(FC a) { ++g_flops; return FC(std::log1p(a.v)); }
inline FC fabs(FC a) { return FC(std::fabs(a.v)); }
inline FC fmax(FC a, FC b) { return FC(std::fmax(a.v, b.v)); }
inline void sincos_t(FC a, FC* s, FC* c) { g_flops += 2; s->v = std::sin(a.v); c->v = std::cos(a.v); }
inline double value(FC a) { return a.v; }
inline bool finite_value(FC a) { return std::isfinite(a.v); }

#include "rt_adjoint.hpp"

using namespace rtd;

static InstT<FC> inst(int plasma, int density, bool oblique) {
    InstT<FC> I;
    I.rs = FC(4.13); I.R = FC(10.0); I.Om = FC(2e-5); I.cm = FC(oblique ? 0.95 : 1.0);
    I.sm = FC(oblique ? 0.3 : 0.0); I.Cwp = FC(1.0); I.R3 = FC(1000.0); I.ma2 = FC(0.99);
    I.iOm = FC(1.0 / I.Om.v); I.Omsm = FC(I.Om.v * I.sm.v); I.msm = FC(-I.sm.v); I.CwpR3 = FC(I.Cwp.v * I.R3.v);
    I.plasma = plasma; I.density = density; I.oblique = oblique ? 1 : 0;
    I.gr_dipole = 0; I.bnorm = FC(1.0); I.larmor = 0; I.kL = FC(0.0);
    return I;
}

int main() {
    const char* pn[2] = {"iso", "aniso"};
    const char* dn[4] = {"gj", "magnetar", "spherical", "none"};
    std::printf("{");
    bool first = true;
    for (int pl = 0; pl < 2; ++pl)
        for (int de = 0; de < 4; ++de)
            for (int ob = 0; ob < 2; ++ob) {
                InstT<FC> I = inst(pl, de, ob != 0);
                FC y[8] = {FC(20.0), FC(5.0), FC(7.0), FC(100.0), FC(0.3), FC(0.2), FC(0.1), FC(-1.0)};
                FC f[8];
                g_flops = 0;
                rhs(I, y, f, 1.0);
                long long frhs = g_flops;
                StagesT<FC> S;
                for (int d = 0; d < 8; ++d) S.K[0][d] = f[d];
                FC ynew[8];
                g_flops = 0;
                auto fn = [&](const FC* yy, FC* ff) { rhs(I, yy, ff, 1.0); };
                dopri_attempt(fn, y, S, FC(0.1), ynew, 1e-8, 1e-12);
                long long fstep = g_flops + 3;  // + step-size update (pow, x0.9, x h)
                // the stages alone (the reverse sweep's recompute of an accepted step: no error
                // estimate, no controller), in the order the adjoint computes them
                long long fstages_only = 0;
                {
                    using namespace dp5;
                    const double A[6][6] = {{a21, 0, 0, 0, 0, 0},       {a31, a32, 0, 0, 0, 0},
                                            {a41, a42, a43, 0, 0, 0},   {a51, a52, a53, a54, 0, 0},
                                            {a61, a62, a63, a64, a65, 0}, {b1, 0.0, b3, b4, b5, b6}};
                    FC Kq[7][8], tmp[8];
                    for (int d = 0; d < 8; ++d) Kq[0][d] = f[d];
                    g_flops = 0;
                    for (int st = 0; st < 6; ++st) {
                        for (int d = 0; d < 8; ++d) {
                            FC acc(0.0);
                            for (int q = 0; q <= st; ++q) acc = acc + A[st][q] * Kq[q][d];
                            tmp[d] = y[d] + FC(0.1) * acc;
                        }
                        rhs(I, tmp, Kq[st + 1], 1.0);
                    }
                    fstages_only = g_flops;
                }
                // adjoint: one stage vector-Jacobian product (a 1-tangent dual-number
                // Hessian-vector product, a 3-tangent pass for the parameter channels and the
                // vacuum part) and the reverse sweep through the six stages of a plain step
                FC v[8], vy[8], vc[5], rows[LR_SLOTS], yb[8], tc[5];
                for (int d = 0; d < 8; ++d) { v[d] = FC(0.1 * (d + 1)); yb[d] = FC(0.0); }
                for (int d = 0; d < LR_SLOTS; ++d) rows[d] = y[d % 8];
                for (int d = 0; d < 8; ++d) rows[8 * LR_YNB + d] = FC(0.01 * d);
                for (int q = 0; q < 5; ++q) tc[q] = FC(0.0);
                g_flops = 0;
                stage_vjp<false, FC>(I, y, v, vy, vc);
                long long fvjp = g_flops;
                g_flops = 0;
                step_adjoint<false, false, FC>(I, ynew, FC(0.1), false, yb, tc,
                                        [&](int r) { return LaneRow<FC, 1>{rows + 8 * r}; }, 0.0);
                long long fstages = g_flops;
                // backward events: one probe of G = g^{mu nu} k k + m^2 on the continuous extension
                FC yt[8];
                for (int d = 0; d < 8; ++d) S.K[6][d] = S.K[0][d];
                g_flops = 0;
                dense_at(y, ynew, S, FC(0.1), FC(0.5), yt, 0, 8);
                FC G = g_kk(I, yt) + I.ma2;
                (void)G;
                long long fprobe = g_flops;
                // the same event function at a step's end point (no continuous extension)
                g_flops = 0;
                FC G1 = g_kk(I, ynew) + I.ma2;
                (void)G1;
                long long fendpt = g_flops;
                std::printf("%s\"%s_%s_%s\": {\"rhs\": %lld, \"attempt\": %lld, \"stages\": %lld, \"vjp\": %lld, "
                            "\"stages_adjoint\": %lld, \"event_probe\": %lld, \"event_g\": %lld}",
                            first ? "" : ", ", pn[pl], dn[de], ob ? "oblique" : "aligned", frhs, fstep, fstages_only,
                            fvjp, fstages, fprobe, fendpt);
                first = false;
            }
    std::printf("}\n");
    return 0;
}
