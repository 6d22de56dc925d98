// Per-ray pieces of the smoothed-flux adjoint (host and device): the step shared
// by the forward pass and the recompute, the arrival direction and smoothing
// kernel, the forward step with checkpoints, and the reverse sweep of one ray.
//
// McDonald & Witte, arXiv:2309.08655: forward estimator Sec. 2.2 eq. (Power),
// rays Sec. 2 eq. (Hamilton) with the Hamiltonian of Sec. 4.1 eq. (StrongBHam),
// seeding and weights Secs. 3-4 (rt_seed.hpp).
//
//   F_j = (1/N) sum_{escaped i} w_i K(n_i . o_j),  K(c) = exp((c - 1)/sigma^2) / (2 pi sigma^2).
//
// Differentiated map (discretise, then differentiate): accepted step sizes h_n and
// every ray's status frozen at the nominal parameters; seed root, photon momentum
// and weight by forward mode (6 tangents); the crossing r = r_max by the implicit
// function theorem on the continuous extension; every accepted step through its
// stages, y_{n+1} = y_n + h sum_i b_i K_i, K_i = f(Y_i), Y_i = y_n + h sum_{j<i} a_ij K_j.
// With f = J grad(H), J = [[0, I], [-I, 0]], the stage products are
//   v^T df/dy = Hess(H) (J^T v)   (one directional derivative of the hand-derived
//   gradient in dual numbers),    v^T df/dp from six further tangents.
#pragma once

#include "rt_integrator.hpp"
#include "rt_seed.hpp"

#define RT_HD_NOINLINE __host__ __device__ __attribute__((noinline))

namespace rtd {

typedef gdual<6> D6;
typedef gdual<14> D14;

// ----------------------------------------------------------------------------
// the step shared by the forward pass and the recompute.  The library compiles this
// file with multiply-add fusion decided per source expression only, so every copy of
// it computes the same bits and the recompute reproduces the forward pass's decisions
// and step sizes (the reverse sweep checks this at every checkpoint).
// ----------------------------------------------------------------------------
// The right-hand side must be a function of the state and the attempt alone (the
// recompute starts from checkpointed states and must reproduce every bit).  The magnetic
// axis is rotated from a reference phase: adj_rhs(I, y, f) takes it at y's own time (the
// first and last stage of an attempt, so the last stage's value serves the next attempt
// as its first, as in the forward pass), and the inner stages take the attempt's
// reference at its starting time and rotate by the small stage angle.  Both avoid a full
// sincos per evaluation.
// gjs: the piece of the GJ density being integrated (0 for the other densities; see
// plasma_eval); the adjoint follows forward tracing, which cuts steps at the null surface.
// FL = false: the star is known to take the strong-field Hamiltonian, and a local copy of the
// instance says so at compile time (its finite-magnetisation terms fold away even where the
// instance itself sits in memory behind the reverse sweep's calls).
template <bool FL = true>
RT_HD void adj_rhs(const InstT<double>& I, const double* y, double* f, const AxisRef& ref, double gjs = 0.0) {
    if constexpr (FL) {
        rhs(I, y, f, 1.0, &ref, gjs);
    } else {
        InstT<double> J = I;
        J.larmor = 0;
        rhs(J, y, f, 1.0, &ref, gjs);
    }
}
template <bool FL = true>
RT_HD void adj_rhs(const InstT<double>& I, const double* y, double* f, double gjs = 0.0) {
    const AxisRef ref = axis_ref_at(I, y[3]);
    adj_rhs<FL>(I, y, f, ref, gjs);
}

// One DOPRI5 attempt from y with K[0..7] = f(y) set; fills K[8..55] (stages 2..7,
// the last = f(ynew)) and ynew, and hands each inner stage state Y_i (i = 2..6) to
// stages(i, Y_i) (NoStages: to nobody).  Applies the step-size controller to *h and
// *facmax and returns 1 if the step is accepted.
struct NoStages {
    RT_HD void operator()(int, const double*) const {}
};

// The stages of a DOPRI5 step of size hh from y with K[0..7] = f(y) set: fills K[8..55]
// (stages 2..7, the last = f(ynew)) and ynew, and hands each inner stage state Y_i
// (i = 2..6) to stages(i, Y_i).  y is anything indexed [d] (registers, or a lane's row).
template <bool FL = true, class Sink, class YV>
RT_HD void adj_stages(const InstT<double>& I, const YV& y, double* K, double* ynew, double hh, Sink&& stages,
                      double gjs) {
    using namespace dp5;
    const double A[6][6] = {{a21, 0, 0, 0, 0, 0},
                            {a31, a32, 0, 0, 0, 0},
                            {a41, a42, a43, 0, 0, 0},
                            {a51, a52, a53, a54, 0, 0},
                            {a61, a62, a63, a64, a65, 0},
                            {b1, 0.0, b3, b4, b5, b6}};
    const AxisRef ref0 = axis_ref_at(I, y[3]);
    double tmp[8];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q <= s; ++q) acc += A[s][q] * K[q * 8 + d];
            tmp[d] = y[d] + hh * acc;
        }
        if (s < 5) {
            stages(s + 2, tmp);
        } else {
            for (int d = 0; d < 8; ++d) ynew[d] = tmp[d];
        }
        if (s < 5)
            adj_rhs<FL>(I, tmp, K + (s + 1) * 8, ref0, gjs);
        else
            adj_rhs<FL>(I, tmp, K + (s + 1) * 8, gjs);
    }
}

template <bool FL = true, class Sink>
RT_HD int adj_attempt(const InstT<double>& I, double rtol, double atol, const double* y, double* K, double* ynew,
                      double* h, double* facmax, Sink&& stages, double gjs = 0.0) {
    using namespace dp5;
    const double hh = *h;
    adj_stages<FL>(I, y, K, ynew, hh, stages, gjs);
    const double E[7] = {e1, 0.0, e3, e4, e5, e6, e7};
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        double e = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) e += E[q] * K[q * 8 + d];
        e *= hh;
        const double sc = atol + rtol * fmax(fabs(y[d]), fabs(ynew[d]));
        const double qq = e * frcp_coarse(sc);
        acc += qq * qq;
    }
    double err2 = acc * 0.125;  // the square of the RMS error ratio
    if (!__builtin_isfinite(err2)) err2 = 1e300;
    if (!(err2 <= 1.0)) {
        *h = hh * step_factor(err2, *facmax, false);
        *facmax = 1.0;
        return 0;
    }
    *h = hh * step_factor(err2, *facmax, true);
    *facmax = 10.0;
    return 1;
}

// The crossing of the GJ null surface inside an accepted step from y (K: its stages, ynew:
// its end), as forward tracing locates it: theta of the first point strictly past the
// surface, or 2 when the step stays on its piece (other densities: always 2).  A function
// of the step alone, so that the recompute reproduces it.
RT_HD double adj_null_crossing(const InstT<double>& I, const double* y, const double* K, const double* ynew, double h,
                               double gjs) {
    if (gjs == 0.0) return 2.0;
    const double g1 = gj_factor(I, ynew);
    if (!(gjs * g1 < 0.0)) return 2.0;
    Stages S;
    for (int s = 0; s < 7; ++s)
        for (int d = 0; d < 8; ++d) S.K[s][d] = K[s * 8 + d];
    double phik;
    return locate_null_crossing(I, y, ynew, S, h, gjs, gjs * gj_factor(I, y), gjs * g1, nullptr, &phik);
}

// the piece of the GJ density a ray starts on (0 for the other densities)
RT_HD double adj_start_piece(const InstT<double>& I, const double* y) {
    if (I.density != DEN_GJ) return 0.0;
    return (gj_factor(I, y) < 0.0) ? -1.0 : 1.0;
}

// Moves an accepted step's start y (stages K, size h, end ynew) to the next step's start:
// ynew, or for a crossing at thk <= 1 the point there on the continuous extension, where
// the ray goes on along the other piece (*gjs flips) with a fresh derivative in K[0..7].
template <bool FL = true>
RT_HD void adj_advance(const InstT<double>& I, double* y, double* K, const double* ynew, double h, double thk,
                       double* gjs) {
    using namespace dp5;
    if (thk <= 1.0) {
        for (int i = 0; i < 8; ++i) {
            const double ydiff = ynew[i] - y[i];
            const double r3 = h * K[i] - ydiff;
            const double r4 = ydiff - h * K[48 + i] - r3;
            const double r5 =
                h * (d1 * K[i] + d3 * K[16 + i] + d4 * K[24 + i] + d5 * K[32 + i] + d6 * K[40 + i] + d7 * K[48 + i]);
            y[i] = dense_value(y[i], ydiff, r3, r4, r5, thk);
        }
        *gjs = -*gjs;
        adj_rhs<FL>(I, y, K, *gjs);
    } else {
        for (int d = 0; d < 8; ++d) {
            y[d] = ynew[d];
            K[d] = K[48 + d];
        }
    }
}

// g = 3 n_z (m . n) - cos theta_m at y and its derivatives: gy[0..3] by (x, t), *gOm by
// Omega, *gth by theta_m (dual numbers, 6 tangents).  The star's constants come by value, so
// that the caller's instance never has its address taken (its switches stay compile-time
// constants where the caller fixes them).
RT_HD_NOINLINE void gj_factor_grad(double Om, double cm, double sm, int oblique, const double* y, double gy[4],
                                   double* gOm, double* gth) {
    typedef gdual<6, double> G6;
    G6 x[4];
    for (int i = 0; i < 4; ++i) {
        x[i] = G6(y[i]);
        x[i].d[i] = 1.0;
    }
    InstT<G6> J;
    J.Om = G6(Om);
    J.Om.d[4] = 1.0;
    J.cm = G6(cm);
    J.cm.d[5] = -sm;
    J.sm = G6(sm);
    J.sm.d[5] = cm;
    J.oblique = oblique;
    const G6 ir = rcp(sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
    const G6 n[3] = {x[0] * ir, x[1] * ir, x[2] * ir};
    G6 m[3], mt[3];
    magnetic_axis(J, x[3], m, mt);
    const G6 g = 3.0 * n[2] * (m[0] * n[0] + m[1] * n[1] + m[2] * n[2]) - J.cm;
    for (int i = 0; i < 4; ++i) gy[i] = g.d[i];
    *gOm = g.d[4];
    *gth = g.d[5];
}

// ----------------------------------------------------------------------------
// observables
// ----------------------------------------------------------------------------
// Arrival direction of Sec. 2.2: static-frame momentum at the final point,
// normalised, rotated by -Omega (t - r) about the rotation axis (frame co-rotating
// with the star at the arrival time).
template <class T>
RT_HD void arrival_direction(const InstT<T>& I, const T yf[8], T nh[3]) {
    T r = sqrt(yf[0] * yf[0] + yf[1] * yf[1] + yf[2] * yf[2]);
    T ir = rcp(r);
    T nn[3] = {yf[0] * ir, yf[1] * ir, yf[2] * ir};
    T A = 1.0 - I.rs * ir;
    T q = nn[0] * yf[4] + nn[1] * yf[5] + nn[2] * yf[6];
    T c = (sqrt(A) - 1.0) * q;
    T v[3] = {yf[4] + c * nn[0], yf[5] + c * nn[1], yf[6] + c * nn[2]};
    T vn = rcp(sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    T sa, ca;
    sincos_t(I.Om * (yf[3] - r), &sa, &ca);
    nh[0] = (v[0] * ca + v[1] * sa) * vn;
    nh[1] = (v[1] * ca - v[0] * sa) * vn;
    nh[2] = v[2] * vn;
}

// G = sum_j gbar_j K(n . o_j), K(c) = exp((c - 1)/sigma^2) / (2 pi sigma^2)
template <class T>
RT_HD T observer_sum(const InstT<T>& I, const T yf[8], const double* obs, const double* gbar, int n_obs,
                     double sigma) {
    T nh[3];
    arrival_direction(I, yf, nh);
    const double is2 = 1.0 / (sigma * sigma);
    const double norm = 1.0 / (2.0 * phys::pi * sigma * sigma);
    T G = T(0.0);
    for (int j = 0; j < n_obs; ++j) {
        T cj = nh[0] * obs[3 * j] + nh[1] * obs[3 * j + 1] + nh[2] * obs[3 * j + 2];
        G = G + (gbar[j] * norm) * exp((cj - 1.0) * is2);
    }
    return G;
}

RT_HD double smoothing_kernel(double c, double sigma) {
    return exp((c - 1.0) / (sigma * sigma)) / (2.0 * phys::pi * sigma * sigma);
}

// ----------------------------------------------------------------------------
// forward pass of one ray, with checkpoints of (y, h, facmax) every C accepted steps
// ----------------------------------------------------------------------------
struct AdjRay {
    double y[8], K[56];
    double h, facmax, lam;
    double gjs;  // the piece of the GJ density being integrated
    int nacc, nrej, nseg;
};

template <bool FL = true, class Store>
RT_HD void adj_ray_start(const InstT<double>& I, const double y0[8], double h0, AdjRay& R, Store&& store) {
    for (int d = 0; d < 8; ++d) R.y[d] = y0[d];
    R.gjs = adj_start_piece(I, R.y);
    adj_rhs<FL>(I, R.y, R.K, R.gjs);
    R.h = h0;
    R.facmax = 10.0;
    R.lam = 0.0;
    R.nacc = 0;
    R.nrej = 0;
    R.nseg = 1;
    store(0, R.y, R.h, R.facmax, R.gjs);
}

// One attempt; returns ST_OK while the ray continues.  On ST_ESCAPED, yf is the
// state at r = r_max on the last step's continuous extension and *theta its location.
template <bool FL = true, class Store>
RT_HD int adj_ray_step(const InstT<double>& I, const TolC& tol, int C, int Kc, AdjRay& R, Store&& store, double yf[8],
                       double* theta) {
    double ynew[8];
    const double hused = R.h;
    if (!adj_attempt<FL>(I, tol.rtol, tol.atol, R.y, R.K, ynew, &R.h, &R.facmax, NoStages{}, R.gjs)) {
        ++R.nrej;
        return (fabs(R.h) >= 1e-14 * (1.0 + fabs(R.lam))) ? ST_OK : ST_STEP_UNDERFLOW;
    }
    ++R.nacc;
    const double rnew = sqrt(ynew[0] * ynew[0] + ynew[1] * ynew[1] + ynew[2] * ynew[2]);
    bool finite_ok = true;
    for (int d = 0; d < 8; ++d) finite_ok = finite_ok && __builtin_isfinite(ynew[d]);
    // a crossing of the GJ null surface ends the step there (the ray restarts on the other
    // piece) unless r = r_max comes first
    const double thk = (finite_ok && rnew > value(I.R)) ? adj_null_crossing(I, R.y, R.K, ynew, hused, R.gjs) : 2.0;
    if (finite_ok && rnew >= tol.rmax) {
        // r = r_max on the continuous extension
        Stages S;
        for (int s = 0; s < 7; ++s)
            for (int d = 0; d < 8; ++d) S.K[s][d] = R.K[s * 8 + d];
        const double th = locate_crossing(R.y, ynew, S, hused, tol.rmax);
        if (th <= thk) {
            dense_at(R.y, ynew, S, hused, th, yf, 0, 8);
            *theta = th;
            R.lam += th * hused;
            return ST_ESCAPED;
        }
    }
    adj_advance<FL>(I, R.y, R.K, ynew, hused, thk, &R.gjs);
    R.lam += (thk <= 1.0) ? thk * hused : hused;
    if (!finite_ok) return ST_NONFINITE;
    if (rnew <= value(I.R)) return ST_HIT_STAR;
    if (R.nacc >= tol.max_steps) return ST_MAX_STEPS;
    if (!(fabs(R.h) >= 1e-14 * (1.0 + fabs(R.lam)))) return ST_STEP_UNDERFLOW;
    if (R.nacc % C == 0) {
        if (R.nseg >= Kc) return ST_MAX_STEPS;  // beyond the checkpoint budget
        store(R.nseg, R.y, R.h, R.facmax, R.gjs);
        ++R.nseg;
    }
    return ST_OK;
}

// ----------------------------------------------------------------------------
// reverse sweep
// ----------------------------------------------------------------------------
// What the reverse sweep of a ray needs besides the double instance: the parameter
// values, from which each dual-number instance is built where it is used (so that no
// dual instance stays live, in registers, across the sweep).
struct AdjParams {
    double p[6];
    StarFixed fx;
};

RT_HD void make_adj_params(const double p[6], const StarFixed& fx, AdjParams& A) {
    for (int q = 0; q < 6; ++q) A.p[q] = p[q];
    A.fx = fx;
}

// The observable at the final state: returns G = sum_j gbar_j K(n . o_j) and writes
// dG/dy_f (8) and dG/dp (6), by dual numbers with 14 tangents.
RT_HD_NOINLINE double observable_grad(const AdjParams& A, const double* yf, const double* obs, const double* gbar,
                                      int n_obs, double sigma, double* gy, double* gp) {
    D14 p14[6];
    for (int q = 0; q < 6; ++q) {
        p14[q] = D14(A.p[q]);
        p14[q].d[8 + q] = 1.0;
    }
    InstT<D14> I14 = make_inst_t<D14>(p14, A.fx);
    I14.oblique = 1;
    D14 yd[8];
    for (int d = 0; d < 8; ++d) {
        yd[d] = D14(yf[d]);
        yd[d].d[d] = 1.0;
    }
    D14 G = observer_sum(I14, yd, obs, gbar, n_obs, sigma);
    for (int d = 0; d < 8; ++d) gy[d] = G.d[d];
    for (int q = 0; q < 6; ++q) gp[q] = G.d[8 + q];
    return G.v;
}

// End of a ray's sweep: the seed's sensitivities (root, momentum and weight in
// 6-tangent dual numbers) contracted with the adjoint of y_0 and with G(y_f), and the
// stage products' parameter channels mapped to the parameters,
//   M = d(rs, Om, theta_m, log(Cwp R^3), log(kL))/dp   (theta_m enters only through its own
//   channel; kL, the finite magnetisation's cyclotron coefficient, carries B0, R and m_a).
template <bool FL = true>
RT_HD_NOINLINE void seed_and_channels(const AdjParams& A, uint64_t seed, int64_t j, const double* yb, double wG,
                                      const double* tc, double* pb) {
    D6 p6[6];
    for (int q = 0; q < 6; ++q) {
        p6[q] = D6(A.p[q]);
        p6[q].d[q] = 1.0;
    }
    InstT<D6> I6 = make_inst_t<D6>(p6, A.fx);
    I6.oblique = 1;
    if constexpr (!FL) I6.larmor = 0;
    const SeedT<D6> C6 = make_seed_t<D6>(p6, A.fx);
    D6 sd[10];
    seed_ray<D6>(I6, C6, seed, 0, j, sd);
    const double cw = I6.Cwp.v, r3 = I6.R3.v;
    for (int q = 0; q < 6; ++q) {
        double a = wG * sd[8].d[q];
        for (int d = 0; d < 8; ++d) a += yb[d] * sd[d].d[q];
        a += tc[0] * I6.rs.d[q] + tc[1] * I6.Om.d[q] + ((q == 2) ? tc[2] : 0.0);
        if (cw != 0.0 && r3 != 0.0) a += tc[3] * (I6.Cwp.d[q] / cw + I6.R3.d[q] / r3);
        if (I6.larmor && I6.kL.v != 0.0) a += tc[4] * (I6.kL.d[q] / I6.kL.v);
        pb[q] += a;
    }
}

// ----------------------------------------------------------------------------
// stage vector-Jacobian products
// ----------------------------------------------------------------------------
// With f = J grad(H), J = [[0, I], [-I, 0]] and Hess(H) symmetric,
//   v^T df/dy = Hess(H) u,  u = J^T v,
// one directional derivative of the hand-derived gradient: a pass in dual numbers with
// one tangent.  The star parameters enter f only through the instance constants rs, Om,
// (cos, sin) theta_m, the plasma coefficient Cwp R^3 and, with finite magnetisation, the
// cyclotron coefficient kL, so v^T df/dp = sum_c T_c dc/dp over the channels
// T_c = v^T df/dc = u . grad(dH/dc) (seed_and_channels maps them to p):
//   Om: H depends on Om and t only through the axis phase Om t, so dH/dOm = (t/Om) dH/dt
//     and T_Om = (u_t dH/dt + t (Hess(H) u)_t) / Om, from the first pass alone;
//   rs, theta_m: a pass with two tangents;
//   log(Cwp R^3): the strong-field Hamiltonian is linear in P, proportional to Cwp R^3
//     (H = H_vac + P or H_vac + P (1 - K)), so T = v.(f - f_vac) (f from the first pass);
//   with finite magnetisation (Sec. 4.1 eq. (DisRel)) H is not linear in P and depends
//     on kL: log(Cwp) (which moves P as log(Cwp R^3) does) and log(kL) by a pass with
//     two tangents.
// The passes run one after another so that few dual values are live at once.
// FL = false: the strong-field Hamiltonian, fixed at compile time.

// v^T df/dy (vy) and f(Y)
template <bool FL, class S>
RT_HD void vjp_state(const InstT<S>& I, const S* Y, const S* v, S* vy, S* f, double gjs) {
    typedef gdual<1, S> D1;
    InstT<D1> J = lift_inst<D1>(I);
    if constexpr (!FL) J.larmor = 0;
    D1 yd[8], fd[8];
    for (int i = 0; i < 4; ++i) {
        yd[i] = D1(Y[i]);
        yd[i].d[0] = S(0.0) - v[4 + i];  // u_x = -v_k
        yd[4 + i] = D1(Y[4 + i]);
        yd[4 + i].d[0] = v[i];  // u_k = v_x
    }
    rhs(J, yd, fd, 1.0, nullptr, gjs);
    // the tangent of f is J Hess(H) u, and Hess(H) u = J^T (J Hess(H) u)
    for (int i = 0; i < 4; ++i) {
        vy[i] = S(0.0) - fd[4 + i].d[0];
        vy[4 + i] = fd[i].d[0];
    }
    for (int i = 0; i < 8; ++i) f[i] = fd[i].v;
}

// sum_i v_i (df_i/dc1, df_i/dc2) for the two tangents set on J by the caller
template <class S>
RT_HD void vjp_pair(const InstT<gdual<2, S>>& J, const S* Y, const S* v, S* t1, S* t2, double gjs) {
    typedef gdual<2, S> D2;
    D2 yd[8], fd[8];
    for (int i = 0; i < 8; ++i) yd[i] = D2(Y[i]);
    rhs(J, yd, fd, 1.0, nullptr, gjs);
    S a = v[0] * fd[0].d[0], b = v[0] * fd[0].d[1];
    for (int i = 1; i < 8; ++i) {
        a = a + v[i] * fd[i].d[0];
        b = b + v[i] * fd[i].d[1];
    }
    *t1 = a;
    *t2 = b;
}

// The isotropic plasma's share of grad(H) (H = H_vac + P) at (x, t) = y[0..3]: grad P in
// (x, t), nothing in k; the same terms grad_h assembles, without the vacuum part
template <class T>
RT_HD void grad_p(const InstT<T>& I, const T* y, T g[4], double gjs) {
    if (I.density == DEN_NONE) {
        for (int i = 0; i < 4; ++i) g[i] = T(0.0);
        return;
    }
    T r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    T ir = frsqrt(r2);
    T n[3] = {y[0] * ir, y[1] * ir, y[2] * ir};
    T m[3], mt[3];
    magnetic_axis(I, y[3], m, mt, nullptr);
    T mu = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
    T dmu = I.oblique ? I.Om * (m[0] * n[1] - m[1] * n[0]) : T(0.0);
    Plasma<T> p = plasma_eval(I, n, ir, m, mu, dmu, gjs);
    for (int i = 0; i < 3; ++i) g[i] = p.pn * n[i] + p.pm * m[i];
    g[2] = g[2] + p.pz;
    g[3] = p.pt;
}

// Stage product of the vacuum part H_vac = -k_t^2/A + k.k - s q^2 (s = r_s/r, A = 1 - s,
// q = n.k; Sec. 4.1 eq. (SchwarzshildMetric1)), derived by hand: its gradient is
//   dH/dk = 2 k + kn n,  dH/dk_t = -2 kti,  dH/dx = Cn n + Ck k,  dH/dt = 0,
//   kn = -2 s q,  kti = k_t / A,  Cn = (s/r) W,  W = kti^2 + 3 q^2,  Ck = kn / r,
// and vy = Hess(H_vac) u is its derivative along u = (-v_k, v_x) (position -v_k, momentum
// v_x), through dr = n.dx, dn = (dx - n dr)/r, ds = -(s/r) dr, d(1/A) = -(s/r) dr / A^2,
// dq = dn.k + n.dk; vc0 = v^T df/dr_s with f = (dH/dk, -dH/dx) takes the same gradient's
// derivative in r_s at fixed state (ds/dr_s = 1/r).
template <class S>
RT_HD void vacuum_vjp(const InstT<S>& I, const S* Y, const S* v, S* vy, S* vc0) {
    const S ir = frsqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]);
    const S n[3] = {Y[0] * ir, Y[1] * ir, Y[2] * ir};
    const S s = I.rs * ir;
    const S iA = frcp(1.0 - s);
    const S q = n[0] * Y[4] + n[1] * Y[5] + n[2] * Y[6];
    const S sr = s * ir;
    const S kti = Y[7] * iA;
    const S kn = -2.0 * s * q;
    const S W = kti * kti + 3.0 * q * q;
    const S Cn = sr * W;
    const S Ck = kn * ir;
    // along u: dx = -v_k, dk = v_x, dk_t = v_3 (dt = -v_7 does not enter the vacuum part)
    const S dr = (S(0.0) - n[0] * v[4]) - n[1] * v[5] - n[2] * v[6];
    S dn[3];
    for (int i = 0; i < 3; ++i) dn[i] = (S(0.0) - v[4 + i] - n[i] * dr) * ir;
    const S sdr = sr * dr;  // -ds
    const S dq = (dn[0] * Y[4] + dn[1] * Y[5] + dn[2] * Y[6]) + (n[0] * v[0] + n[1] * v[1] + n[2] * v[2]);
    const S dkti = (v[3] - kti * sdr) * iA;
    const S dkn = 2.0 * (sdr * q - s * dq);
    const S dCn = sr * (2.0 * kti * dkti + 6.0 * q * dq) - 2.0 * sdr * ir * W;
    const S dCk = (dkn - kn * ir * dr) * ir;
    for (int i = 0; i < 3; ++i) {
        vy[i] = dCn * n[i] + Cn * dn[i] + dCk * Y[4 + i] + Ck * v[i];
        vy[4 + i] = dkn * n[i] + kn * dn[i] + 2.0 * v[i];
    }
    vy[3] = S(0.0);
    vy[7] = -2.0 * dkti;
    // r_s: d kn = -2 q / r, d kti = kti / (A r), d Cn = W / r^2 + 2 (s/r) kti d kti, d Ck = d kn / r
    const S pkn = -2.0 * q * ir;
    const S pkti = kti * iA * ir;
    const S pCn = W * ir * ir + 2.0 * sr * kti * pkti;
    const S vxn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    const S vkn = v[4] * n[0] + v[5] * n[1] + v[6] * n[2];
    const S vkk = v[4] * Y[4] + v[5] * Y[5] + v[6] * Y[6];
    *vc0 = pkn * vxn - 2.0 * v[3] * pkti - pCn * vkn - pkn * ir * vkk;
}

// The same for an isotropic plasma (or none) and the strong-field Hamiltonian: H = H_vac + P
// with P a function of (x, t) alone, r_s only in H_vac, and Om, theta_m and the plasma
// coefficient only in P.  The vacuum part in closed form (vacuum_vjp), then grad P in dual
// numbers with tangents u's (x, t) part and theta_m (Hess(P) u, the theta_m channel, and
// through its value, which is the plasma part of f, the plasma channel and the Om channel).
template <class S>
RT_HD void stage_vjp_iso(const InstT<S>& I, const S* Y, const S* v, S* vy, S* vc, double gjs) {
    typedef gdual<2, S> D2;
    vacuum_vjp(I, Y, v, vy, &vc[0]);
    {
        InstT<D2> J = lift_inst<D2>(I);  // grad P
        J.larmor = 0;
        J.oblique = 1;  // the theta_m tangent needs the rotating axis, also where sin theta_m = 0
        J.cm.d[1] = I.msm;  // d/dtheta_m of (cos, sin)
        J.sm.d[1] = I.cm;
        D2 yd[4], gp[4];
        for (int i = 0; i < 4; ++i) {
            yd[i] = D2(Y[i]);
            yd[i].d[0] = S(0.0) - v[4 + i];
        }
        grad_p(J, yd, gp, gjs);
        for (int i = 0; i < 4; ++i) vy[i] = vy[i] + gp[i].d[0];  // + Hess(P) u
        // f's plasma part is -grad P in the k rows
        S a = v[4] * gp[0].d[1], b = v[4] * gp[0].v;
        for (int i = 1; i < 4; ++i) {
            a = a + v[4 + i] * gp[i].d[1];
            b = b + v[4 + i] * gp[i].v;
        }
        vc[2] = S(0.0) - a;
        vc[3] = S(0.0) - b;
        // Om (see stage_vjp): dH/dt = dP/dt, u_t = -v_7
        vc[1] = (Y[3] * vy[3] - v[7] * gp[3].v) * I.iOm;
    }
    vc[4] = S(0.0);
}

// v^T df/dy (vy) and the channels vc[0..4] = v^T df/dc for c = rs, Om, theta_m, the plasma
// coefficient and kL (vc[4] = 0 for the strong-field Hamiltonian) at the state Y (S = double;
// generic for the host operation counter); an isotropic plasma (or none) takes stage_vjp_iso.
template <bool FL = true, class S = double>
RT_HD void stage_vjp(const InstT<S>& I, const S* Y, const S* v, S* vy, S* vc, double gjs = 0.0) {
    if (!(FL && I.larmor) && (I.plasma == PL_ISO || I.density == DEN_NONE)) {
        stage_vjp_iso<S>(I, Y, v, vy, vc, gjs);
        return;
    }
    S f[8];
    vjp_state<FL, S>(I, Y, v, vy, f, gjs);
    // Om: u_t = -v_7, dH/dt = -f_7, (Hess(H) u)_t = vy_3
    vc[1] = (v[7] * f[7] + Y[3] * vy[3]) * I.iOm;
    {
        InstT<gdual<2, S>> J = lift_inst<gdual<2, S>>(I);
        if constexpr (!FL) J.larmor = 0;
        J.rs.d[0] = S(1.0);
        J.cm.d[1] = I.msm;  // d/dtheta_m of (cos, sin)
        J.sm.d[1] = I.cm;
        vjp_pair<S>(J, Y, v, &vc[0], &vc[2], gjs);
    }
    if (FL && I.larmor) {
        InstT<gdual<2, S>> J = lift_inst<gdual<2, S>>(I);
        J.Cwp.d[0] = I.Cwp;
        J.kL.d[1] = I.kL;
        vjp_pair<S>(J, Y, v, &vc[3], &vc[4], gjs);
    } else {
        InstT<S> Iv = I;  // the same star without plasma
        Iv.density = DEN_NONE;
        Iv.larmor = 0;
        S fv[8];
        rhs(Iv, Y, fv, 1.0);
        S a = v[0] * (f[0] - fv[0]);
        for (int i = 1; i < 8; ++i) a = a + v[i] * (f[i] - fv[i]);
        vc[3] = a;
        vc[4] = S(0.0);
    }
}

// Per-lane scratch of the reverse sweep's step adjoint, in rows of 8 values: lr(r) is row r,
// indexed [d], d < 8.
//   rows 0..4  the stage state Y_{r+2} of the step being walked; once stage r + 2 has taken
//              its state, the row holds that stage's adjoint w_{r+2} instead
//   LR_YNB     the adjoint of the step's end y_{n+1}
//   LR_GYF     the adjoint of the step's output where it ends on its continuous extension
//   LR_DC      that output's weights of K_1..K_7 (7 values)
//   LR_YN      the step's start y_n
// Kept there rather than in registers, these leave the stage products room to run without
// spilling.
constexpr int LR_YNB = 5, LR_GYF = 6, LR_DC = 7, LR_YN = 8, LR_ROWS = 9;
constexpr int LR_SLOTS = 8 * LR_ROWS;

// A row of 8 values of one lane, the d-th at p[d * STRIDE] (STRIDE = the wave's width where
// the lanes' values interleave, 1 for a lane of its own)
template <class T, int STRIDE>
struct LaneRow {
    T* p;
    RT_HD T& operator[](int d) const { return p[d * STRIDE]; }
};

// Adjoint of one accepted step y_n -> y_{n+1} through its stages,
//   Y_l = y_n + h sum_{i<l} a_li K_i,  y_{n+1} = y_n + h sum_i b_i K_i,  K_i = f(Y_i).
// On entry rows 0..4 of lr hold Y_2..Y_6, LR_YN holds y_n and y7 the step's end
// y_{n+1} = Y_7, where K_7 = f(Y_7) is taken (read for dense = true only, before the first
// stage); yb holds the adjoint of y_n from the step's output and row LR_YNB that of
// y_{n+1}; with dense = true the step ends on its continuous extension, whose value depends
// on K_1..K_7, and the output's adjoint of K_i is dc_i gyf (rows LR_DC and LR_GYF);
// otherwise the output is y_{n+1} itself and K_7 is not visited.
// Each stage, last first, takes Kbar_i = dc_i gyf + h b_i ynb + h sum_{l>i} a_li w_l and
// gives w_i = (df/dy(Y_i))^T Kbar_i, which goes to ynb for i = 7 and to yb otherwise;
// w_2..w_6 replace Y_2..Y_6 in their rows.  On return yb holds the adjoint of y_n; the
// parameter channels are added to tc.
template <bool FL, bool ISO, class S, class Rows>
RT_HD void step_adjoint(const InstT<S>& I, const S* y7, S h, bool dense, S* yb, S* tc, Rows&& lr, double gjs) {
    using namespace dp5;
    // stage i's coefficients in row i - 1: b_i, then a_{l,i} at 1 + l - 2 for l = 2..6 (the
    // column of a), contiguous so that the wave-uniform i reads them with one wide scalar load,
    // issued at the top of the stage so that it lands while the stage rows are read
    const double Cf[7][6] = {{b1, a21, a31, a41, a51, a61},
                             {0.0, 0, a32, a42, a52, a62},
                             {b3, 0, 0, a43, a53, a63},
                             {b4, 0, 0, 0, a54, a64},
                             {b5, 0, 0, 0, 0, a65},
                             {b6, 0, 0, 0, 0, 0},
                             {0.0, 0, 0, 0, 0, 0}};
    S v[8], Y[8], vy[8], vc[5];
    const int top = dense ? 7 : 6;
#pragma unroll 1
    for (int i0 = 7; i0 >= 1; --i0) {
        // read before any lane leaves the iteration: the stage index is the wave's
        const int i = wave_uniform(i0);
        if (i > top) continue;
        double cf[6];
        for (int q = 0; q < 6; ++q) cf[q] = Cf[i - 1][q];
        if (i == 7) {
            for (int d = 0; d < 8; ++d) Y[d] = y7[d];
        } else {
            const auto r = lr(i >= 2 ? i - 2 : LR_YN);
            for (int d = 0; d < 8; ++d) Y[d] = r[d];
        }
        const S hb = h * cf[0];
        {
            const auto r = lr(LR_YNB);
            for (int d = 0; d < 8; ++d) v[d] = hb * r[d];
        }
        if (dense) {
            const S c = lr(LR_DC)[i - 1];
            const auto r = lr(LR_GYF);
            for (int d = 0; d < 8; ++d) v[d] = v[d] + c * r[d];
        }
#pragma unroll
        for (int l = 2; l <= 6; ++l) {
            if (l <= i) continue;
            const S c = h * cf[l - 1];
            const auto r = lr(l - 2);
            S w[8];  // the whole row first: its reads go out together
            for (int d = 0; d < 8; ++d) w[d] = r[d];
            for (int d = 0; d < 8; ++d) v[d] = v[d] + c * w[d];
        }
        if constexpr (ISO)
            stage_vjp_iso<S>(I, Y, v, vy, vc, gjs);
        else
            stage_vjp<FL, S>(I, Y, v, vy, vc, gjs);
        for (int c = 0; c < 5; ++c) tc[c] = tc[c] + vc[c];
        if (i == 7) {
            const auto r = lr(LR_YNB);
            for (int d = 0; d < 8; ++d) r[d] = r[d] + vy[d];
        } else {
            for (int d = 0; d < 8; ++d) yb[d] = yb[d] + vy[d];
            if (i >= 2) {
                const auto r = lr(i - 2);
                for (int d = 0; d < 8; ++d) r[d] = vy[d];
            }
        }
    }
    const auto r = lr(LR_YNB);
    for (int d = 0; d < 8; ++d) yb[d] = yb[d] + r[d];
}

// E(theta) and dE/dtheta on the continuous extension of the step yn -> ynew (yn indexed [d])
template <class YV>
RT_HD void dense_point_deriv(const YV& yn, const double* K, const double* ynew, double hn, double t, double* e,
                             double* et) {
    using namespace dp5;
    const double om = 1.0 - t;
    const double dd[7] = {d1, 0.0, d3, d4, d5, d6, d7};
    for (int d = 0; d < 8; ++d) {
        const double ydiff = ynew[d] - yn[d];
        const double r3 = hn * K[d] - ydiff;
        const double r4 = ydiff - hn * K[48 + d] - r3;
        double r5 = 0.0;
        for (int q = 0; q < 7; ++q) r5 += dd[q] * K[q * 8 + d];
        r5 *= hn;
        const double Qq = r3 + t * (r4 + om * r5);
        e[d] = yn[d] + t * (ydiff + om * Qq);
        const double dP = -Qq + om * (r4 + (1.0 - 2.0 * t) * r5);
        et[d] = ydiff + om * Qq + t * dP;
    }
}

// Reverse sweep of one escaped ray (S accepted steps, nseg checkpoints, crossing of r_max
// at theta on the last step).  load(s, y, &h, &facmax, &gjs) reads checkpoint s; rb(idx, d)
// is the replay buffer (C steps x 11 values: y, h, the null-surface crossing thk (2: none)
// and the piece gjs of the step); lr(r) gives the per-lane rows of step_adjoint.  Adds
// d(w G(y_f))/dp to pb.  Returns the number of steps or checkpoints the recompute could not
// reproduce (0 when all is well).
template <bool FL = true, bool ISO = false, class Load, class Replay, class Rows>
RT_HD int adj_reverse_ray(const InstT<double>& I, const AdjParams& A, const TolC& tol, uint64_t seed, int64_t j, int S,
                          int nseg, double th, double w, int C, Load&& load, Replay&& rb, Rows&& lr,
                          const double* obs, const double* gbar, int n_obs, double sigma, double pb[6]) {
    using namespace dp5;
    double tc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // parameter channels of the stage products
    double yb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double wG = 0.0;
    int missing = 0;
    for (int s = nseg - 1; s >= 0; --s) {
        // recompute the segment from its checkpoint, with the forward pass's decisions
        double y[8], ynew[8], K[56], h, facmax, gjs;
        load(s, y, &h, &facmax, &gjs);
        const int first = s * C;
        const int count = (S - first < C) ? (S - first) : C;
        adj_rhs<FL>(I, y, K, gjs);
        int stored = 0;
        for (int guard = 0; stored < count && guard < 64 * C; ++guard) {
            const double hused = h;
            if (!adj_attempt<FL>(I, tol.rtol, tol.atol, y, K, ynew, &h, &facmax, NoStages{}, gjs)) continue;
            // the last step ends at r_max (its own crossing test does not matter)
            const double thk = (first + stored == S - 1) ? 2.0 : adj_null_crossing(I, y, K, ynew, hused, gjs);
            for (int d = 0; d < 8; ++d) rb(stored, d) = y[d];
            rb(stored, 8) = hused;
            rb(stored, 9) = thk;
            rb(stored, 10) = gjs;
            ++stored;
            adj_advance<FL>(I, y, K, ynew, hused, thk, &gjs);
        }
        missing += count - stored;
        if (stored == count && s + 1 < nseg) {
            // the recomputed segment must end exactly on the next checkpoint
            double yc[8], hc, fc, gc;
            load(s + 1, yc, &hc, &fc, &gc);
            bool same = (hc == h) && (fc == facmax) && (gc == gjs);
            for (int d = 0; d < 8; ++d) same = same && (yc[d] == y[d]);
            if (!same) ++missing;
        }
        // walk the segment backwards; each step's replay entry is loaded one step ahead, so
        // that its latency hides behind the step before
        double nyn[8], nhn = 0.0, nthk = 2.0, ngn = 0.0;
        auto fetch = [&](int k) {
            for (int d = 0; d < 8; ++d) nyn[d] = rb(k, d);
            nhn = rb(k, 8);
            nthk = rb(k, 9);
            ngn = rb(k, 10);
        };
        if (stored > 0) fetch(stored - 1);
        for (int idx = stored - 1; idx >= 0; --idx) {
            double yn[8];
            for (int d = 0; d < 8; ++d) yn[d] = nyn[d];
            const double hn = nhn, thk = nthk, gn = ngn;
            if (idx > 0) fetch(idx - 1);
            {
                const auto r = lr(LR_YN);
                for (int d = 0; d < 8; ++d) r[d] = yn[d];
            }
            // the step's stages again (no error estimate: the step is known accepted), its
            // inner stage states into rows 0..4
            adj_rhs<FL>(I, yn, K, gn);
            // from here on y_n is read from its row, which keeps it out of the registers
            const auto ynr = lr(LR_YN);
            adj_stages<FL>(I, ynr, K, ynew, hn,
                           [&](int i, const double* Yi) {
                               const auto r = lr(i - 2);
                               for (int d = 0; d < 8; ++d) r[d] = Yi[d];
                           },
                           gn);
            const bool last = (first + idx == S - 1);
            const bool dense = last || thk <= 1.0;
            if (dense) {
                // the step ends inside, at E(theta): y_f at r(E) = r_max, or the restart
                // point on the null surface g(E) = 0.  The adjoint of E(theta) loses its
                // component along dE/dtheta against the surface's gradient q:
                //   beta = (ybar . dE/dtheta) / (q . dE/dtheta),  ybar -= beta q,
                // and for g the parameters' part -beta dg/dp joins the channels.
                const double t = last ? th : thk;
                double e[8], et[8], q[4], gyf[8], dc[7], gOm = 0.0, gth = 0.0;
                dense_point_deriv(ynr, K, ynew, hn, t, e, et);
                if (last) {
                    // the observable with 8 state and 6 parameter tangents (the non-inlined
                    // helpers get copies, so that the sweep's own arrays never leave registers)
                    double gp[6], gy[8];
                    wG = observable_grad(A, e, obs, gbar, n_obs, sigma, gy, gp);
                    for (int d = 0; d < 8; ++d) gyf[d] = gy[d] * w;
                    for (int k = 0; k < 6; ++k) pb[k] += w * gp[k];
                    const double r = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                    q[0] = e[0] / r; q[1] = e[1] / r; q[2] = e[2] / r; q[3] = 0.0;
                } else {
                    for (int d = 0; d < 8; ++d) gyf[d] = yb[d];
                    gj_factor_grad(I.Om, I.cm, I.sm, 1, e, q, &gOm, &gth);  // theta_m tangents: rotating axis
                }
                double num = 0.0, den = 0.0;
                for (int d = 0; d < 8; ++d) num += gyf[d] * et[d];
                for (int d = 0; d < 4; ++d) den += q[d] * et[d];
                const double beta = num / den;
                for (int d = 0; d < 4; ++d) gyf[d] -= beta * q[d];
                tc[1] -= beta * gOm;
                tc[2] -= beta * gth;
                // E(theta) = (1 - cy) y_n + cy y_{n+1} + h sum_i dc_i K_i (nested form of the
                // continuous extension): its adjoint to y_n, y_{n+1} and each K_i
                const double om = 1.0 - t;
                const double c3 = t * om, c4 = t * t * om, c5 = t * t * om * om, cy = t - c3 + 2.0 * c4;
                dc[0] = hn * (c3 - c4 + c5 * d1);
                dc[1] = 0.0;
                dc[2] = hn * c5 * d3;
                dc[3] = hn * c5 * d4;
                dc[4] = hn * c5 * d5;
                dc[5] = hn * c5 * d6;
                dc[6] = hn * (c5 * d7 - c4);
                const auto rg = lr(LR_GYF), rd = lr(LR_DC), rn = lr(LR_YNB);
                for (int i = 0; i < 7; ++i) rd[i] = dc[i];
                for (int d = 0; d < 8; ++d) {
                    rg[d] = gyf[d];
                    rn[d] = cy * gyf[d];
                    yb[d] = (1.0 - cy) * gyf[d];
                }
            } else {
                // y_{n+1} = y_n + h sum_i b_i K_i is the step's output; yb holds its adjoint
                const auto rn = lr(LR_YNB);
                for (int d = 0; d < 8; ++d) {
                    rn[d] = yb[d];
                    yb[d] = 0.0;
                }
            }
            step_adjoint<FL, ISO, double>(I, ynew, hn, dense, yb, tc, lr, gn);
        }
    }
    // seed: y_0(p) and w(p); the stage products' channels
    double ybc[8], tcc[5], pbc[6];
    for (int d = 0; d < 8; ++d) ybc[d] = yb[d];
    for (int c = 0; c < 5; ++c) tcc[c] = tc[c];
    for (int k = 0; k < 6; ++k) pbc[k] = 0.0;
    seed_and_channels<FL>(A, seed, j, ybc, wG, tcc, pbc);
    for (int k = 0; k < 6; ++k) pb[k] += pbc[k];
    return missing;
}

}  // namespace rtd
