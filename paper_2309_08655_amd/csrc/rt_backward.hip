// Backward tracing from an image plane (McDonald & Witte, arXiv:2309.08655,
// Sec. 2.1 eq. (BackPower); Sec. 2.3 on gravity's stabilising role; Sec. 2.4 and
// Sec. 3 on multiple production sites along one worldline).
//
// Each pixel of an nx x ny plane at distance D, perpendicular to the line of
// sight, launches a parallel ray with k_t = -1 (monochromatic) and |k| on the LO
// branch of eq. (AnisotropicDisp).  Rays are integrated backwards in the
// worldline parameter with the same DOPRI5 scheme as the forward tracer, in a
// persistent work-queue kernel.  Production events are the sign changes of
// G = g^{mu nu} k_mu k_nu + m_a^2 (the photon momentum on the axion mass shell),
// sampled at 1/4, 1/2, 3/4 and 1 of every accepted step on the continuous
// extension and located by 60 bisections.
#include "rt_common.hpp"

namespace rtd {

// a step never moves the ray by more than a tenth of its radius (rays start in
// near-vacuum far away, where the error estimate alone would let the step grow
// across the whole plasma region)
__device__ __forceinline__ double step_cap(const double y[8], const double f[8], double h) {
    double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double sp = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    return fmin(h, 0.1 * r / sp);
}

__device__ __forceinline__ double event_G(const InstT<double>& I, const double y[8]) {
    return g_kk(I, y) + I.ma2;
}

// image plane: pixel centres of an nx x ny grid of side db, or (b1 != nullptr) the
// explicit plane offsets b1[p], b2[p] of each ray
struct ImageC {
    double D, no[3], e1[3], e2[3], db;
    int nx, ny;
    const double* b1;
    const double* b2;
};

__global__ void __launch_bounds__(256) bwd_init_kernel(InstT<double> I, TolC tol, ImageC im, int64_t n, WorkCtr* ctr,
                                                       int32_t* __restrict__ list, double* __restrict__ h0s,
                                                       double* __restrict__ k1s, double* __restrict__ y0s,
                                                       int32_t* __restrict__ nev) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        int64_t p = base + threadIdx.x;
        bool valid = p < n;
        if (valid) {
            double b1, b2;
            if (im.b1 != nullptr) {
                b1 = im.b1[p];
                b2 = im.b2[p];
            } else {
                int pi = (int)(p / im.ny), pj = (int)(p % im.ny);
                b1 = (pi + 0.5 - 0.5 * im.nx) * im.db;
                b2 = (pj + 0.5 - 0.5 * im.ny) * im.db;
            }
            double y[8];
            for (int d = 0; d < 3; ++d) y[d] = im.D * im.no[d] + b1 * im.e1[d] + b2 * im.e2[d];
            y[3] = 0.0;
            double r0 = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
            double ir = 1.0 / r0;
            double nn[3] = {y[0] * ir, y[1] * ir, y[2] * ir};
            double A0 = 1.0 - I.rs * ir;
            double w2 = 1.0 / A0;
            double m[3], mt[3];
            magnetic_axis(I, y[3], m, mt);
            double mu = m[0] * nn[0] + m[1] * nn[1] + m[2] * nn[2];
            Plasma<double> pl = plasma_eval(I, nn, ir, m, mu, 0.0);
            double kap2;
            if (I.plasma == PL_ISO) {
                kap2 = w2 - pl.P;
            } else {
                const DipoleShape<double> sh = dipole_shape(I, ir);
                double u[3];
                dipole_dir(nn, m, mu, u, sh.g);
                double cB = (im.no[0] * u[0] + im.no[1] * u[1] + im.no[2] * u[2]) / sqrt(1.0 + sh.c * mu * mu);
                kap2 = w2 * (w2 - pl.P) / (w2 - pl.P * cB * cB);
            }
            double kap = sqrt(kap2);
            double ko[3] = {kap * im.no[0], kap * im.no[1], kap * im.no[2]};
            double nko = nn[0] * ko[0] + nn[1] * ko[1] + nn[2] * ko[2];
            double corr = nko / sqrt(A0) - nko;
            for (int d = 0; d < 3; ++d) y[4 + d] = ko[d] + corr * nn[d];
            y[7] = -1.0;
            // GJ density: the smooth piece of |g| the pixel's ray starts on, which the tracing
            // kernel integrates from here (also for the starting step's probe)
            const double gjs = (I.density == DEN_GJ) ? ((gj_factor(I, y) < 0.0) ? -1.0 : 1.0) : 0.0;
            double f0[8];
            auto f = [&](const double* yy, double* ff) { rhs(I, yy, ff, -1.0, nullptr, gjs); };
            f(y, f0);
            double h = step_cap(y, f0, initial_step(f, y, f0, tol.rtol, tol.atol));
            h0s[p] = h;
            for (int d = 0; d < 8; ++d) { k1s[d * n + p] = f0[d]; y0s[d * n + p] = y[d]; }
            nev[p] = 0;
        }
        unsigned long long mask = __ballot(valid);
        if (mask) {
            int lane = __lane_id();
            int leader = __ffsll((long long)mask) - 1;
            unsigned long long pos = 0;
            if (lane == leader) pos = atomicAdd(&ctr->len, (unsigned long long)__popcll(mask));
            pos = __shfl(pos, leader);
            if (valid) list[pos + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)p;
        }
    }
}

__device__ __forceinline__ void write_final_bwd(const InstT<double>& I, const double y[8], double lam, double h,
                                                int nacc, int nrej, int status, int64_t p, int64_t n,
                                                double* __restrict__ fin, int32_t* __restrict__ ifin,
                                                const AxisRef* ref) {
    for (int d = 0; d < 8; ++d) fin[d * n + p] = y[d];
    for (int d = 8; d < 12; ++d) fin[d * n + p] = 0.0;
    fin[12 * n + p] = hamiltonian(I, y, ref);
    fin[13 * n + p] = lam;
    fin[14 * n + p] = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    fin[15 * n + p] = h;
    ifin[p] = nacc;
    ifin[n + p] = nrej;
    ifin[2 * n + p] = status;
}

template <int BLOCK, int MINW, int SPEC = 0>
__global__ void __launch_bounds__(BLOCK, MINW) trace_bwd_kernel(InstT<double> I, TolC tol, double D, int64_t n,
                                                          WorkCtr* ctr, const int32_t* __restrict__ list,
                                                          const double* __restrict__ h0s,
                                                          const double* __restrict__ k1s,
                                                          const double* __restrict__ y0s, int32_t K,
                                                          double* __restrict__ ev, int32_t* __restrict__ nev,
                                                          double* __restrict__ fin, int32_t* __restrict__ ifin,
                                                          int refill_min) {
    // specialised instantiations (SPEC = 1 + plasma + 2 density + 8 oblique) fix these
    // switches at compile time, with the same arithmetic as the generic kernel
    if constexpr (SPEC > 0) {  // the flat dipole (GR-dipole stars take the generic kernel)
        I.plasma = (SPEC - 1) & 1;
        I.density = ((SPEC - 1) >> 1) & 3;
        I.oblique = ((SPEC - 1) >> 3) & 1;
        I.gr_dipole = 0;
        I.larmor = 0;
    }
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long nlist = ctr->len;
    unsigned long long iters = 0;
    bool active = false, exhausted = false;
    int64_t p = 0;
    double y[8], ynew[8];
    Stages S;
    double h = 0.0, lam = 0.0, facmax = 10.0, Gprev = 0.0, rprev = 0.0;
    double gjs = 0.0;  // the piece of the GJ density being integrated (0: other densities)
    int nacc = 0, nrej = 0, ne = 0;
    for (int d = 0; d < 8; ++d) { y[d] = 0.0; S.K[0][d] = 0.0; }
    y[0] = 1e5;
    y[7] = -1.0;
    AxisRef ref = axis_ref_at(I, 0.0);
    // gnew: the GJ factor at the last state f was evaluated at (after an attempt, the step's
    // end), for the null-surface test
    double gnew = 0.0;
    auto f = [&](const double* yy, double* ff) { rhs(I, yy, ff, -1.0, &ref, gjs, &gnew); };

    while (true) {
        unsigned long long idle = __ballot(!active);
        if (idle && !exhausted) {
            int cnt = __popcll(idle);
            if (cnt >= refill_min || idle == __ballot(true)) {
                int leader = __ffsll((long long)idle) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(&ctr->head, (unsigned long long)cnt);
                base = __shfl(base, leader);
                if (!active) {
                    unsigned long long q = base + __popcll(idle & below);
                    if (q < nlist) {
                        p = list[q];
                        for (int d = 0; d < 8; ++d) { y[d] = y0s[d * n + p]; S.K[0][d] = k1s[d * n + p]; }
                        h = h0s[p];
                        lam = 0.0; facmax = 10.0; nacc = 0; nrej = 0; ne = 0;
                        if (I.oblique) ref = axis_ref_at(I, y[3]);
                        gjs = (I.density == DEN_GJ) ? ((gj_factor(I, y, &ref) < 0.0) ? -1.0 : 1.0) : 0.0;
                        Gprev = event_G(I, y);
                        rprev = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                        active = true;
                    }
                }
                if (base + (unsigned long long)cnt >= nlist) exhausted = true;
            }
        }
        if (__ballot(active) == 0ull) {
            if (exhausted) break;
            continue;
        }
        ++iters;

        double err2 = dopri_attempt(f, y, S, h, ynew, tol.rtol, tol.atol);
        if (!active) continue;
        if (!(err2 <= 1.0)) {
            ++nrej;
            h *= step_factor(err2, facmax, false);
            facmax = 1.0;
            if (!(fabs(h) >= 1e-14 * (1.0 + fabs(lam)))) {
                write_final_bwd(I, y, lam, h, nacc, nrej, ST_STEP_UNDERFLOW, p, n, fin, ifin, &ref);
                nev[p] = ne;
                active = false;
            }
            continue;
        }
        ++nacc;
        // a step that crosses the GJ density's null surface ends there: the ray goes on
        // along the other piece from the first point past it (thk > 1: no crossing)
        double thk = 2.0;
        if (gjs != 0.0) {
            const double g1 = gnew;  // = gj_factor(I, ynew, &ref), from the last stage
            if (gjs * g1 < 0.0) {
                double phik;
                thk = locate_null_crossing(I, y, ynew, S, h, gjs, gjs * gj_factor(I, y, &ref), gjs * g1, &ref, &phik);
            }
        }
        const double tend = (thk <= 1.0) ? thk : 1.0;
        // production events on the part of the step taken
        double thp = 0.0, Gp = Gprev;
        for (int qq = 1; qq <= 4; ++qq) {
            double thq = 0.25 * qq * tend;
            double Gq;
            if (qq == 4 && thk > 1.0) {
                Gq = event_G(I, ynew);
            } else {
                double yq[8];
                dense_at(y, ynew, S, h, thq, yq, 0, 8);
                Gq = event_G(I, yq);
            }
            if ((Gp > 0.0 && Gq <= 0.0) || (Gp < 0.0 && Gq >= 0.0)) {
                double lo = thp, hi = thq, ym[8];
                for (int it = 0; it < 60; ++it) {
                    double mid = 0.5 * (lo + hi);
                    dense_at(y, ynew, S, h, mid, ym, 0, 8);
                    double Gm = event_G(I, ym);
                    if ((Gp > 0.0) == (Gm > 0.0)) lo = mid; else hi = mid;
                }
                dense_at(y, ynew, S, h, 0.5 * (lo + hi), ym, 0, 8);
                if (ne < K) {
                    for (int d = 0; d < 8; ++d) ev[((int64_t)ne * RT_NEV_ + d) * n + p] = ym[d];
                    double re = sqrt(ym[0] * ym[0] + ym[1] * ym[1] + ym[2] * ym[2]);
                    ev[((int64_t)ne * RT_NEV_ + 8) * n + p] = -ym[7] - 1.0;
                    ev[((int64_t)ne * RT_NEV_ + 9) * n + p] = -ym[7] / sqrt(1.0 - I.rs / re);
                }
                ++ne;
            }
            thp = thq;
            Gp = Gq;
        }
        Gprev = Gp;
        if (thk <= 1.0) {
            double yk[8];
            dense_at(y, ynew, S, h, thk, yk, 0, 8);
            lam += thk * h;
            for (int d = 0; d < 8; ++d) y[d] = yk[d];
            gjs = -gjs;
            if (I.oblique) axis_ref_advance(I, ref, y[3]);
            f(y, S.K[0]);
        } else {
            lam += h;
            if (I.oblique) axis_ref_advance(I, ref, ynew[3]);
            for (int d = 0; d < 8; ++d) { y[d] = ynew[d]; S.K[0][d] = S.K[6][d]; }
        }
        double rnew = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
        bool finite_ok = true;
        for (int d = 0; d < 8; ++d) finite_ok = finite_ok && isfinite(y[d]);
        int status = ST_OK;
        if (!finite_ok) status = ST_NONFINITE;
        else if (rnew <= I.R) status = ST_HIT_STAR;
        else if (rnew > 1.01 * D && rnew > rprev) status = ST_ESCAPED;
        if (status == ST_OK) {
            rprev = rnew;
            h = step_cap(y, S.K[0], h * step_factor(err2, facmax, true));
            facmax = 10.0;
            if (nacc >= tol.max_steps) status = ST_MAX_STEPS;
            else if (!(fabs(h) >= 1e-14 * (1.0 + fabs(lam)))) status = ST_STEP_UNDERFLOW;
        }
        if (status != ST_OK) {
            write_final_bwd(I, y, lam, h, nacc, nrej, status, p, n, fin, ifin, &ref);
            nev[p] = ne;
            active = false;
        }
    }
    if (lane == 0) atomicAdd(&ctr->iters, iters);
}

template <int BLOCK, int MINW, int SPEC = 0>
static int launch_bwd_block(const rt_schedule& sc, const InstT<double>& I, const TolC& T, double D, int64_t n,
                            const FwdWs& W, const double* y0s, int32_t K, double* ev, int32_t* nev, double* fin,
                            int32_t* ifin, hipStream_t st) {
    int grid = persistent_grid(sc, (const void*)trace_bwd_kernel<BLOCK, MINW, SPEC>, BLOCK);
    timing_begin(st, RT_KERNEL_TRACE_BACKWARD);
    hipLaunchKernelGGL((trace_bwd_kernel<BLOCK, MINW, SPEC>), dim3(grid), dim3(BLOCK), 0, st, I, T, D, n, W.ctr,
                       W.list, W.h0, W.k1, y0s, K, ev, nev, fin, ifin, sc.refill_min);
    timing_end(st);
    return check_launch("trace_bwd_kernel");
}

// ---------------------------------------------------------------------------
// Backward power (Sec. 2.1 eq. (BackPower)): per-ray sums of the event weights and the
// image sum dP/dOmega = sum_rays area * wsum / (hbar c)^2.  The sum is reduced in a fixed
// order (per-thread strided sums, an LDS tree per block, one block over the block
// partials), so it does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int POWER_BLOCK = 256;
constexpr int POWER_MAX_BLOCKS = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

__global__ void __launch_bounds__(POWER_BLOCK) event_power_kernel(InstT<double> I, SeedT<double> C,
                                                                  const double* __restrict__ ev,
                                                                  const int32_t* __restrict__ nev, int64_t n,
                                                                  int32_t K, double Lc_max,
                                                                  const double* __restrict__ area, double area0,
                                                                  double* __restrict__ wsum,
                                                                  double* __restrict__ partial) {
    __shared__ double sh[POWER_BLOCK];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * POWER_BLOCK;
    for (int64_t p = (int64_t)blockIdx.x * POWER_BLOCK + threadIdx.x; p < n; p += stride) {
        const int m = min(nev[p], K);
        double w = 0.0;
        for (int e = 0; e < m; ++e) {
            double y[8];
            for (int d = 0; d < 8; ++d) y[d] = ev[((int64_t)e * RT_NEV_ + d) * n + p];
            w += event_weight(I, C, y, Lc_max, nullptr);
        }
        wsum[p] = w;
        acc += w * (area != nullptr ? area[p] : area0);
    }
    if (partial == nullptr) return;
    const double b = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

__global__ void __launch_bounds__(POWER_MAX_BLOCKS) power_total_kernel(const double* __restrict__ partial, int nb,
                                                                       double scale, double* __restrict__ total) {
    __shared__ double sh[POWER_MAX_BLOCKS];
    const double v = ((int)threadIdx.x < nb) ? partial[threadIdx.x] : 0.0;
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) *total = t * scale;
}

// shared tail of the two backward entry points
static int trace_backward_common(const rt_star* star, const rt_tol* tol, const ImageC& im, int64_t n, int32_t K,
                                 double* ev, int32_t* nev, double* fin, int32_t* ifin, void* ws,
                                 const rt_schedule* sched, hipStream_t st) {
    rt_schedule sc = resolve_schedule(sched);
    InstT<double> I = make_inst(*star);
    TolC T{tol->rtol, tol->atol, tol->r_max_km, (long long)tol->max_steps};
    FwdWs W = carve_fwd_ws(ws, n);
    double* y0s = (double*)((char*)ws + fwd_ws_bytes(n));
    hipLaunchKernelGGL(zero_ctr_kernel, dim3(1), dim3(64), 0, st, W.ctr);
    if (n == 0) return check_launch("zero_ctr_kernel");
    int grid = grid_for(n, 256, 8);
    hipLaunchKernelGGL(bwd_init_kernel, dim3(grid), dim3(256), 0, st, I, T, im, n, W.ctr, W.list, W.h0, W.k1, y0s, nev);
    int rc = check_launch("bwd_init_kernel");
    if (rc) return rc;
    if (sc.occupancy == 2 && sc.block != 64 && sc.block != 128 && !I.gr_dipole) {
        const int spec = 1 + (I.plasma & 1) + 2 * (I.density & 3) + 8 * (I.oblique ? 1 : 0);
#define RT_BWD_SPEC(S) \
    case S: return launch_bwd_block<256, 2, S>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
        switch (spec) {
            RT_BWD_SPEC(1) RT_BWD_SPEC(2) RT_BWD_SPEC(3) RT_BWD_SPEC(4) RT_BWD_SPEC(5) RT_BWD_SPEC(6)
            RT_BWD_SPEC(7) RT_BWD_SPEC(8) RT_BWD_SPEC(9) RT_BWD_SPEC(10) RT_BWD_SPEC(11) RT_BWD_SPEC(12)
            RT_BWD_SPEC(13) RT_BWD_SPEC(14) RT_BWD_SPEC(15)
            default: return launch_bwd_block<256, 2, 16>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
        }
#undef RT_BWD_SPEC
    }
    if (sc.occupancy == 2) {
        switch (sc.block) {
            case 64: return launch_bwd_block<64, 2>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
            case 128: return launch_bwd_block<128, 2>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
            default: return launch_bwd_block<256, 2>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
        }
    }
    switch (sc.block) {
        case 64: return launch_bwd_block<64, 1>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
        case 128: return launch_bwd_block<128, 1>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
        default: return launch_bwd_block<256, 1>(sc, I, T, im.D, n, W, y0s, K, ev, nev, fin, ifin, st);
    }
}

static void image_axes(double incl, double phi_o, ImageC& im) {
    double si = std::sin(incl), ci = std::cos(incl);
    double sp = std::sin(phi_o), cp = std::cos(phi_o);
    im.no[0] = si * cp; im.no[1] = si * sp; im.no[2] = ci;
    im.e1[0] = ci * cp; im.e1[1] = ci * sp; im.e1[2] = -si;
    im.e2[0] = -sp; im.e2[1] = cp; im.e2[2] = 0.0;
}

}  // namespace rtd

using namespace rtd;

extern "C" int rt_trace_backward(const rt_star* star, const rt_tol* tol, const rt_image* image, int32_t K, double* ev,
                                 int32_t* nev, double* fin, int32_t* ifin, void* ws, size_t ws_bytes,
                                 const rt_schedule* sched, void* stream) {
    clear_error();
    if (!validate_star(star) || !validate_tol(tol)) return RT_EINVAL;
    if (!image) return fail(RT_EINVAL, "rt_trace_backward: null image");
    if (image->nx <= 0 || image->ny <= 0 || !(image->D_km > 0) || !(image->half_width_km > 0) ||
        !std::isfinite(image->D_km) || !std::isfinite(image->incl) || !std::isfinite(image->phi_o) ||
        !std::isfinite(image->half_width_km))
        return fail(RT_EINVAL, "rt_trace_backward: invalid image plane");
    if (image->D_km <= image->half_width_km * 2.0 || image->D_km <= star->R_km)
        return fail(RT_EINVAL, "rt_trace_backward: image plane must lie far outside the star");
    if (K < 0) return fail(RT_EINVAL, "rt_trace_backward: negative K");
    if (star->flags & (RT_FLAG_FLAT_PROPAGATION | RT_FLAG_FINITE_LARMOR))
        return fail(RT_EUNSUPPORTED, "rt_trace_backward: the approximation variants are forward only");
    int64_t n = (int64_t)image->nx * image->ny;
    if (n > INT32_MAX) return fail(RT_EINVAL, "rt_trace_backward: too many pixels");
    if (!nev || !fin || !ifin || (K > 0 && !ev)) return fail(RT_EINVAL, "rt_trace_backward: null array");
    size_t need = rt_workspace_size(RT_OP_TRACE_BACKWARD, n);
    if (!ws || ws_bytes < need) return fail(RT_ENOWS, "rt_trace_backward: workspace too small");
    ImageC im;
    image_axes(image->incl, image->phi_o, im);
    im.D = image->D_km;
    im.db = 2.0 * image->half_width_km / image->nx;
    im.nx = image->nx;
    im.ny = image->ny;
    im.b1 = nullptr;
    im.b2 = nullptr;
    return trace_backward_common(star, tol, im, n, K, ev, nev, fin, ifin, ws, sched, (hipStream_t)stream);
}

extern "C" int rt_trace_backward_rays(const rt_star* star, const rt_tol* tol, double D_km, double incl,
                                      double phi_o, const double* b1, const double* b2, int64_t n, int32_t K,
                                      double* ev, int32_t* nev, double* fin, int32_t* ifin, void* ws,
                                      size_t ws_bytes, const rt_schedule* sched, void* stream) {
    clear_error();
    if (!validate_star(star) || !validate_tol(tol)) return RT_EINVAL;
    if (!(D_km > 0) || !std::isfinite(D_km) || !std::isfinite(incl) || !std::isfinite(phi_o))
        return fail(RT_EINVAL, "rt_trace_backward_rays: invalid image plane");
    if (D_km <= star->R_km) return fail(RT_EINVAL, "rt_trace_backward_rays: image plane must lie outside the star");
    if (K < 0) return fail(RT_EINVAL, "rt_trace_backward_rays: negative K");
    if (star->flags & (RT_FLAG_FLAT_PROPAGATION | RT_FLAG_FINITE_LARMOR))
        return fail(RT_EUNSUPPORTED, "rt_trace_backward_rays: the approximation variants are forward only");
    if (n < 0 || n > INT32_MAX) return fail(RT_EINVAL, "rt_trace_backward_rays: invalid ray count");
    if (n > 0 && (!b1 || !b2 || !nev || !fin || !ifin || (K > 0 && !ev)))
        return fail(RT_EINVAL, "rt_trace_backward_rays: null array");
    size_t need = rt_workspace_size(RT_OP_TRACE_BACKWARD, n);
    if (!ws || ws_bytes < need) return fail(RT_ENOWS, "rt_trace_backward_rays: workspace too small");
    ImageC im;
    image_axes(incl, phi_o, im);
    im.D = D_km;
    im.db = 0.0;
    im.nx = 0;
    im.ny = 0;
    im.b1 = b1;
    im.b2 = b2;
    return trace_backward_common(star, tol, im, n, K, ev, nev, fin, ifin, ws, sched, (hipStream_t)stream);
}

extern "C" int rt_backward_power(const rt_star* star, const double* ev, const int32_t* nev, int64_t n, int32_t K,
                                 double Lc_max_km, const double* area, double pixel_area_km2, double* wsum,
                                 double* total, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!validate_star(star)) return RT_EINVAL;
    if (star->speeds != RT_SPEEDS_MONO)
        return fail(RT_EUNSUPPORTED, "rt_backward_power: the event weights assume monochromatic axions");
    if (star->flags & (RT_FLAG_FLAT_PROPAGATION | RT_FLAG_RENORM_WEIGHTS | RT_FLAG_THIN_SURFACE |
                       RT_FLAG_FINITE_LARMOR))
        return fail(RT_EUNSUPPORTED, "rt_backward_power: the approximation variants are forward only");
    if (n < 0 || K < 0) return fail(RT_EINVAL, "rt_backward_power: negative size");
    if (!std::isfinite(Lc_max_km)) return fail(RT_EINVAL, "rt_backward_power: non-finite cutoff");
    if (!area && !(pixel_area_km2 >= 0.0 && std::isfinite(pixel_area_km2)))
        return fail(RT_EINVAL, "rt_backward_power: invalid pixel area");
    if (n > 0 && (!nev || !wsum || (K > 0 && !ev))) return fail(RT_EINVAL, "rt_backward_power: null array");
    size_t need = rt_workspace_size(RT_OP_BACKWARD_POWER, n);
    if (total && (!ws || ws_bytes < need)) return fail(RT_ENOWS, "rt_backward_power: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    InstT<double> I = make_inst(*star);
    SeedT<double> C = make_seed_consts(*star);
    const double hc = phys::hbarc_eVkm;
    const int nb =
        (int)std::min<int64_t>(POWER_MAX_BLOCKS, std::max<int64_t>(1, (n + POWER_BLOCK - 1) / POWER_BLOCK));
    double* partial = total ? (double*)ws : nullptr;  // block partials of the image sum
    if (n == 0 && !total) return RT_OK;
    timing_begin(st, RT_KERNEL_EVENT_POWER);
    hipLaunchKernelGGL(event_power_kernel, dim3(nb), dim3(POWER_BLOCK), 0, st, I, C, ev, nev, n, K, Lc_max_km, area,
                       pixel_area_km2, wsum, partial);
    timing_end(st);
    int rc = check_launch("event_power_kernel");
    if (rc || !total) return rc;
    hipLaunchKernelGGL(power_total_kernel, dim3(1), dim3(POWER_MAX_BLOCKS), 0, st, (const double*)partial, nb,
                       1.0 / (hc * hc), total);
    return check_launch("power_total_kernel");
}
