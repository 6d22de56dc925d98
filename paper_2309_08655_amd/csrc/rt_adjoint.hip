// Gaussian-smoothed flux and its gradient with respect to the star parameters
// p = (B0, P, theta_m, M, R, m_a) by a hand-written discretise-then-differentiate
// adjoint of the DOPRI5 ray integrator (McDonald & Witte, arXiv:2309.08655: the
// forward estimator of Sec. 2.2 with the conversion weights of Sec. 4, rays of
// Sec. 2 eq. (Hamilton) with the Hamiltonian of Sec. 4.1 eq. (StrongBHam)).
//
//   F_j = (1/N) sum_{escaped i} w_i K(n_i . o_j),  K(c) = exp((c - 1)/sigma^2) / (2 pi sigma^2),
//   n_i = static-frame direction at r = r_max, rotated into the frame co-rotating
//         with the star at the arrival time t - r.
//
// The differentiated map is the one the forward pass computed: the accepted step
// sizes h_n are frozen (the controller is not differentiated), each ray's status
// is frozen, the resonance root, the photon momentum and the weight are
// differentiated through the seeding (forward mode, 6 tangents), the crossing
// r = r_max through the implicit function theorem on the continuous extension,
// and every accepted step through its stages:
//   y_{n+1} = y_n + h sum_i b_i K_i,  K_i = f(Y_i),  Y_i = y_n + h sum_{j<i} a_ij K_j.
// Stage vector-Jacobian products: with f = J grad(H), J = [[0, I], [-I, 0]],
//   v^T df/dy = Hess(H) (J^T v), one directional derivative of the hand-derived
//   gradient in dual numbers, and v^T df/dp through the few instance constants that
//   carry the parameters (a second, three-tangent pass).
// Memory: (y, h, facmax) is checkpointed every C accepted steps into a pool shared by all
// rays (slots handed out in order of need; each ray's checkpoints form a chain from its last
// back to its first), so the pool holds what the rays need, not a worst case; the reverse
// sweep recomputes each segment from its checkpoint into a per-lane replay
// buffer and walks it backwards, one step at a time, with the step's stage states, their
// adjoints and the step's other per-lane vectors in LDS (72 doubles a lane: 36 KB for a wave
// of 64).  This file is compiled with multiply-add fusion
// decided per source expression only (-ffp-contract=on), so the forward pass and the
// recompute, which inline the same step code, produce the same bits; a ray whose
// recompute does not end exactly on its next checkpoint gets a NaN gradient share.
// The per-ray pieces live in rt_adjoint.hpp (also compiled for the host in tests);
// this file holds the workspace layout, the two persistent kernels and the entry.
#include "rt_adjoint.hpp"
#include "rt_common.hpp"

namespace rtd {

constexpr int REV_LANES = 65536;  // lanes of the reverse kernel (one replay buffer each)
constexpr int MAX_OBS = 64;

struct ParamVec {
    double p[6];  // (B0 [G], P [s], theta_m [rad], M [Msun], R [km], m_a [eV])
};

struct AdjWs {
    FwdWs fw;
    double* rays;     // [10][n] seeds
    int32_t* status;  // [n] seed status
    double* fin;      // [RT_NFIN][n] (phase 0): the trace set-up's records of rays it does not trace;
                      // rows 0..7 of an escaped ray: its final state, for the flux kernel
    int32_t* ifin;    // [RT_NIFIN][n]: n_acc, n_rej, status
    int32_t* nseg;    // [n] checkpoints stored
    int32_t* ckhead;  // [n] pool slot of each ray's last checkpoint
    double* theta;    // [n] location of r = r_max on the last step
    double* pool;     // [ckpt_pool][CK_SLOT]: y[8], h, facmax, gjs, slot of the ray's previous checkpoint
    WorkCtr* rctr;    // reverse pass: head of the work list, seal (pad[0]), pool slots asked for
                      // (pad[1]), iters = steps the recompute missed
    double* obs;      // [n_obs][3]
    double* facc;     // [MAX_OBS] flux accumulators
    double* gacc;     // [8] gradient accumulators
    double* replay;   // [C * 11][REV_LANES] (phase 1), over the phase-0-only part of fw and fin
};

constexpr int CK_SLOT = 12;  // doubles per checkpoint slot

static size_t adj_ws_layout(void* base, int64_t n, int32_t n_obs, int32_t C, int64_t ckpt_pool, AdjWs* W) {
    char* p = (char*)base;
    auto take = [&](size_t bytes) {
        char* q = p;
        p += align256(bytes);
        return q;
    };
    // The forward workspace, then the final records (which phase 0 writes: the set-up for seeds
    // it does not trace, the forward kernel for escaped rays): from the forward workspace's transient part on, both are
    // used by phase 0 only, and the replay buffer of phase 1 lies over them (extending past
    // them if it is larger).
    char* fwbase = take(fwd_ws_bytes(n));
    char* fin = take(sizeof(double) * RT_NFIN_ * (size_t)n);
    char* replay = fwbase + fwd_ws_transient_offset(n);
    {
        char* rend = replay + align256(sizeof(double) * 11 * (size_t)C * REV_LANES);
        if (rend > p) p = rend;
    }
    char* rays = take(sizeof(double) * 10 * (size_t)n);
    char* status = take(sizeof(int32_t) * (size_t)n);
    char* ifin = take(sizeof(int32_t) * RT_NIFIN_ * (size_t)n);
    char* nseg = take(sizeof(int32_t) * (size_t)n);
    char* ckhead = take(sizeof(int32_t) * (size_t)n);
    char* theta = take(sizeof(double) * (size_t)n);
    char* pool = take(sizeof(double) * CK_SLOT * (size_t)ckpt_pool);
    char* rctr = take(sizeof(WorkCtr));
    char* obs = take(sizeof(double) * 3 * (size_t)n_obs);
    char* facc = take(sizeof(double) * MAX_OBS);
    char* gacc = take(sizeof(double) * 8);
    if (W) {
        W->fw = carve_fwd_ws(fwbase, n);
        W->rays = (double*)rays;
        W->status = (int32_t*)status;
        W->fin = (double*)fin;
        W->ifin = (int32_t*)ifin;
        W->nseg = (int32_t*)nseg;
        W->ckhead = (int32_t*)ckhead;
        W->theta = (double*)theta;
        W->pool = (double*)pool;
        W->rctr = (WorkCtr*)rctr;
        W->obs = (double*)obs;
        W->facc = (double*)facc;
        W->gacc = (double*)gacc;
        W->replay = (double*)replay;
    }
    return (size_t)(p - (char*)base);
}

// Compile-time forms of the adjoint kernels: the strong-field Hamiltonian with its plasma and
// density switches read at run time (MODE_GENERIC), the finite-magnetisation one
// (MODE_LARMOR), and the strong-field isotropic plasma with the GJ density and the flat dipole
// (MODE_ISO_GJ, the smoothed-flux workload's star; MODE_ISO_GJ_ALIGNED for an aligned rotator),
// whose switches become constants: the right-hand side and the stage products are then
// branch-free, so the compiler can interleave a product's independent passes.  The aligned
// form evaluates the axis without the rotation wherever only values are needed (the same
// values, sin theta_m being zero); the stage products, which carry theta_m tangents, always
// take the rotating formula.  The arithmetic is the same in every form (this file is built
// with -ffp-contract=on), so a star gives the same bits whichever form traces it.
constexpr int MODE_GENERIC = 0, MODE_LARMOR = 1, MODE_ISO_GJ = 2, MODE_ISO_GJ_ALIGNED = 3;

template <int MODE>
__device__ __forceinline__ void fix_mode(InstT<double>& I) {
    I.larmor = (MODE == MODE_LARMOR) ? 1 : 0;
    // the rotating-axis formula (as the entry point sets it), but for an aligned rotator
    I.oblique = (MODE == MODE_ISO_GJ_ALIGNED) ? 0 : 1;
    if constexpr (MODE == MODE_ISO_GJ || MODE == MODE_ISO_GJ_ALIGNED) {
        I.plasma = PL_ISO;
        I.density = DEN_GJ;
        I.gr_dipole = 0;
    }
}

static int adj_mode(const InstT<double>& I) {
    if (I.larmor) return MODE_LARMOR;
    if (I.plasma == PL_ISO && I.density == DEN_GJ && !I.gr_dipole)
        return (I.sm == 0.0) ? MODE_ISO_GJ_ALIGNED : MODE_ISO_GJ;
    return MODE_GENERIC;
}

constexpr int ADJ_REFILL_MIN = 4;

// forward pass: persistent, one ray per lane with wave-aggregated refill from the
// cost-ordered work list; checkpoints, per-ray counters, and the final state of each escaped
// ray in fin (rows 0..7), from which adj_flux_kernel forms the flux outside this loop (the
// observer sum of a finishing lane would hold its whole wave).  Each checkpoint takes
// the next free pool slot (one atomic per wave for the lanes storing together) and links
// to the ray's previous one; a request beyond the pool is counted but not stored (the
// count then tells the caller the pool it needs, and the reverse pass refuses to run).
// MODE fixes the Hamiltonian's switches at compile time (fix_mode below).
template <int MODE>
__global__ void __launch_bounds__(256, 2) adj_fwd_kernel(InstT<double> I, TolC tol, int64_t n, WorkCtr* ctr,
                                                      const int32_t* __restrict__ list, const double* __restrict__ rays,
                                                      const double* __restrict__ y0q, const double* __restrict__ h0s,
                                                      int C, int Kc, double* __restrict__ pool,
                                                      long long ckpt_pool, int32_t* __restrict__ ckhead,
                                                      unsigned long long* __restrict__ pool_next,
                                                      int32_t* __restrict__ nseg_out,
                                                      double* __restrict__ theta_out, int32_t* __restrict__ ifin,
                                                      double* __restrict__ fin) {
    constexpr bool LARMOR = (MODE == MODE_LARMOR);
    fix_mode<MODE>(I);
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long nlist = ctr->len;
    bool active = false, exhausted = false;
    int64_t j = 0;
    int32_t head = -1;  // pool slot of the ray's last checkpoint (-2: a request found the pool full)
    AdjRay R;
    auto store = [&](int s, const double* y, double h, double facmax, double gjs) {
        const unsigned long long storing = __ballot(1);
        const int leader = __ffsll((long long)storing) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(pool_next, (unsigned long long)__popcll(storing));
        base = __shfl(base, leader);
        const unsigned long long slot = base + (unsigned long long)__popcll(storing & below);
        if (s == 0) head = -1;
        if (slot < (unsigned long long)ckpt_pool && head != -2) {
            double* c = pool + (int64_t)slot * CK_SLOT;
            for (int d = 0; d < 8; ++d) c[d] = y[d];
            c[8] = h;
            c[9] = facmax;
            c[10] = gjs;
            c[11] = (double)head;
            head = (int32_t)slot;
        } else {
            head = -2;
        }
    };
    while (true) {
        unsigned long long idle = __ballot(!active);
        // refill once four lanes are idle (or the whole wave): one atomic and one pass of
        // the start-up code for several lanes, as in the tracing kernels
        if (idle && !exhausted && (__popcll(idle) >= ADJ_REFILL_MIN || idle == __ballot(true))) {
            int cnt = __popcll(idle);
            int leader = __ffsll((long long)idle) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(&ctr->head, (unsigned long long)cnt);
            base = __shfl(base, leader);
            if (!active) {
                unsigned long long qq = base + __popcll(idle & below);
                if (qq < nlist) {
                    j = list[qq];
                    double y0[8];
                    for (int d = 0; d < 8; ++d) y0[d] = y0q[d * n + qq];  // seed states in list order
                    adj_ray_start<LARMOR>(I, y0, h0s[qq], R, store);
                    active = true;
                }
            }
            if (base + (unsigned long long)cnt >= nlist) exhausted = true;
        }
        if (__ballot(active) == 0ull) {
            if (exhausted) break;
            continue;
        }
        if (!active) continue;
        double yf[8], th = 0.0;
        const int status = adj_ray_step<LARMOR>(I, tol, C, Kc, R, store, yf, &th);
        if (status != ST_OK) {
            ifin[j] = R.nacc;
            ifin[n + j] = R.nrej;
            ifin[2 * n + j] = status;
            nseg_out[j] = R.nseg;
            ckhead[j] = head;
            if (status == ST_ESCAPED) {
                theta_out[j] = th;
                for (int d = 0; d < 8; ++d) fin[d * n + j] = yf[d];
            }
            active = false;
        }
    }
}

// Smoothed flux of the forward pass, Sec. 2.2 eq. (Power) smoothed on the sky:
// F_o += w_j K(n_j . o) over the escaped rays (final states in fin rows 0..7, arrival
// direction n_j), summed across each wave by shuffles, per workgroup in LDS, then over
// workgroups with one atomic per observer.  The ray loop's bound is the workgroup's, so
// every lane of a wave takes part in each shuffle.
__global__ void __launch_bounds__(256) adj_flux_kernel(InstT<double> I, const double* __restrict__ fin,
                                                       const int32_t* __restrict__ ifin,
                                                       const double* __restrict__ rays, int64_t n,
                                                       const double* __restrict__ obs, int n_obs, double sigma,
                                                       double* __restrict__ facc) {
    __shared__ double sh_f[MAX_OBS];
    for (int q = threadIdx.x; q < MAX_OBS; q += blockDim.x) sh_f[q] = 0.0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t j = base + threadIdx.x;
        const bool esc = (j < n) && ifin[2 * n + j] == ST_ESCAPED;
        double nh[3] = {0.0, 0.0, 0.0}, w = 0.0;
        if (esc) {
            double yf[8];
            for (int d = 0; d < 8; ++d) yf[d] = fin[d * n + j];
            arrival_direction(I, yf, nh);
            w = rays[8 * n + j];
        }
        for (int o = 0; o < n_obs; ++o) {
            const double c = nh[0] * obs[3 * o] + nh[1] * obs[3 * o + 1] + nh[2] * obs[3 * o + 2];
            double v = esc ? w * smoothing_kernel(c, sigma) : 0.0;
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (__lane_id() == 0 && v != 0.0) atomicAdd(&sh_f[o], v);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_obs; q += blockDim.x)
        if (sh_f[q] != 0.0) atomicAdd(&facc[q], sh_f[q]);
}

// Reverse work list: escaped rays ordered by accepted steps, longest first, so that the
// 64 rays a wave takes together have (nearly) the same segment and step counts and
// its lanes walk them in lockstep.
__global__ void adj_rev_keys_kernel(const int32_t* __restrict__ ifin, int64_t n, int32_t* __restrict__ keys) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const int32_t na = ifin[j];
        keys[j] = (ifin[2 * n + j] == ST_ESCAPED)
                      ? (ORDER_BUCKETS - 1) - (na < ORDER_BUCKETS - 1 ? (na > 0 ? na : 0) : ORDER_BUCKETS - 1)
                      : -1;
    }
}

__global__ void adj_scale_kernel(const double* acc, int m, double s, double* out) {
    for (int q = threadIdx.x; q < m; q += blockDim.x) out[q] = acc[q] * s;
}

// Seal of a completed forward phase: a word derived from the arguments that shape the
// workspace.  The reverse kernel does nothing unless it finds the seal of its own
// arguments (a reverse call on a workspace without its forward phase, or after a forward
// phase whose checkpoints did not fit the pool).
static unsigned long long adj_seal(int64_t n, int32_t n_obs, int32_t C, int32_t Kc, int64_t ckpt_pool) {
    unsigned long long h = 0x9e3779b97f4a7c15ull;
    const unsigned long long v[5] = {(unsigned long long)n, (unsigned long long)n_obs, (unsigned long long)C,
                                     (unsigned long long)Kc, (unsigned long long)ckpt_pool};
    for (int i = 0; i < 5; ++i) h = (h ^ v[i]) * 0x100000001b3ull;
    return h;
}

// seals the forward phase if its checkpoints fit the pool; reports the slots asked for
__global__ void adj_set_seal_kernel(WorkCtr* rctr, unsigned long long seal, long long ckpt_pool,
                                    long long* ckpt_used) {
    if (threadIdx.x == 0) {
        const unsigned long long asked = rctr->pad[1];
        rctr->pad[0] = (asked <= (unsigned long long)ckpt_pool) ? seal : 0ull;
        if (ckpt_used) *ckpt_used = (long long)asked;
    }
}

__global__ void adj_bad_seal_kernel(const WorkCtr* rctr, unsigned long long seal, double* grad) {
    if (threadIdx.x < 6 && rctr->pad[0] != seal) grad[threadIdx.x] = __builtin_nan("");
}

__global__ void adj_clear_kernel(double* facc, double* gacc, WorkCtr* rctr, int clear_list) {
    for (int q = threadIdx.x; q < MAX_OBS; q += blockDim.x) facc[q] = 0.0;
    for (int q = threadIdx.x; q < 8; q += blockDim.x) gacc[q] = 0.0;
    if (threadIdx.x == 0) {
        rctr->head = 0ull;
        rctr->iters = 0ull;
        if (clear_list) {
            rctr->len = 0ull;
            rctr->pad[0] = 0ull;
            rctr->pad[1] = 0ull;
        }
    }
}

// This lane's index in the wave (the reverse kernel's blocks are one wave, so also its thread
// index), recomputed where the LDS rows are addressed: held in a register across the sweep it
// is spilled to scratch, and every row access then waits on a reload.
__device__ inline int lane_now() {
    int r;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(r));
    return r;
}

// reverse pass: one escaped ray per lane, handed out by a lane atomic (MODE as above)
template <int MODE>
__global__ void __launch_bounds__(64) adj_rev_kernel(InstT<double> I, ParamVec P, StarFixed fx, TolC tol,
                                                     uint64_t seed, int64_t n, const double* __restrict__ rays,
                                                     const int32_t* __restrict__ ifin,
                                                     const int32_t* __restrict__ nseg_in,
                                                     const double* __restrict__ theta_in,
                                                     const double* __restrict__ pool, long long ckpt_pool,
                                                     const int32_t* __restrict__ ckhead, int C, WorkCtr* rctr,
                                                     const WorkCtr* lctr, const int32_t* __restrict__ rlist,
                                                     const double* __restrict__ obs,
                                                     int n_obs, double sigma, const double* __restrict__ gbar,
                                                     double* __restrict__ replay, double* __restrict__ gacc,
                                                     double* __restrict__ grad_rays, double inv_n, int Kc,
                                                     unsigned long long seal) {
    if (rctr->pad[0] != seal) return;  // no forward phase of these arguments in this workspace
    constexpr bool LARMOR = (MODE == MODE_LARMOR);
    fix_mode<MODE>(I);
    AdjParams A;
    make_adj_params(P.p, fx, A);
    double pacc[6] = {0, 0, 0, 0, 0, 0};
    unsigned long long missing = 0;
    const unsigned long long rlen = lctr->len < (unsigned long long)n ? lctr->len : (unsigned long long)n;
    // the replay buffer, addressed from a fresh lane index too: a spilled address would be
    // reloaded just after the one-step-ahead loads, and waiting for that reload would wait
    // for them
    auto rb = [&](int idx, int d) -> double& {
        return replay[((int64_t)idx * 11 + d) * REV_LANES + (int64_t)blockIdx.x * 64 + lane_now()];
    };
    // the walked step's rows in LDS (one wave a block: 36 KB, so that four blocks, one a
    // SIMD, fit a CU's 160 KB)
    __shared__ double lsh[LR_SLOTS * 64];
    auto lr = [&](int r) { return LaneRow<double, 64>{lsh + r * 512 + lane_now()}; };
    const int lane = __lane_id();
    while (true) {
        // the wave takes 64 consecutive rays of the step-ordered list
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&rctr->head, 64ull);
        base = __shfl(base, 0);
        if (base >= rlen) break;
        const unsigned long long qq = base + (unsigned long long)lane;
        if (qq >= rlen) continue;
        const int64_t j = rlist[qq];
        if (j < 0 || j >= n) continue;
        const int S = ifin[j], nseg = nseg_in[j];
        if (nseg < 1 || nseg > Kc || S < 1 || S > nseg * C) continue;
        // the sweep reads checkpoint s, then s + 1 (the end check), then s - 1 ...: walk the
        // ray's chain from its last checkpoint back, keeping the slot of the one after
        int32_t cur = ckhead[j], nxt = -1;
        int cur_s = nseg - 1;
        bool chain_ok = true;
        auto in_pool = [&](int32_t sl) { return sl >= 0 && (long long)sl < ckpt_pool; };
        auto load = [&](int s, double* y, double* h, double* facmax, double* gjs) {
            if (s == cur_s - 1) {
                nxt = cur;
                cur = in_pool(cur) ? (int32_t)pool[(int64_t)cur * CK_SLOT + 11] : -1;
                cur_s = s;
            }
            const int32_t sl = (s == cur_s) ? cur : ((s == cur_s + 1) ? nxt : -1);
            if (!in_pool(sl)) {
                chain_ok = false;
                for (int d = 0; d < 8; ++d) y[d] = __builtin_nan("");
                *h = __builtin_nan("");
                *facmax = 10.0;
                *gjs = 0.0;
                return;
            }
            const double* c = pool + (int64_t)sl * CK_SLOT;
            for (int d = 0; d < 8; ++d) y[d] = c[d];
            *h = c[8];
            *facmax = c[9];
            *gjs = c[10];
        };
        double pb[6] = {0, 0, 0, 0, 0, 0};
        int miss = adj_reverse_ray<LARMOR, MODE == MODE_ISO_GJ || MODE == MODE_ISO_GJ_ALIGNED>(I, A, tol, seed, j, S, nseg, theta_in[j], rays[8 * n + j], C, load, rb, lr,
                                           obs, gbar, n_obs, sigma, pb);
        if (!chain_ok) ++miss;
        if (miss) {
            // the recompute did not reproduce the forward pass: no gradient for this ray
            missing += (unsigned long long)miss;
            for (int q = 0; q < 6; ++q) pb[q] = __builtin_nan("");
        }
        for (int q = 0; q < 6; ++q) pacc[q] += pb[q];
        if (grad_rays)
            for (int q = 0; q < 6; ++q) grad_rays[j * 6 + q] = pb[q] * inv_n;
    }
    for (int q = 0; q < 6; ++q) {
        double v = pacc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (threadIdx.x == 0) atomicAdd(&gacc[q], v);
    }
    if (missing) atomicAdd(&rctr->iters, missing);
}

template <int MODE>
static void launch_adj_fwd(int grid, hipStream_t st, const InstT<double>& I, const TolC& T, int64_t n, const AdjWs& W,
                           int C, int Kc, int64_t ckpt_pool, unsigned long long* pool_next) {
    hipLaunchKernelGGL(adj_fwd_kernel<MODE>, dim3(grid), dim3(256), 0, st, I, T, n, W.fw.ctr, W.fw.list, W.rays,
                       W.fw.y0, W.fw.h0, C, Kc, W.pool, (long long)ckpt_pool, W.ckhead, pool_next, W.nseg, W.theta,
                       W.ifin, W.fin);
}

template <int MODE>
static void launch_adj_rev(hipStream_t st, const InstT<double>& I, const ParamVec& P, const StarFixed& fx,
                           const TolC& T, uint64_t seed, int64_t n, const AdjWs& W, int C, int Kc, int64_t ckpt_pool,
                           int n_obs, double sigma, const double* gbar, double* grad_rays, unsigned long long seal) {
    hipLaunchKernelGGL(adj_rev_kernel<MODE>, dim3(REV_LANES / 64), dim3(64), 0, st, I, P, fx, T, seed, n, W.rays,
                       W.ifin, W.nseg, W.theta, W.pool, (long long)ckpt_pool, W.ckhead, C, W.rctr, W.fw.ctr,
                       W.fw.list, W.obs, n_obs, sigma, gbar, W.replay, W.gacc, grad_rays, 1.0 / (double)n, Kc, seal);
}

}  // namespace rtd

using namespace rtd;

extern "C" size_t rt_flux_grad_workspace_size(int64_t n, int32_t n_obs, int32_t ckpt_every, int64_t ckpt_pool) {
    if (n < 0 || n_obs <= 0 || n_obs > MAX_OBS || ckpt_every <= 0 || ckpt_pool <= 0 || ckpt_pool > INT32_MAX)
        return 0;
    return adj_ws_layout(nullptr, n, n_obs, ckpt_every, ckpt_pool, nullptr);
}

__global__ void adj_ray_info_kernel(const int32_t* __restrict__ ifin, int64_t n, int32_t* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += stride) out[i] = ifin[i];
}

extern "C" int rt_flux_grad(const rt_star* star, const rt_tol* tol, uint64_t seed, int64_t n, const double* obs,
                            int32_t n_obs, double sigma, int32_t ckpt_every, int32_t max_ckpt, int64_t ckpt_pool,
                            int32_t phase, const double* gbar, double* flux, double* grad, double* grad_rays,
                            int32_t* ray_info, int64_t* ckpt_used, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!validate_star(star) || !validate_tol(tol)) return RT_EINVAL;
    if (n <= 0 || n > INT32_MAX) return fail(RT_EINVAL, "rt_flux_grad: n must be in [1, 2^31 - 1]");
    if (n_obs <= 0 || n_obs > MAX_OBS || !obs) return fail(RT_EINVAL, "rt_flux_grad: 1 <= n_obs <= 64 observers");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(RT_EINVAL, "rt_flux_grad: sigma must be positive");
    if (ckpt_every <= 0 || ckpt_every > 1024 || max_ckpt <= 0)
        return fail(RT_EINVAL, "rt_flux_grad: need 1 <= ckpt_every <= 1024 and max_ckpt >= 1");
    if (ckpt_pool <= 0 || ckpt_pool > INT32_MAX)
        return fail(RT_EINVAL, "rt_flux_grad: need 1 <= ckpt_pool <= 2^31 - 1");
    if (star->weights == RT_WEIGHTS_CONST_B) return fail(RT_EUNSUPPORTED, "rt_flux_grad: constant-B test weights");
    if (star->flags & RT_FLAG_FLAT_PROPAGATION)
        return fail(RT_EUNSUPPORTED, "rt_flux_grad: flat-propagation variant");
    if (phase != 0 && phase != 1) return fail(RT_EINVAL, "rt_flux_grad: phase must be 0 (forward) or 1 (reverse)");
    const size_t need = rt_flux_grad_workspace_size(n, n_obs, ckpt_every, ckpt_pool);
    if (!ws || ws_bytes < need) return fail(RT_ENOWS, "rt_flux_grad: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    AdjWs W;
    adj_ws_layout(ws, n, n_obs, ckpt_every, ckpt_pool, &W);
    unsigned long long* pool_next = &W.rctr->pad[1];
    InstT<double> I = make_inst(*star);
    // the rotating-axis formula (exact at theta_m = 0, and theta_m tangents flow); the aligned
    // isotropic GJ form leaves it out where only values are needed
    I.oblique = 1;
    TolC T{tol->rtol, tol->atol, tol->r_max_km, (long long)tol->max_steps};
    if (phase == 0) {
        if (!flux) return fail(RT_EINVAL, "rt_flux_grad: null flux");
        if (hipMemcpyAsync(W.obs, obs, sizeof(double) * 3 * n_obs, hipMemcpyHostToDevice, st) != hipSuccess)
            return fail(RT_EHIP, "rt_flux_grad: observer upload failed");
        hipLaunchKernelGGL(adj_clear_kernel, dim3(1), dim3(64), 0, st, W.facc, W.gacc, W.rctr, 1);
        int rc = check_launch("adj_clear_kernel");
        if (rc) return rc;
        rc = rt_sample_resonance(star, seed, 0, 0, n, W.rays, W.status, stream);
        if (rc) return rc;
        rc = launch_trace_init(I, nullptr, nullptr, T, W.rays, W.status, n, W.fw, W.fin, W.ifin, st);
        if (rc) return rc;
        const rt_schedule sc = resolve_schedule(nullptr);
        const int mode = adj_mode(I);
        const void* fk = (mode == MODE_LARMOR)           ? (const void*)adj_fwd_kernel<MODE_LARMOR>
                         : (mode == MODE_ISO_GJ)         ? (const void*)adj_fwd_kernel<MODE_ISO_GJ>
                         : (mode == MODE_ISO_GJ_ALIGNED) ? (const void*)adj_fwd_kernel<MODE_ISO_GJ_ALIGNED>
                                                         : (const void*)adj_fwd_kernel<MODE_GENERIC>;
        const int grid = persistent_grid(sc, fk, 256);
        timing_begin(st, RT_KERNEL_ADJOINT_FORWARD);
        if (mode == MODE_LARMOR)
            launch_adj_fwd<MODE_LARMOR>(grid, st, I, T, n, W, ckpt_every, max_ckpt, ckpt_pool, pool_next);
        else if (mode == MODE_ISO_GJ)
            launch_adj_fwd<MODE_ISO_GJ>(grid, st, I, T, n, W, ckpt_every, max_ckpt, ckpt_pool, pool_next);
        else if (mode == MODE_ISO_GJ_ALIGNED)
            launch_adj_fwd<MODE_ISO_GJ_ALIGNED>(grid, st, I, T, n, W, ckpt_every, max_ckpt, ckpt_pool, pool_next);
        else
            launch_adj_fwd<MODE_GENERIC>(grid, st, I, T, n, W, ckpt_every, max_ckpt, ckpt_pool, pool_next);
        timing_end(st);
        rc = check_launch("adj_fwd_kernel");
        if (rc) return rc;
        hipLaunchKernelGGL(adj_flux_kernel, dim3(grid_for(n, 256, 2)), dim3(256), 0, st, I, W.fin, W.ifin, W.rays, n,
                           W.obs, n_obs, sigma, W.facc);
        rc = check_launch("adj_flux_kernel");
        if (rc) return rc;
        // the forward list is spent: reuse its buffers for the step-ordered reverse list
        hipLaunchKernelGGL(adj_rev_keys_kernel, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.ifin, n, W.fw.keys);
        rc = check_launch("adj_rev_keys_kernel");
        if (rc) return rc;
        rc = order_work_list(W.fw, n, st);
        if (rc) return rc;
        hipLaunchKernelGGL(adj_scale_kernel, dim3(1), dim3(64), 0, st, W.facc, n_obs, 1.0 / (double)n, flux);
        hipLaunchKernelGGL(adj_set_seal_kernel, dim3(1), dim3(64), 0, st, W.rctr,
                           adj_seal(n, n_obs, ckpt_every, max_ckpt, ckpt_pool), (long long)ckpt_pool,
                           (long long*)ckpt_used);
        rc = check_launch("adj_set_seal_kernel");
        if (rc || !ray_info) return rc;
        hipLaunchKernelGGL(adj_ray_info_kernel, dim3(grid_for(3 * n, 256, 8)), dim3(256), 0, st, W.ifin, n, ray_info);
        return check_launch("adj_ray_info_kernel");
    }
    if (!gbar || !grad) return fail(RT_EINVAL, "rt_flux_grad: null gbar or grad");
    hipLaunchKernelGGL(adj_clear_kernel, dim3(1), dim3(64), 0, st, W.facc, W.gacc, W.rctr, 0);
    int rc = check_launch("adj_clear_kernel");
    if (rc) return rc;
    if (grad_rays) {
        hipLaunchKernelGGL(fill_kernel, dim3(grid_for(6 * n, 256, 8)), dim3(256), 0, st, grad_rays, 6 * n, 0.0);
        rc = check_launch("fill_kernel");
        if (rc) return rc;
    }
    const unsigned long long seal = adj_seal(n, n_obs, ckpt_every, max_ckpt, ckpt_pool);
    ParamVec P{{star->B0_G, star->P_s, star->theta_m, star->M_Msun, star->R_km, star->m_a_eV}};
    StarFixed fx = star_fixed(*star);
    timing_begin(st, RT_KERNEL_ADJOINT_REVERSE);
    const int mode = adj_mode(I);
    if (mode == MODE_LARMOR)
        launch_adj_rev<MODE_LARMOR>(st, I, P, fx, T, seed, n, W, ckpt_every, max_ckpt, ckpt_pool, n_obs, sigma, gbar,
                                    grad_rays, seal);
    else if (mode == MODE_ISO_GJ)
        launch_adj_rev<MODE_ISO_GJ>(st, I, P, fx, T, seed, n, W, ckpt_every, max_ckpt, ckpt_pool, n_obs, sigma, gbar,
                                    grad_rays, seal);
    else if (mode == MODE_ISO_GJ_ALIGNED)
        launch_adj_rev<MODE_ISO_GJ_ALIGNED>(st, I, P, fx, T, seed, n, W, ckpt_every, max_ckpt, ckpt_pool, n_obs, sigma,
                                            gbar, grad_rays, seal);
    else
        launch_adj_rev<MODE_GENERIC>(st, I, P, fx, T, seed, n, W, ckpt_every, max_ckpt, ckpt_pool, n_obs, sigma, gbar,
                                     grad_rays, seal);
    timing_end(st);
    rc = check_launch("adj_rev_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(adj_scale_kernel, dim3(1), dim3(64), 0, st, W.gacc, 6, 1.0 / (double)n, grad);
    hipLaunchKernelGGL(adj_bad_seal_kernel, dim3(1), dim3(64), 0, st, W.rctr, seal, grad);
    return check_launch("adj_bad_seal_kernel");
}
