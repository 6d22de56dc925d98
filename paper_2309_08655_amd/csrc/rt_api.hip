// Host side of the C ABI: validation, constants, schedules, workspace sizes,
// error strings.
#include "rt_common.hpp"
#include <mutex>

#include <string>

namespace rtd {

static thread_local std::string g_err;

void set_error(const char* msg) { g_err = msg ? msg : ""; }
void clear_error() { g_err.clear(); }

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::string m = std::string(what) + ": " + hipGetErrorString(e);
        set_error(m.c_str());
        return RT_EHIP;
    }
    return RT_OK;
}

static bool finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool validate_star(const rt_star* s) {
    if (!s) { set_error("null rt_star"); return false; }
    double v[12] = {s->B0_G, s->P_s, s->theta_m, s->M_Msun, s->R_km, s->m_a_eV,
                    s->g_agg_GeV, s->v0_kms, s->rho_GeVcm3, s->multiplicity, s->psi_twist, s->B_test_G};
    if (!finite_all(v, 12)) { set_error("rt_star: non-finite parameter"); return false; }
    if (!(s->B0_G > 0 && s->P_s > 0 && s->R_km > 0 && s->m_a_eV > 0 && s->v0_kms > 0 && s->rho_GeVcm3 > 0 &&
          s->multiplicity > 0)) {
        set_error("rt_star: B0, P, R, m_a, v0, rho and multiplicity must be positive");
        return false;
    }
    if (!(2.0 * phys::GMsun_km * s->M_Msun < s->R_km)) {
        set_error("rt_star: the star must be larger than its Schwarzschild radius");
        return false;
    }
    if (s->plasma < 0 || s->plasma > 1 || s->density < 0 || s->density > 3 || s->weights < 0 || s->weights > 2 ||
        s->kdir < 0 || s->kdir > 1 || s->speeds < 0 || s->speeds > 1 || (s->flags & ~63) != 0) {
        set_error("rt_star: enumeration out of range");
        return false;
    }
    if ((s->flags & RT_FLAG_FINITE_LARMOR) && s->plasma != RT_PLASMA_ANISO) {
        set_error("rt_star: finite magnetisation needs the anisotropic (magnetised) plasma");
        return false;
    }
    if ((s->flags & RT_FLAG_FINITE_LARMOR) && (s->flags & RT_FLAG_THIN_SURFACE)) {
        set_error("rt_star: finite magnetisation is not combined with the thin-surface variant (unsupported)");
        return false;
    }
    return true;
}

bool validate_tol(const rt_tol* t) {
    if (!t) { set_error("null rt_tol"); return false; }
    if (!(std::isfinite(t->rtol) && t->rtol > 0 && std::isfinite(t->atol) && t->atol > 0 &&
          std::isfinite(t->r_max_km) && t->r_max_km > 0 && t->max_steps > 0)) {
        set_error("rt_tol: rtol, atol, r_max must be positive and finite, max_steps positive");
        return false;
    }
    if (t->max_steps > INT32_MAX) { set_error("rt_tol: max_steps exceeds 2^31 - 1"); return false; }
    return true;
}

StarFixed star_fixed(const rt_star& s) {
    StarFixed f;
    f.g_agg_GeV = s.g_agg_GeV;
    f.v0_kms = s.v0_kms;
    f.rho_GeVcm3 = s.rho_GeVcm3;
    f.multiplicity = s.multiplicity;
    f.psi_twist = s.psi_twist;
    f.B_test_G = s.B_test_G;
    f.plasma = s.plasma;
    f.density = s.density;
    f.weights = s.weights;
    f.kdir = s.kdir;
    f.speeds = s.speeds;
    f.flags = s.flags;
    return f;
}

InstT<double> make_inst(const rt_star& s) {
    double p[6] = {s.B0_G, s.P_s, s.theta_m, s.M_Msun, s.R_km, s.m_a_eV};
    return make_inst_t<double>(p, star_fixed(s));
}

SeedT<double> make_seed_consts(const rt_star& s) {
    double p[6] = {s.B0_G, s.P_s, s.theta_m, s.M_Msun, s.R_km, s.m_a_eV};
    return make_seed_t<double>(p, star_fixed(s));
}

int device_cu_count() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

rt_schedule resolve_schedule(const rt_schedule* s) {
    rt_schedule r;
    r.block = 256;
    r.waves_per_cu = 0;
    r.refill_min = 4;
    r.occupancy = 2;
    r.cross_batch = 8;
    r.chunk = 0;
    if (s) {
        if (s->block == 64 || s->block == 128 || s->block == 256) r.block = s->block;
        if (s->waves_per_cu > 0 && s->waves_per_cu <= 32) r.waves_per_cu = s->waves_per_cu;
        if (s->refill_min >= 1 && s->refill_min <= 64) r.refill_min = s->refill_min;
        if (s->occupancy == 1 || s->occupancy == 2) r.occupancy = s->occupancy;
        if (s->cross_batch >= 1 && s->cross_batch <= 64) r.cross_batch = s->cross_batch;
        if (s->chunk >= 64 && s->chunk <= 65536) r.chunk = s->chunk;
    }
    return r;
}

int persistent_grid(const rt_schedule& sc, const void* kernel, int block) {
    int cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    if (sc.waves_per_cu > 0) {
        int want = (sc.waves_per_cu * 64 + block - 1) / block;
        if (want < per_cu) per_cu = want;
        if (per_cu < 1) per_cu = 1;
    }
    return cus * per_cu;
}

// ---------------------------------------------------------------------------
// partition: counting sort of indices by bucket, without per-element global atomics
// ---------------------------------------------------------------------------
// Workgroup g owns the contiguous chunk [g c, (g+1) c) of the keys.  Pass 1 counts its
// chunk per bucket in LDS and writes the counts as row g of tab (G x nb).  Pass 2 turns
// every column of tab into exclusive offsets over g and emits the column totals; pass 3
// scans the totals into bucket starts.  Pass 4 re-reads the chunk and places element i
// at start[b] + tab[g][b] + (its rank among the chunk's elements of bucket b, from an LDS
// counter).  Element i belongs to bucket keys[i] >> shift when keys[i] >= 0 and that
// bucket is below nb; every other element is left out of the list.

static __global__ void __launch_bounds__(256) part_hist_kernel(const int32_t* __restrict__ keys, int64_t n,
                                                                int64_t chunk, int shift, int nb,
                                                                int32_t* __restrict__ tab) {
    __shared__ int32_t sh[PART_BUCKETS];
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sh[b] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const int32_t k = keys[i];
        if (k >= 0 && (k >> shift) < nb) atomicAdd(&sh[k >> shift], 1);
    }
    __syncthreads();
    int32_t* row = tab + (int64_t)blockIdx.x * nb;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) row[b] = sh[b];
}

// 64 buckets per workgroup (one per lane); its 16 waves split the G rows in 16 slices
static __global__ void __launch_bounds__(1024) part_cols_kernel(int32_t* __restrict__ tab, int G, int nb,
                                                                 int32_t* __restrict__ totals) {
    constexpr int NW = 16;
    __shared__ int32_t part[NW][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + lane;
    const int g0 = (G * wv) / NW, g1 = (G * (wv + 1)) / NW;
    int32_t s = 0;
    if (b < nb)
        for (int g = g0; g < g1; ++g) s += tab[(int64_t)g * nb + b];
    part[wv][lane] = s;
    __syncthreads();
    int32_t run = 0;
    for (int q = 0; q < wv; ++q) run += part[q][lane];
    if (b < nb)
        for (int g = g0; g < g1; ++g) {
            const int32_t c = tab[(int64_t)g * nb + b];
            tab[(int64_t)g * nb + b] = run;
            run += c;
        }
    if (wv == NW - 1 && b < PART_BUCKETS) totals[b] = (b < nb) ? run : 0;
}

// exclusive prefix sum of the PART_BUCKETS totals in place (one workgroup of 1024 threads,
// 4 buckets each); start[PART_BUCKETS] receives the list length.  With a work counter, the
// list is also armed for a persistent kernel: length set, head and iteration count cleared.
static __global__ void __launch_bounds__(1024) part_scan_kernel(int32_t* start, WorkCtr* ctr) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    int32_t v[4], s = 0;
    for (int q = 0; q < 4; ++q) { v[q] = start[4 * t + q]; s += v[q]; }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t add = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int32_t base = part[t] - s;
    for (int q = 0; q < 4; ++q) { start[4 * t + q] = base; base += v[q]; }
    if (t == 1023) {
        start[PART_BUCKETS] = part[1023];
        if (ctr) {
            ctr->head = 0ull;
            ctr->len = (unsigned long long)part[1023];
            ctr->iters = 0ull;
            ctr->pad[1] = 0ull;
        }
    }
}

static __global__ void __launch_bounds__(256) part_scatter_kernel(const int32_t* __restrict__ keys, int64_t n,
                                                                   int64_t chunk, int shift, int nb,
                                                                   const int32_t* __restrict__ tab,
                                                                   const int32_t* __restrict__ start,
                                                                   int32_t* __restrict__ list) {
    __shared__ int32_t sh[PART_BUCKETS];
    __shared__ int32_t base[PART_BUCKETS];
    const int32_t* row = tab + (int64_t)blockIdx.x * nb;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        sh[b] = 0;
        base[b] = start[b] + row[b];
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const int32_t k = keys[i];
        if (k >= 0 && (k >> shift) < nb) {
            const int b = k >> shift;
            list[base[b] + atomicAdd(&sh[b], 1)] = (int32_t)i;
        }
    }
}

int partition_keys(const int32_t* keys, int64_t n, int shift, int nb, int32_t* tab, int32_t* start,
                   int32_t* list, WorkCtr* ctr, hipStream_t st) {
    if (nb < 1 || nb > PART_BUCKETS || n < 0 || n > INT32_MAX)
        return fail(RT_EINVAL, "partition_keys: bucket count or length out of range");
    const int G = partition_blocks(n);
    const int64_t chunk = (n + G - 1) / G;
    hipLaunchKernelGGL(part_hist_kernel, dim3(G), dim3(256), 0, st, keys, n, chunk, shift, nb, tab);
    hipLaunchKernelGGL(part_cols_kernel, dim3(PART_BUCKETS / 64), dim3(1024), 0, st, tab, G, nb, start);
    hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, st, start, ctr);
    hipLaunchKernelGGL(part_scatter_kernel, dim3(G), dim3(256), 0, st, keys, n, chunk, shift, nb, tab, start, list);
    return check_launch("partition_keys");
}

int order_work_list(const FwdWs& W, int64_t n, hipStream_t st) {
    static_assert(ORDER_BUCKETS == PART_BUCKETS, "the work list uses one bucket per partition slot");
    return partition_keys(W.keys, n, 0, ORDER_BUCKETS, W.tab, W.buckets, W.list, W.ctr, st);
}

}  // namespace rtd

using namespace rtd;

extern "C" size_t rt_workspace_size(int32_t op, int64_t n) {
    if (n < 0) n = 0;
    switch (op) {
        case RT_OP_TRACE_FORWARD:
        case RT_OP_BATCHED:
            return fwd_ws_bytes(n);
        case RT_OP_TRACE_BACKWARD:  // + initial states of the pixels
            return fwd_ws_bytes(n) + align256(sizeof(double) * 8 * (size_t)n);
        case RT_OP_BIN:
            return bin_ws_bytes(n);
        case RT_OP_BACKWARD_POWER:  // block partials of the image sum
            return align256(sizeof(double) * 1024);
        case RT_OP_FLUX_GRAD:  // 64 observers, a checkpoint every 64 steps, a pool of 2 per ray
            return rt_flux_grad_workspace_size(n, 64, 64, (n > 0 && n < INT32_MAX / 2) ? 2 * n + 1 : INT32_MAX);
        default:
            return 0;
    }
}

extern "C" const char* rt_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// kernel timing: a pool of event pairs, one per timed launch, read after the fact.
// One record list for the process, guarded by a mutex: a launch takes its slot under
// the lock when its start event is recorded (the slot stays with the calling thread
// until its stop event is recorded), and rt_kernel_times reports completed slots only.
// ---------------------------------------------------------------------------
namespace {
constexpr int TIMING_SLOTS = 1024;
struct Timing {
    std::mutex mu;
    bool on = false;
    int used = 0;  // slots handed out since recording started
    int kinds[TIMING_SLOTS];
    bool done[TIMING_SLOTS];
    hipEvent_t ev[TIMING_SLOTS][2];
    bool created = false;
};
Timing g_timing;
thread_local int t_open = -1;  // this thread's slot whose stop event is pending
}  // namespace

void rtd::timing_begin(hipStream_t st, int kind) {
    Timing& T = g_timing;
    std::lock_guard<std::mutex> lock(T.mu);
    t_open = -1;
    if (!T.on || T.used >= TIMING_SLOTS) return;
    const int k = T.used;
    if (hipEventRecord(T.ev[k][0], st) != hipSuccess) return;
    T.kinds[k] = kind;
    T.done[k] = false;
    T.used = k + 1;
    t_open = k;
}

void rtd::timing_end(hipStream_t st) {
    Timing& T = g_timing;
    std::lock_guard<std::mutex> lock(T.mu);
    const int k = t_open;
    t_open = -1;
    if (!T.on || k < 0 || k >= T.used) return;
    if (hipEventRecord(T.ev[k][1], st) == hipSuccess) T.done[k] = true;
}

extern "C" int rt_timing(int32_t on) {
    clear_error();
    Timing& T = g_timing;
    std::lock_guard<std::mutex> lock(T.mu);
    if (on && !T.created) {
        for (int k = 0; k < TIMING_SLOTS; ++k)
            for (int e = 0; e < 2; ++e)
                if (hipEventCreate(&T.ev[k][e]) != hipSuccess) return fail(RT_EHIP, "rt_timing: hipEventCreate failed");
        T.created = true;
    }
    T.on = on != 0;
    if (T.on) T.used = 0;  // stopping keeps the records for rt_kernel_times
    return RT_OK;
}

extern "C" int32_t rt_kernel_times(double* ms, int32_t* kind, int32_t max) {
    Timing& T = g_timing;
    std::lock_guard<std::mutex> lock(T.mu);
    int m = 0;
    for (int k = 0; k < T.used && m < max; ++k) {
        if (!T.done[k]) continue;
        float t = -1.0f;
        if (hipEventSynchronize(T.ev[k][1]) != hipSuccess || hipEventElapsedTime(&t, T.ev[k][0], T.ev[k][1]) != hipSuccess)
            t = -1.0f;
        if (ms) ms[m] = (double)t;
        if (kind) kind[m] = T.kinds[k];
        ++m;
    }
    return m;
}

extern "C" const char* rt_version(void) {
    return "rt-gfx950 FP64 DOPRI5 ray tracer (hipcc " __VERSION__ ")";
}
