// Host-side helpers shared by the translation units of the HIP library:
// argument validation, error reporting, physical constants and the
// conversion of an rt_star into integrator units, workspace layout and
// launch geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/rt.h"
#include "rt_device.hpp"
#include "rt_integrator.hpp"
#include "rt_seed.hpp"

#define RT_NFIN_ 16
#define RT_NIFIN_ 3
#define RT_NEV_ 10

namespace rtd {

// ---------------------------------------------------------------------------
// error reporting (thread-local message)
// ---------------------------------------------------------------------------
void set_error(const char* msg);
void clear_error();
inline int fail(int code, const char* msg) {
    set_error(msg);
    return code;
}
int check_launch(const char* what);

bool validate_star(const rt_star* s);
bool validate_tol(const rt_tol* t);
InstT<double> make_inst(const rt_star& s);
SeedT<double> make_seed_consts(const rt_star& s);
StarFixed star_fixed(const rt_star& s);

// ---------------------------------------------------------------------------
// workspace of the persistent kernels
// ---------------------------------------------------------------------------
struct WorkCtr {
    unsigned long long head;   // next list entry to hand out
    unsigned long long len;    // list length
    unsigned long long iters;  // wave-iterations of the persistent loop (lane efficiency diagnostic)
    unsigned long long pad[29];  // pad[0]: the adjoint's seal; pad[1]: null-surface restarts of a forward launch
};

// Work-list ordering: rays are handed out in ascending order of a cost key (a
// bucket of log2(r/R) of the seed radius for forward rays: rays seeded deep in
// the magnetosphere take the most steps), so long rays start first and the
// persistent kernel's tail stays short.
constexpr int ORDER_BUCKETS = 4096;

// Partition (counting sort by bucket) of up to 2^31 - 1 indices into at most
// PART_BUCKETS buckets: one workgroup per chunk of at least PART_CHUNK_MIN keys, at most
// PART_MAX_BLOCKS of them, each with a row of PART_BUCKETS counters in the table.
constexpr int PART_BUCKETS = 4096;
constexpr int PART_MAX_BLOCKS = 256;
constexpr int64_t PART_CHUNK_MIN = 4096;

inline int partition_blocks(int64_t n) {
    int64_t g = (n + PART_CHUNK_MIN - 1) / PART_CHUNK_MIN;
    if (g > PART_MAX_BLOCKS) g = PART_MAX_BLOCKS;
    if (g < 1) g = 1;
    return (int)g;
}

// Per-lane slots of the forward tracing kernel for a lane whose step crossed the GJ null
// surface and waits for its restart: the step's start y (8), the coefficients a, b, c, d of
// its continuous extension (4 x 8), a spare field, phi(0), phi(1), the step's error and
// |x(1)|^2 (the step size stays in the lane's registers).
// Lane-major ([lane][STASH_STRIDE]): one base address and immediate field offsets.
constexpr int STASH_FIELDS = 45;
constexpr int STASH_STRIDE = 48;
constexpr int STASH_LANES_PER_CU = 512;  // the tracing kernels run at most 8 waves per CU

struct FwdWs {
    WorkCtr* ctr;
    double* stash;  // [stash_lanes][STASH_STRIDE]
    int64_t stash_lanes;
    int32_t* list;
    double* h0;  // forward tracing: in work-list order (entry q), like k1 and y0
    double* k1;
    double* y0;  // [8][n] seed states in work-list order
    int32_t* keys;     // [n] bucket of each ray (-1: not traced)
    int32_t* buckets;  // [ORDER_BUCKETS + 1] first list entry of each bucket, then the list length
    int32_t* tab;      // [partition_blocks(n) x ORDER_BUCKETS] per-workgroup bucket offsets
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline size_t part_tab_bytes(int64_t n) {
    return align256(sizeof(int32_t) * (size_t)partition_blocks(n) * PART_BUCKETS);
}
inline size_t part_start_bytes() { return align256(sizeof(int32_t) * (PART_BUCKETS + 1)); }

int device_cu_count();
inline int64_t stash_lanes() { return (int64_t)device_cu_count() * STASH_LANES_PER_CU; }
inline size_t stash_bytes() { return align256(sizeof(double) * STASH_STRIDE * (size_t)stash_lanes()); }

// Layout: first what outlives a trace (the work counter and the ordered work list with its sort
// keys, bucket starts and partition table, which the adjoint reuses for its reverse list),
// then what only the trace itself uses (the restart stash and the seeds in list order), from
// fwd_ws_transient_offset(n) to the end, which the adjoint's reverse phase overlays.
inline FwdWs carve_fwd_ws(void* ws, int64_t n) {
    char* p = (char*)ws;
    FwdWs W;
    W.ctr = (WorkCtr*)p;
    p += align256(sizeof(WorkCtr));
    W.list = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)n);
    W.keys = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)n);
    W.buckets = (int32_t*)p;
    p += part_start_bytes();
    W.tab = (int32_t*)p;
    p += part_tab_bytes(n);
    W.stash = (double*)p;
    W.stash_lanes = stash_lanes();
    p += stash_bytes();
    W.h0 = (double*)p;
    p += align256(sizeof(double) * (size_t)n);
    W.k1 = (double*)p;
    p += align256(sizeof(double) * 8 * (size_t)n);
    W.y0 = (double*)p;
    return W;
}

inline size_t fwd_ws_transient_offset(int64_t n) {
    return align256(sizeof(WorkCtr)) + 2 * align256(sizeof(int32_t) * (size_t)n) + part_start_bytes() +
           part_tab_bytes(n);
}

inline size_t fwd_ws_bytes(int64_t n) {
    return fwd_ws_transient_offset(n) + stash_bytes() + align256(sizeof(double) * (size_t)n) +
           2 * align256(sizeof(double) * 8 * (size_t)n);
}

// Groups the indices i < n with keys[i] >= 0 and keys[i] >> shift < nb (nb <= PART_BUCKETS)
// by bucket keys[i] >> shift into list (order inside a bucket is arbitrary); start[b] is
// the first list entry of bucket b and start[nb .. PART_BUCKETS] the list length.  tab
// holds part_tab_bytes(n).  With ctr, the list is armed for a persistent kernel.
int partition_keys(const int32_t* keys, int64_t n, int shift, int nb, int32_t* tab, int32_t* start,
                   int32_t* list, WorkCtr* ctr, hipStream_t st);

// workspace of rt_bin_flux: bin key and tile-ordered list of every ray, partition table
struct BinWs {
    int32_t* keys;
    int32_t* list;
    int32_t* start;
    int32_t* tab;
};
inline size_t bin_ws_bytes(int64_t n) {
    return 2 * align256(sizeof(int32_t) * (size_t)n) + part_start_bytes() + part_tab_bytes(n);
}
inline BinWs carve_bin_ws(void* ws, int64_t n) {
    char* p = (char*)ws;
    BinWs B;
    B.keys = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)n);
    B.list = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)n);
    B.start = (int32_t*)p;
    p += part_start_bytes();
    B.tab = (int32_t*)p;
    return B;
}

// builds W.list from W.keys (counting sort by bucket; order inside a bucket is arbitrary)
int order_work_list(const FwdWs& W, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
int device_cu_count();
inline int grid_for(int64_t n, int block, int per_thread) {
    int64_t g = (n + (int64_t)block * per_thread - 1) / ((int64_t)block * per_thread);
    int64_t cap = (int64_t)device_cu_count() * 16;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}
rt_schedule resolve_schedule(const rt_schedule* s);
// workgroups of a persistent launch: CUs x resident workgroups per CU
int persistent_grid(const rt_schedule& sc, const void* kernel, int block);

int launch_trace_fwd(const rt_schedule& sc, const InstT<double>& I, const TolC& T, const double* rays, int64_t n,
                     const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st);
int launch_trace_fwd_batched(const rt_schedule& sc, const InstT<double>& I0, const InstT<double>* itab,
                             const int32_t* inst_of, int any_oblique, const TolC& T, const double* rays, int64_t n,
                             const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st);
int launch_sample_batched(const InstT<double>* itab, const SeedT<double>* ctab, const int64_t* off, int32_t n_inst,
                          uint64_t seed, int64_t N, double* rays, int32_t* status, int32_t* inst_of, hipStream_t st);
// Set-up of a forward trace: the cost keys of the seeds (and the final records of seeds
// not traced), the work list ordered by them, then for every list entry q the seed state,
// its FSAL derivative (on the seed's smooth piece of the GJ density) and its starting step,
// written in list order so that the tracing kernels read them contiguously
int launch_trace_init(const InstT<double>& I0, const InstT<double>* itab, const int32_t* inst_of, const TolC& T,
                      const double* rays, const int32_t* status, int64_t n, const FwdWs& W, double* fin,
                      int32_t* ifin, hipStream_t st);
int launch_bin(const double* fin, const int32_t* ifin, const double* w, int64_t n, const rt_bins* bins,
               const int64_t* inst_offset, int32_t n_inst, double* hist, double* cnt, double* over, void* ws,
               hipStream_t st);

// optional HIP-event timing of the persistent kernels (rt_timing / rt_kernel_times):
// record a start/stop pair on the launch stream around one kernel launch
void timing_begin(hipStream_t st, int kind);
void timing_end(hipStream_t st);

// small utility kernels (defined per translation unit)
static __global__ void zero_ctr_kernel(WorkCtr* c) {
    if (threadIdx.x == 0) { c->head = 0ull; c->len = 0ull; c->iters = 0ull; }
}
static __global__ void fill_kernel(double* p, int64_t n, double v) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

}  // namespace rtd
