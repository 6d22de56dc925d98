// Batched persistent launch: many star instances (a parameter scan) traced by
// one persistent work-queue kernel, with seeding, ordering, finalisation and
// per-instance sky maps, as one fixed sequence of kernels (no host
// synchronisation), so the whole pipeline can be captured into a hipGraph.
//
// Workspace layout (after rt_batch_prepare):
//   [forward-tracer workspace for N rays]
//   inst_of[N] (int32)   bin keys[N] (int32)
//   itab[n_inst] (InstT)  ctab[n_inst] (SeedT)  offsets[n_inst + 1] (int64)
//   bin block table[n_blocks] (instance, first ray, end ray)
#include "rt_common.hpp"

namespace rtd {

constexpr int64_t BIN_CHUNK = 16384;  // rays per binning workgroup
constexpr int INST_TILE = 4096;       // bins per LDS tile (2 x 32 KiB of FP64)

struct BinBlock {
    int32_t inst;
    int32_t pad;
    int64_t r0, r1;
};

struct BatchWs {
    FwdWs fw;
    int32_t* inst_of;
    int32_t* keys;
    InstT<double>* itab;
    SeedT<double>* ctab;
    int64_t* off;
    BinBlock* blocks;
};

static int64_t bin_blocks_for(const int64_t* off, int32_t n_inst) {
    int64_t nb = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        int64_t nk = off[k + 1] - off[k];
        nb += (nk + BIN_CHUNK - 1) / BIN_CHUNK;
    }
    return nb;
}

static size_t batch_tail_bytes(int32_t n_inst, int64_t N, int64_t n_blocks) {
    return align256(sizeof(int32_t) * (size_t)N) * 2 + align256(sizeof(InstT<double>) * (size_t)n_inst) +
           align256(sizeof(SeedT<double>) * (size_t)n_inst) + align256(sizeof(int64_t) * (size_t)(n_inst + 1)) +
           align256(sizeof(BinBlock) * (size_t)(n_blocks > 0 ? n_blocks : 1));
}

static BatchWs carve_batch_ws(void* ws, int32_t n_inst, int64_t N) {
    BatchWs B;
    B.fw = carve_fwd_ws(ws, N);
    char* p = (char*)ws + fwd_ws_bytes(N);
    B.inst_of = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)N);
    B.keys = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)N);
    B.itab = (InstT<double>*)p;
    p += align256(sizeof(InstT<double>) * (size_t)n_inst);
    B.ctab = (SeedT<double>*)p;
    p += align256(sizeof(SeedT<double>) * (size_t)n_inst);
    B.off = (int64_t*)p;
    p += align256(sizeof(int64_t) * (size_t)(n_inst + 1));
    B.blocks = (BinBlock*)p;
    return B;
}

// Per-instance binning: workgroup b takes the rays [r0, r1) of one instance and
// accumulates them in LDS, one tile of that instance's map at a time, then merges
// the tile into the global map with FP64 atomics.
__global__ void __launch_bounds__(256) bin_inst_kernel(const int32_t* __restrict__ keys, const double* __restrict__ w,
                                                       const BinBlock* __restrict__ blocks, int64_t per,
                                                       double* __restrict__ hist, double* __restrict__ cnt) {
    __shared__ double sh_w[INST_TILE];
    __shared__ double sh_c[INST_TILE];
    const BinBlock b = blocks[blockIdx.x];
    const int64_t base = (int64_t)b.inst * per;
    for (int64_t t0 = 0; t0 < per; t0 += INST_TILE) {
        for (int q = threadIdx.x; q < INST_TILE; q += blockDim.x) { sh_w[q] = 0.0; sh_c[q] = 0.0; }
        __syncthreads();
        for (int64_t i = b.r0 + threadIdx.x; i < b.r1; i += blockDim.x) {
            int32_t k = keys[i];
            int64_t rel = (int64_t)k - base - t0;
            if (k >= 0 && rel >= 0 && rel < INST_TILE) {
                atomicAdd(&sh_w[rel], w[i]);
                atomicAdd(&sh_c[rel], 1.0);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < INST_TILE; q += blockDim.x) {
            int64_t gb = t0 + q;
            if (gb < per && sh_c[q] != 0.0) {
                atomicAdd(&hist[base + gb], sh_w[q]);
                atomicAdd(&cnt[base + gb], sh_c[q]);
            }
        }
        __syncthreads();
    }
}

// sky keys of escaped rays using the per-ray instance (no search)
__global__ void __launch_bounds__(256) bin_keys_inst_kernel(const double* __restrict__ fin,
                                                            const int32_t* __restrict__ ifin, int64_t n, int32_t nt,
                                                            int32_t np, int32_t nw, double dw,
                                                            const int32_t* __restrict__ inst_of,
                                                            int32_t* __restrict__ keys) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const double dth = M_PI / nt, dps = 2.0 * M_PI / np;
    const int64_t per = (int64_t)nt * np * nw;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t key = -1;
        if (ifin[2 * n + i] == ST_ESCAPED) {
            double th = fin[8 * n + i], ps = fin[10 * n + i], om = fin[11 * n + i];
            int it = (int)floor(th / dth);
            it = it < 0 ? 0 : (it > nt - 1 ? nt - 1 : it);
            int ip = (int)floor(ps / dps);
            ip = ip < 0 ? 0 : (ip > np - 1 ? np - 1 : ip);
            double iwf = floor((om - 1.0) / dw + 0.5) + (double)(nw / 2);
            if (iwf >= 0.0 && iwf < (double)nw)
                key = (int32_t)((int64_t)inst_of[i] * per + ((int64_t)it * np + ip) * nw + (int64_t)iwf);
        }
        keys[i] = key;
    }
}

}  // namespace rtd

using namespace rtd;

extern "C" size_t rt_batch_workspace_size(int32_t n_inst, const int64_t* ray_offset) {
    if (n_inst <= 0 || !ray_offset) return 0;
    int64_t N = ray_offset[n_inst];
    if (N < 0) return 0;
    return fwd_ws_bytes(N) + batch_tail_bytes(n_inst, N, bin_blocks_for(ray_offset, n_inst));
}

extern "C" int rt_batch_prepare(const rt_star* stars, int32_t n_inst, const int64_t* ray_offset, rt_batch* out,
                                void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!stars || n_inst <= 0 || !ray_offset || !out) return fail(RT_EINVAL, "rt_batch_prepare: null or empty");
    if (ray_offset[0] != 0) return fail(RT_EINVAL, "rt_batch_prepare: ray_offset[0] must be 0");
    for (int32_t k = 0; k < n_inst; ++k) {
        if (ray_offset[k + 1] < ray_offset[k]) return fail(RT_EINVAL, "rt_batch_prepare: offsets must not decrease");
        if (!validate_star(&stars[k])) return RT_EINVAL;
        if (stars[k].plasma != stars[0].plasma || stars[k].density != stars[0].density ||
            stars[k].weights != stars[0].weights || stars[k].kdir != stars[0].kdir)
            return fail(RT_EINVAL, "rt_batch_prepare: instances must share plasma, density, weights and kdir");
        if (stars[k].flags & RT_FLAG_FLAT_PROPAGATION)
            return fail(RT_EUNSUPPORTED, "rt_batch_prepare: flat-propagation variant");
        if (stars[k].flags & RT_FLAG_FINITE_LARMOR)
            return fail(RT_EUNSUPPORTED, "rt_batch_prepare: finite-magnetisation variant");
    }
    int64_t N = ray_offset[n_inst];
    if (N > INT32_MAX) return fail(RT_EINVAL, "rt_batch_prepare: more than 2^31 - 1 rays");
    size_t need = rt_batch_workspace_size(n_inst, ray_offset);
    if (!ws || ws_bytes < need) return fail(RT_ENOWS, "rt_batch_prepare: workspace too small");
    BatchWs B = carve_batch_ws(ws, n_inst, N);
    int64_t nb = bin_blocks_for(ray_offset, n_inst);
    InstT<double>* it = new InstT<double>[n_inst];
    SeedT<double>* ct = new SeedT<double>[n_inst];
    BinBlock* bb = new BinBlock[nb > 0 ? nb : 1];
    int any_oblique = 0;
    int64_t q = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        it[k] = make_inst(stars[k]);
        ct[k] = make_seed_consts(stars[k]);
        any_oblique |= it[k].oblique;
        for (int64_t r = ray_offset[k]; r < ray_offset[k + 1]; r += BIN_CHUNK) {
            bb[q].inst = k;
            bb[q].pad = 0;
            bb[q].r0 = r;
            bb[q].r1 = (r + BIN_CHUNK < ray_offset[k + 1]) ? r + BIN_CHUNK : ray_offset[k + 1];
            ++q;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(B.itab, it, sizeof(InstT<double>) * n_inst, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(B.ctab, ct, sizeof(SeedT<double>) * n_inst, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.off, ray_offset, sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nb > 0) e = hipMemcpyAsync(B.blocks, bb, sizeof(BinBlock) * nb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    delete[] it;
    delete[] ct;
    delete[] bb;
    if (e != hipSuccess) return fail(RT_EHIP, "rt_batch_prepare: upload of the instance tables failed");
    out->n_inst = n_inst;
    out->any_oblique = any_oblique;
    out->n_rays = N;
    out->n_bin_blocks = nb;
    out->plasma = stars[0].plasma;
    out->density = stars[0].density;
    out->ws_bytes = need;
    return RT_OK;
}

extern "C" int rt_trace_batched(const rt_batch* batch, uint64_t seed, const rt_tol* tol, const rt_bins* bins,
                                double* rays, int32_t* status, double* fin, int32_t* ifin, double* maps, double* cnt,
                                void* ws, size_t ws_bytes, const rt_schedule* sched, void* stream) {
    clear_error();
    if (!batch || batch->n_inst <= 0) return fail(RT_EINVAL, "rt_trace_batched: batch not prepared");
    if (!validate_tol(tol)) return RT_EINVAL;
    if (!bins || bins->n_theta <= 0 || bins->n_psi <= 0 || bins->n_omega <= 0 || !(bins->d_omega > 0.0))
        return fail(RT_EINVAL, "rt_trace_batched: invalid bins");
    const int64_t N = batch->n_rays;
    const int32_t n_inst = batch->n_inst;
    int64_t per = (int64_t)bins->n_theta * bins->n_psi * bins->n_omega;
    if (per * n_inst > INT32_MAX) return fail(RT_EINVAL, "rt_trace_batched: too many bins");
    if (!ws || ws_bytes < batch->ws_bytes) return fail(RT_ENOWS, "rt_trace_batched: workspace too small");
    if (!maps || !cnt || (N > 0 && (!rays || !status || !fin || !ifin)))
        return fail(RT_EINVAL, "rt_trace_batched: null array");
    rt_schedule sc = resolve_schedule(sched);
    TolC T{tol->rtol, tol->atol, tol->r_max_km, (long long)tol->max_steps};
    BatchWs B = carve_batch_ws(ws, n_inst, N);
    hipStream_t st = (hipStream_t)stream;
    int zg = grid_for(per * n_inst, 256, 4);
    hipLaunchKernelGGL(fill_kernel, dim3(zg), dim3(256), 0, st, maps, per * n_inst, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3(zg), dim3(256), 0, st, cnt, per * n_inst, 0.0);
    if (N == 0) return check_launch("fill_kernel");
    // a representative instance carries the uniform plasma / density types
    InstT<double> I0;
    memset(&I0, 0, sizeof(I0));
    I0.plasma = batch->plasma;
    I0.density = batch->density;
    I0.oblique = batch->any_oblique;
    int rc = launch_sample_batched(B.itab, B.ctab, B.off, n_inst, seed, N, rays, status, B.inst_of, st);
    if (rc) return rc;
    rc = launch_trace_init(I0, B.itab, B.inst_of, T, rays, status, N, B.fw, fin, ifin, st);
    if (rc) return rc;
    rc = launch_trace_fwd_batched(sc, I0, B.itab, B.inst_of, batch->any_oblique, T, rays, N, B.fw, fin, ifin, st);
    if (rc) return rc;
    hipLaunchKernelGGL(bin_keys_inst_kernel, dim3(grid_for(N, 256, 8)), dim3(256), 0, st, fin, ifin, N,
                       bins->n_theta, bins->n_psi, bins->n_omega, bins->d_omega, B.inst_of, B.keys);
    rc = check_launch("bin_keys_inst_kernel");
    if (rc) return rc;
    if (batch->n_bin_blocks > 0) {
        if (batch->n_bin_blocks > INT32_MAX) return fail(RT_EINVAL, "rt_trace_batched: too many bin blocks");
        hipLaunchKernelGGL(bin_inst_kernel, dim3((unsigned)batch->n_bin_blocks), dim3(256), 0, st, B.keys, rays + 8 * N,
                           B.blocks, per, maps, cnt);
    }
    return check_launch("bin_inst_kernel");
}
