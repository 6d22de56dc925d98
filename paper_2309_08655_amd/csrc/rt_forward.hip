// Forward path of the ray tracer on gfx950: resonance seeding, the persistent
// DOPRI5 tracing kernel and sky binning.  One ray per lane, FP64 throughout.
//
// McDonald & Witte, arXiv:2309.08655: Sec. 2.2 (forward Monte Carlo power,
// eq. (Power), top-hat binning), Sec. 3 (foliation, eq. (Hypersurfaces);
// forward-tracing equation (ForwardTracingEquation1)), Sec. 4.1-4.4
// (Hamiltonian, surface measure, focusing, conversion probability).
#include "rt_common.hpp"

#include <mutex>

namespace rtd {

// ----------------------------------------------------------------------------
// seeding
// ----------------------------------------------------------------------------

// Not inlined: the single-instance and the batched sampling kernels run this one copy of
// the code, so a ray's seed is the same bits whichever kernel produced it.
__device__ static __noinline__ void seed_one(const InstT<double>& I, const SeedT<double>& C, uint64_t seed,
                                             int32_t instance, int64_t gi, double out[10], int32_t* status) {
    *status = seed_ray<double>(I, C, seed, instance, gi, out);
}

// instance owning global ray i: largest k with off[k] <= i
__device__ __forceinline__ int32_t find_instance(const int64_t* __restrict__ off, int32_t n_inst, int64_t i) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) sample_batched_kernel(const InstT<double>* __restrict__ itab,
                                                             const SeedT<double>* __restrict__ ctab,
                                                             const int64_t* __restrict__ off, int32_t n_inst,
                                                             uint64_t seed, int64_t N, double* __restrict__ rays,
                                                             int32_t* __restrict__ status,
                                                             int32_t* __restrict__ inst_of) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < N; gi += stride) {
        int32_t k = find_instance(off, n_inst, gi);
        double o[10];
        int32_t st;
        seed_one(itab[k], ctab[k], seed, k, gi - off[k], o, &st);
        for (int d = 0; d < 10; ++d) rays[d * N + gi] = o[d];
        status[gi] = st;
        inst_of[gi] = k;
    }
}

__global__ void __launch_bounds__(256) sample_kernel(InstT<double> I, SeedT<double> C, uint64_t seed, int32_t instance,
                                                     int64_t first, int64_t n, double* __restrict__ rays,
                                                     int32_t* __restrict__ status) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        double o[10];
        int32_t st;
        seed_one(I, C, seed, instance, first + j, o, &st);
        for (int d = 0; d < 10; ++d) rays[d * n + j] = o[d];
        status[j] = st;
    }
}

// ----------------------------------------------------------------------------
// tracing set-up: cost keys, then (after the work list is ordered) the starting state,
// FSAL derivative and starting step of every list entry, in list order
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) trace_keys_kernel(InstT<double> I0, const InstT<double>* __restrict__ itab,
                                                         const int32_t* __restrict__ inst_of,
                                                         const double* __restrict__ rays,
                                                         const int32_t* __restrict__ status, int64_t n,
                                                         int32_t* __restrict__ keys, double* __restrict__ fin,
                                                         int32_t* __restrict__ ifin) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        int32_t key = -1;
        if (status != nullptr && status[j] != ST_OK) {
            for (int d = 0; d < RT_NFIN_; ++d) fin[d * n + j] = 0.0;
            ifin[j] = 0;
            ifin[n + j] = 0;
            ifin[2 * n + j] = status[j];
        } else {
            const double R = (itab != nullptr) ? itab[inst_of[j]].R : I0.R;
            const double x = rays[j], y = rays[n + j], z = rays[2 * n + j];
            // cost key: rays seeded close to the star take the most steps
            const double r = sqrt(x * x + y * y + z * z);
            const double u = log2(fmax(r / R, 1.0)) * (ORDER_BUCKETS / 8.0);
            key = (u >= 0.0 && u < (double)(ORDER_BUCKETS - 1)) ? (int32_t)u : ORDER_BUCKETS - 1;
        }
        keys[j] = key;
    }
}

__global__ void __launch_bounds__(256) trace_init_kernel(InstT<double> I0, const InstT<double>* __restrict__ itab,
                                                         const int32_t* __restrict__ inst_of, TolC tol,
                                                         const double* __restrict__ rays, int64_t n,
                                                         const WorkCtr* __restrict__ ctr,
                                                         const int32_t* __restrict__ list, double* __restrict__ y0q,
                                                         double* __restrict__ h0q, double* __restrict__ k1q) {
    const int64_t nlist = (int64_t)ctr->len;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nlist; q += stride) {
        const int64_t j = list[q];
        const InstT<double> I = (itab != nullptr) ? itab[inst_of[j]] : I0;
        double y[8], f0[8];
        for (int d = 0; d < 8; ++d) y[d] = rays[d * n + j];
        // GJ density, cut at the null surface: the smooth piece of |g| the seed lies on,
        // which the tracing kernels (forward, batched and the adjoint's) integrate from
        // here, also for the starting step's probe
        const double gjs = (I.density == DEN_GJ) ? ((gj_factor(I, y) < 0.0) ? -1.0 : 1.0) : 0.0;
        auto f = [&](const double* yy, double* ff) { rhs(I, yy, ff, 1.0, nullptr, gjs); };
        f(y, f0);
        const double h = initial_step(f, y, f0, tol.rtol, tol.atol);
        h0q[q] = h;
        for (int d = 0; d < 8; ++d) {
            y0q[d * n + q] = y[d];
            k1q[d * n + q] = f0[d];
        }
    }
}

// ----------------------------------------------------------------------------
// persistent tracing kernel: each lane integrates rays taken from the work list
// until the list is exhausted; a wave refills its idle lanes with one atomic
// ----------------------------------------------------------------------------
// BATCHED: rays of many star instances share the queue; a lane loads its ray's
// instance constants on refill (plasma and density types are common to all
// instances; the rotating-axis formula is used for every lane when any instance
// is oblique, exact for the aligned ones).
template <int BLOCK, int MINW, bool BATCHED, int SPEC = 0>
__global__ void __launch_bounds__(BLOCK, MINW) trace_fwd_kernel(InstT<double> I0, const InstT<double>* __restrict__ itab,
                                                          const int32_t* __restrict__ inst_of, int any_oblique,
                                                          TolC tol, const double* __restrict__ rays,
                                                          int64_t n, WorkCtr* ctr, const int32_t* __restrict__ list,
                                                          const double* __restrict__ y0q, const double* __restrict__ h0s,
                                                          const double* __restrict__ k1s, double* __restrict__ fin,
                                                          int32_t* __restrict__ ifin, int refill_min,
                                                          int cross_batch, double* __restrict__ stash, int chunk) {
    // a specialised instantiation (SPEC = 1 + plasma + 2 density + 8 oblique) fixes these
    // switches at compile time: the Hamiltonian and its gradient become branch-free code with
    // the same arithmetic (the file is built with -ffp-contract=on, so the generic and the
    // specialised kernels round identically).  Batched instances share plasma and density,
    // and all take the batch's rotation switch.
    auto fix = [&](InstT<double>& J) {
        if (BATCHED) J.oblique = any_oblique;
        if constexpr (SPEC > 0) {  // the flat dipole, strong field (other stars take the generic kernel)
            J.plasma = (SPEC - 1) & 1;
            J.density = ((SPEC - 1) >> 1) & 3;
            J.oblique = ((SPEC - 1) >> 3) & 1;
            J.gr_dipole = 0;
            J.larmor = 0;
        }
    };
    InstT<double> I = I0;
    fix(I);
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long nlist = ctr->len;
    unsigned long long iters = 0;
    bool active = false;
    bool exhausted = false;
    int64_t j = 0;
    double y[8], ynew[8];
    Stages S;
    double h = 0.0, lam = 0.0, facmax = 10.0;
    int nacc = 0, nrej = 0;
    for (int d = 0; d < 8; ++d) { y[d] = 0.0; S.K[0][d] = 0.0; }
    y[0] = 1e4;  // harmless dummy state for idle lanes
    y[7] = -1.0;
    AxisRef ref = axis_ref_at(I, 0.0);
    // GJ density: the lane integrates the smooth piece gjs g of |g| (gjs = +1 or -1) and
    // restarts on the other piece where a step crosses the null surface g = 0; phi = gjs g
    // at y.  Other densities: gjs = 0.
    double gjs = 0.0, phi = 0.0;
    bool pending = false;  // a crossing waits for its restart, its step in the lane's stash slot
    unsigned int ncross = 0;  // restarts of this lane (diagnostic)
    double* slot = stash + ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * STASH_STRIDE;
    auto st_put = [&](int fld, double v) { slot[fld] = v; };
    auto st_get = [&](int fld) { return slot[fld]; };
    // gnew: the GJ factor at the last state f was evaluated at, which after an attempt is the
    // step's end (its last stage); the crossing test takes it from there
    double gnew = 0.0;
    auto f = [&](const double* yy, double* ff) { rhs(I, yy, ff, 1.0, &ref, gjs, &gnew); };
    const double rmax2 = tol.rmax * tol.rmax;
    double R2 = I.R * I.R;

    // list entry q: its ray j, whose seed state, FSAL derivative and starting step the set-up
    // wrote in list order (consecutive entries read consecutive addresses)
    auto start_ray = [&](unsigned long long q) {
        j = list[q];
        if (BATCHED) {
            I = itab[inst_of[j]];
            fix(I);
            R2 = I.R * I.R;
        }
        for (int d = 0; d < 8; ++d) { y[d] = y0q[d * n + q]; S.K[0][d] = k1s[d * n + q]; }
        h = h0s[q];
        lam = 0.0; facmax = 10.0; nacc = 0; nrej = 0;
        if (I.oblique) ref = axis_ref_at(I, y[3]);
        if (I.density == DEN_GJ) {
            const double g0 = gj_factor(I, y, &ref);
            gjs = (g0 < 0.0) ? -1.0 : 1.0;
            phi = gjs * g0;
        }
        pending = false;
        active = true;
    };
    // chunk > 0: the wave claims `chunk` list entries at a time and hands them to its idle
    // lanes over several refills (one atomic per chunk); 0: exactly the idle lanes' worth
    unsigned long long cpos = 0, cend = 0;

    while (true) {
        unsigned long long idle = __ballot(!active);
        if (idle && !exhausted) {
            int cnt = __popcll(idle);
            if (cnt >= refill_min || idle == __ballot(true)) {
                if (chunk <= 0) {
                    int leader = __ffsll((long long)idle) - 1;
                    unsigned long long base = 0;
                    if (lane == leader) base = atomicAdd(&ctr->head, (unsigned long long)cnt);
                    base = __shfl(base, leader);
                    if (!active) {
                        unsigned long long q = base + __popcll(idle & below);
                        if (q < nlist) start_ray(q);
                    }
                    if (base + (unsigned long long)cnt >= nlist) exhausted = true;
                } else {
                    unsigned long long want = idle;
                    while (want) {
                        if (cpos >= cend) {
                            unsigned long long b = 0;
                            if (lane == 0) b = atomicAdd(&ctr->head, (unsigned long long)chunk);
                            b = __shfl(b, 0);
                            if (b >= nlist) {
                                exhausted = true;
                                break;
                            }
                            cpos = b;
                            cend = (b + (unsigned long long)chunk < nlist) ? b + (unsigned long long)chunk : nlist;
                        }
                        const unsigned long long avail = cend - cpos;
                        const unsigned long long rank = (unsigned long long)__popcll(want & below);
                        if (((want >> lane) & 1ull) && rank < avail) start_ray(cpos + rank);
                        const unsigned long long nw = (unsigned long long)__popcll(want);
                        cpos += (avail < nw) ? avail : nw;
                        want = __ballot(!active);
                    }
                }
            }
        }
        if (__ballot(active) == 0ull) {
            if (exhausted) break;
            continue;
        }
        ++iters;

        // on termination y holds the final state (the raw record is completed by
        // finalize_kernel, which keeps the observables out of this loop)
        int status = ST_OK;
        double lam_out = lam;
        // Lanes whose last accepted step crossed the GJ null surface wait (their step,
        // stages and error kept) and are restarted together once cross_batch of them, or
        // half of the wave's active lanes, wait: the restart (locating the crossing and a
        // fresh derivative) then costs the wave one pass for many lanes.
        const unsigned long long waiting = __ballot(pending);
        const int nwait = __popcll(waiting);
        if (nwait > 0 && (nwait >= cross_batch || 2 * nwait >= __popcll(__ballot(active)))) {
            if (pending) {
                // components 0..3 (position and time) locate the crossings
                double y0[4], ca[4], cb[4], cc[4], cd[4];
                for (int d = 0; d < 4; ++d) {
                    y0[d] = st_get(d);
                    ca[d] = st_get(8 + d);
                    cb[d] = st_get(16 + d);
                    cc[d] = st_get(24 + d);
                    cd[d] = st_get(32 + d);
                }
                const double phi0 = st_get(41), phi1 = st_get(42), errp = st_get(43), r2new = st_get(44);
                double phik;
                const double thk = locate_null_crossing_c(I, y0, ca, cb, cc, cd, gjs, phi0, phi1, &ref, &phik);
                // the step may also have reached r_max: whichever comes first
                const double th = (r2new >= rmax2) ? locate_crossing_c(y0, ca, cb, cc, cd, sqrt(r2new), tol.rmax)
                                                   : 2.0;
                const double tc = (th <= thk) ? th : thk;
                for (int d = 0; d < 8; ++d)
                    y[d] = dense_value(st_get(d), st_get(8 + d), st_get(16 + d), st_get(24 + d), st_get(32 + d), tc);
                if (th <= thk) {
                    status = ST_ESCAPED;
                    lam_out = lam + th * h;
                } else {
                    lam += thk * h;
                    lam_out = lam;
                    gjs = -gjs;
                    phi = -phik;  // the new piece's value there, >= 0
                    if (I.oblique) axis_ref_advance(I, ref, y[3]);
                    f(y, S.K[0]);
                    ++ncross;
                    h *= step_factor(errp, facmax, true);
                    facmax = 10.0;
                    if (nacc >= tol.max_steps) status = ST_MAX_STEPS;
                    else if (!(fabs(h) >= 1e-14 * (1.0 + fabs(lam)))) status = ST_STEP_UNDERFLOW;
                }
                pending = false;
            }
        }
        if (active && !pending && status == ST_OK) {
            const double err2 = dopri_attempt(f, y, S, h, ynew, tol.rtol, tol.atol);
            if (!(err2 <= 1.0)) {
                ++nrej;
                h *= step_factor(err2, facmax, false);
                facmax = 1.0;
                if (!(fabs(h) >= 1e-14 * (1.0 + fabs(lam)))) status = ST_STEP_UNDERFLOW;
            } else {
                ++nacc;
                // radii compared squared (r >= r_max <=> r^2 >= r_max^2)
                double r2new = ynew[0] * ynew[0] + ynew[1] * ynew[1] + ynew[2] * ynew[2];
                bool finite_ok = true;
                for (int d = 0; d < 8; ++d) finite_ok = finite_ok && isfinite(ynew[d]);
                // crossing of the GJ null surface inside the step
                double g1 = 0.0;
                bool cross = false;
                if (I.density == DEN_GJ && finite_ok && r2new > R2) {
                    g1 = gnew;  // = gj_factor(I, ynew, &ref), from the last stage
                    cross = (gjs * g1 < 0.0);
                }
                if (cross) {
                    // restarted (or ended at r_max) with the next batch: the step goes to the
                    // stash, so that no register stays held while the lane waits
                    pending = true;
                    for (int d = 0; d < 8; ++d) {
                        double ca, cb, cc, cd;
                        dense_coeffs(y, ynew, S, h, d, d + 1, &ca, &cb, &cc, &cd);
                        st_put(d, y[d]);
                        st_put(8 + d, ca);
                        st_put(16 + d, cb);
                        st_put(24 + d, cc);
                        st_put(32 + d, cd);
                    }
                    st_put(41, phi);
                    st_put(42, gjs * g1);
                    st_put(43, err2);
                    st_put(44, r2new);
                } else if (finite_ok && r2new >= rmax2) {
                    // locate r(theta) = r_max on the continuous extension
                    const double th = locate_crossing(y, ynew, S, h, tol.rmax);
                    double yt[8];
                    dense_at(y, ynew, S, h, th, yt, 0, 8);
                    for (int d = 0; d < 8; ++d) y[d] = yt[d];
                    status = ST_ESCAPED;
                    lam_out = lam + th * h;
                } else {
                    if (I.oblique && finite_ok && r2new > R2) axis_ref_advance(I, ref, ynew[3]);
                    for (int d = 0; d < 8; ++d) { y[d] = ynew[d]; S.K[0][d] = S.K[6][d]; }
                    lam += h;
                    lam_out = lam;
                    phi = gjs * g1;
                    if (!finite_ok) {
                        status = ST_NONFINITE;
                    } else if (r2new <= R2) {
                        status = ST_HIT_STAR;
                    } else {
                        h *= step_factor(err2, facmax, true);
                        facmax = 10.0;
                        if (nacc >= tol.max_steps) status = ST_MAX_STEPS;
                        else if (!(fabs(h) >= 1e-14 * (1.0 + fabs(lam)))) status = ST_STEP_UNDERFLOW;
                    }
                }
            }
        }
        if (!active) continue;
        if (status != ST_OK) {
            for (int d = 0; d < 8; ++d) fin[d * n + j] = y[d];
            fin[13 * n + j] = lam_out;
            fin[15 * n + j] = h;
            ifin[j] = nacc;
            ifin[n + j] = nrej;
            ifin[2 * n + j] = status;
            active = false;
        }
    }
    if (lane == 0) atomicAdd(&ctr->iters, iters);
    if (ncross) atomicAdd(&ctr->pad[1], (unsigned long long)ncross);
}

// Observables of every traced ray from its final state (Sec. 2.2: the asymptotic
// direction is binned on the sky): static-frame direction (theta, phi), the
// azimuth psi in the frame co-rotating with the star at the arrival time t - r,
// the energy at infinity -k_t, H and r.
__global__ void __launch_bounds__(256) finalize_kernel(InstT<double> I0, const InstT<double>* __restrict__ itab,
                                                       const int32_t* __restrict__ inst_of,
                                                       const int32_t* __restrict__ keys, int64_t n,
                                                       double* __restrict__ fin) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        if (keys[j] < 0) continue;  // not traced: the init pass wrote its final record
        const InstT<double> I = (itab != nullptr) ? itab[inst_of[j]] : I0;
        double yf[8];
        for (int d = 0; d < 8; ++d) yf[d] = fin[d * n + j];
        double r = sqrt(yf[0] * yf[0] + yf[1] * yf[1] + yf[2] * yf[2]);
        double ir = 1.0 / r;
        double nn[3] = {yf[0] * ir, yf[1] * ir, yf[2] * ir};
        double A = 1.0 - I.rs * ir;
        double qn = nn[0] * yf[4] + nn[1] * yf[5] + nn[2] * yf[6];
        double c = (sqrt(A) - 1.0) * qn;
        double v[3] = {yf[4] + c * nn[0], yf[5] + c * nn[1], yf[6] + c * nn[2]};
        double vn = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        v[0] *= vn; v[1] *= vn; v[2] *= vn;
        double theta = atan2(sqrt(v[0] * v[0] + v[1] * v[1]), v[2]);
        double phi = atan2(v[1], v[0]);
        double psi = fmod(phi - I.Om * (yf[3] - r), 2.0 * M_PI);
        if (psi < 0.0) psi += 2.0 * M_PI;
        if (psi >= 2.0 * M_PI) psi -= 2.0 * M_PI;
        fin[8 * n + j] = theta;
        fin[9 * n + j] = phi;
        fin[10 * n + j] = psi;
        fin[11 * n + j] = -yf[7];
        fin[12 * n + j] = hamiltonian(I, yf);
        fin[14 * n + j] = r;
    }
}

// ----------------------------------------------------------------------------
// binning: per-ray keys, then LDS-privatised tiles merged with FP64 atomics
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) bin_keys_kernel(const double* __restrict__ fin, const int32_t* __restrict__ ifin,
                                                       int64_t n, int32_t nt, int32_t np, int32_t nw, double dw,
                                                       const int64_t* __restrict__ inst_offset, int32_t n_inst,
                                                       int32_t* __restrict__ keys, const double* __restrict__ w,
                                                       double* __restrict__ over) {
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
            if (iwf >= 0.0 && iwf < (double)nw) {
                int64_t inst = 0;
                if (inst_offset != nullptr) {
                    // instance owning ray i: largest k with inst_offset[k] <= i
                    int lo = 0, hi = n_inst - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (inst_offset[mid] <= i) lo = mid; else hi = mid - 1;
                    }
                    inst = lo;
                }
                key = (int32_t)(inst * per + ((int64_t)it * np + ip) * nw + (int64_t)iwf);
            } else {
                atomicAdd(&over[0], w[i]);
                atomicAdd(&over[1], 1.0);
            }
        }
        keys[i] = key;
    }
}

constexpr int BIN_SHIFT = 12;
constexpr int BIN_TILE = 1 << BIN_SHIFT;  // bins per LDS tile: 2 x 32 KiB of FP64

// The rays are first partitioned by tile (key >> BIN_SHIFT); workgroup (t, s) then takes
// slice s of tile t's rays, accumulates them in LDS and merges the touched bins into the
// global map with FP64 atomics.  Every ray is read once.
__global__ void __launch_bounds__(256) bin_part_kernel(const int32_t* __restrict__ keys, const double* __restrict__ w,
                                                       const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ start, int64_t nbins,
                                                       int32_t slices, double* __restrict__ hist,
                                                       double* __restrict__ cnt) {
    __shared__ double sh_w[BIN_TILE];
    __shared__ double sh_c[BIN_TILE];
    const int64_t t = blockIdx.x;
    const int64_t lo = start[t], len = (int64_t)start[t + 1] - lo;
    const int64_t a = lo + (len * blockIdx.y) / slices;
    const int64_t e = lo + (len * (blockIdx.y + 1)) / slices;
    if (a == e) return;  // uniform over the workgroup
    const int64_t tile0 = t * BIN_TILE;
    for (int b = threadIdx.x; b < BIN_TILE; b += blockDim.x) { sh_w[b] = 0.0; sh_c[b] = 0.0; }
    __syncthreads();
    for (int64_t q = a + threadIdx.x; q < e; q += blockDim.x) {
        const int32_t i = list[q];
        const int rel = (int)((int64_t)keys[i] - tile0);
        atomicAdd(&sh_w[rel], w[i]);
        atomicAdd(&sh_c[rel], 1.0);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BIN_TILE; b += blockDim.x) {
        const int64_t gb = tile0 + b;
        if (gb < nbins && sh_c[b] != 0.0) {
            atomicAdd(&hist[gb], sh_w[b]);
            atomicAdd(&cnt[gb], sh_c[b]);
        }
    }
}

// maps of more than PART_BUCKETS tiles: one FP64 atomic pair per ray
__global__ void __launch_bounds__(256) bin_direct_kernel(const int32_t* __restrict__ keys, const double* __restrict__ w,
                                                         int64_t n, double* __restrict__ hist,
                                                         double* __restrict__ cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t k = keys[i];
        if (k >= 0) {
            atomicAdd(&hist[k], w[i]);
            atomicAdd(&cnt[k], 1.0);
        }
    }
}

// resonant cyclotron depth of each escaped ray and the attenuated weight w e^{-tau}
__global__ void __launch_bounds__(256) cyclotron_kernel(InstT<double> I, SeedT<double> C,
                                                        const double* __restrict__ rays,
                                                        const double* __restrict__ fin,
                                                        const int32_t* __restrict__ ifin, int64_t n,
                                                        double* __restrict__ tau, double* __restrict__ rcyc,
                                                        double* __restrict__ w_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        double t = 0.0, rr = -1.0;
        if (ifin[2 * n + j] == ST_ESCAPED)
            t = cyclotron_tau(I, C, fin[8 * n + j], fin[9 * n + j], fin[3 * n + j], fin[14 * n + j],
                              fin[11 * n + j], rays[9 * n + j], &rr);
        tau[j] = t;
        if (rcyc) rcyc[j] = rr;
        if (w_out) w_out[j] = rays[8 * n + j] * ::exp(-t);
    }
}

}  // namespace rtd

using namespace rtd;

extern "C" int rt_cyclotron_depth(const rt_star* star, const double* rays, const double* fin, const int32_t* ifin,
                                  int64_t n, double* tau, double* r_cyc, double* w_out, void* stream) {
    clear_error();
    if (!validate_star(star)) return RT_EINVAL;
    if (n < 0) return fail(RT_EINVAL, "rt_cyclotron_depth: negative n");
    if (n == 0) return RT_OK;
    if (!rays || !fin || !ifin || !tau) return fail(RT_EINVAL, "rt_cyclotron_depth: null array");
    InstT<double> I = make_inst(*star);
    SeedT<double> C = make_seed_consts(*star);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(cyclotron_kernel, dim3(grid_for(n, 256, 4)), dim3(256), 0, st, I, C, rays, fin, ifin, n, tau,
                       r_cyc, w_out);
    return check_launch("cyclotron_kernel");
}

extern "C" int rt_sample_resonance(const rt_star* star, uint64_t seed, int32_t instance, int64_t first, int64_t n,
                                   double* rays, int32_t* status, void* stream) {
    clear_error();
    if (!validate_star(star)) return RT_EINVAL;
    if (n < 0 || first < 0) return fail(RT_EINVAL, "rt_sample_resonance: negative n or first");
    if (n == 0) return RT_OK;
    if (!rays || !status) return fail(RT_EINVAL, "rt_sample_resonance: null output array");
    InstT<double> I = make_inst(*star);
    SeedT<double> C = make_seed_consts(*star);
    int grid = grid_for(n, 256, 8);
    hipLaunchKernelGGL(sample_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, I, C, seed, instance, first, n,
                       rays, status);
    return check_launch("sample_kernel");
}

extern "C" int rt_trace_forward(const rt_star* star, const rt_tol* tol, const double* rays, const int32_t* status,
                                int64_t n, double* fin, int32_t* ifin, void* ws, size_t ws_bytes,
                                const rt_schedule* sched, void* stream) {
    clear_error();
    if (!validate_star(star) || !validate_tol(tol)) return RT_EINVAL;
    if (n < 0) return fail(RT_EINVAL, "rt_trace_forward: negative n");
    if (n == 0) return RT_OK;
    if (n > INT32_MAX) return fail(RT_EINVAL, "rt_trace_forward: n exceeds 2^31 - 1");
    if (!rays || !fin || !ifin) return fail(RT_EINVAL, "rt_trace_forward: null array");
    size_t need = rt_workspace_size(RT_OP_TRACE_FORWARD, n);
    if (!ws || ws_bytes < need) return fail(RT_ENOWS, "rt_trace_forward: workspace too small");
    rt_schedule sc = resolve_schedule(sched);
    InstT<double> I = make_inst(*star);
    // flat-propagation variant: Hamilton's equations with M = 0 for curved initial conditions
    if (star->flags & RT_FLAG_FLAT_PROPAGATION) I.rs = 0.0;
    TolC T{tol->rtol, tol->atol, tol->r_max_km, (long long)tol->max_steps};
    FwdWs W = carve_fwd_ws(ws, n);
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_trace_init(I, nullptr, nullptr, T, rays, status, n, W, fin, ifin, st);
    if (rc) return rc;
    return launch_trace_fwd(sc, I, T, rays, n, W, fin, ifin, st);
}

namespace rtd {
template <int BLOCK, int MINW, bool BATCHED, int SPEC = 0>
static int launch_fwd_block(const rt_schedule& sc, const InstT<double>& I, const InstT<double>* itab,
                            const int32_t* inst_of, int any_oblique, const TolC& T, const double* rays, int64_t n,
                            const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    int grid = persistent_grid(sc, (const void*)trace_fwd_kernel<BLOCK, MINW, BATCHED, SPEC>, BLOCK);
    if ((int64_t)grid * BLOCK > W.stash_lanes) return fail(RT_EINVAL, "trace_fwd_kernel: more lanes than stash slots");
    timing_begin(st, BATCHED ? RT_KERNEL_TRACE_BATCHED : RT_KERNEL_TRACE_FORWARD);
    hipLaunchKernelGGL((trace_fwd_kernel<BLOCK, MINW, BATCHED, SPEC>), dim3(grid), dim3(BLOCK), 0, st, I, itab,
                       inst_of, any_oblique, T, rays, n, W.ctr, W.list, W.y0, W.h0, W.k1, fin, ifin, sc.refill_min,
                       sc.cross_batch, W.stash, sc.chunk);
    timing_end(st);
    int rc = check_launch("trace_fwd_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(finalize_kernel, dim3(grid_for(n, 256, 4)), dim3(256), 0, st, I, itab, inst_of, W.keys, n,
                       fin);
    return check_launch("finalize_kernel");
}

// the default schedule (256 threads, occupancy 2) of a single star: one instantiation per
// (plasma, density, rotation)
template <int S>
static int launch_spec(const rt_schedule& sc, const InstT<double>& I, const TolC& T, const double* rays, int64_t n,
                       const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    return launch_fwd_block<256, 2, false, S>(sc, I, nullptr, nullptr, 0, T, rays, n, W, fin, ifin, st);
}

static int launch_specialised(const rt_schedule& sc, const InstT<double>& I, const TolC& T, const double* rays,
                              int64_t n, const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    const int spec = 1 + (I.plasma & 1) + 2 * (I.density & 3) + 8 * (I.oblique ? 1 : 0);
    switch (spec) {
        case 1: return launch_spec<1>(sc, I, T, rays, n, W, fin, ifin, st);
        case 2: return launch_spec<2>(sc, I, T, rays, n, W, fin, ifin, st);
        case 3: return launch_spec<3>(sc, I, T, rays, n, W, fin, ifin, st);
        case 4: return launch_spec<4>(sc, I, T, rays, n, W, fin, ifin, st);
        case 5: return launch_spec<5>(sc, I, T, rays, n, W, fin, ifin, st);
        case 6: return launch_spec<6>(sc, I, T, rays, n, W, fin, ifin, st);
        case 7: return launch_spec<7>(sc, I, T, rays, n, W, fin, ifin, st);
        case 8: return launch_spec<8>(sc, I, T, rays, n, W, fin, ifin, st);
        case 9: return launch_spec<9>(sc, I, T, rays, n, W, fin, ifin, st);
        case 10: return launch_spec<10>(sc, I, T, rays, n, W, fin, ifin, st);
        case 11: return launch_spec<11>(sc, I, T, rays, n, W, fin, ifin, st);
        case 12: return launch_spec<12>(sc, I, T, rays, n, W, fin, ifin, st);
        case 13: return launch_spec<13>(sc, I, T, rays, n, W, fin, ifin, st);
        case 14: return launch_spec<14>(sc, I, T, rays, n, W, fin, ifin, st);
        case 15: return launch_spec<15>(sc, I, T, rays, n, W, fin, ifin, st);
        default: return launch_spec<16>(sc, I, T, rays, n, W, fin, ifin, st);
    }
}

// batched launches at 256 threads: one instantiation per (plasma, density, rotation) and occupancy
template <int MINW, int S>
static int launch_bspec(const rt_schedule& sc, const InstT<double>& I, const InstT<double>* itab,
                        const int32_t* inst_of, int any_oblique, const TolC& T, const double* rays, int64_t n,
                        const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    return launch_fwd_block<256, MINW, true, S>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
}

template <int MINW>
static int launch_batched_specialised(const rt_schedule& sc, const InstT<double>& I, const InstT<double>* itab,
                                      const int32_t* inst_of, int any_oblique, const TolC& T, const double* rays,
                                      int64_t n, const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    const int spec = 1 + (I.plasma & 1) + 2 * (I.density & 3) + 8 * (any_oblique ? 1 : 0);
#define RT_BSPEC(S) \
    case S: return launch_bspec<MINW, S>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
    switch (spec) {
        RT_BSPEC(1) RT_BSPEC(2) RT_BSPEC(3) RT_BSPEC(4) RT_BSPEC(5) RT_BSPEC(6) RT_BSPEC(7) RT_BSPEC(8)
        RT_BSPEC(9) RT_BSPEC(10) RT_BSPEC(11) RT_BSPEC(12) RT_BSPEC(13) RT_BSPEC(14) RT_BSPEC(15)
        default: return launch_bspec<MINW, 16>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
    }
#undef RT_BSPEC
}

template <bool BATCHED>
static int launch_trace_variant(const rt_schedule& sc, const InstT<double>& I, const InstT<double>* itab,
                                const int32_t* inst_of, int any_oblique, const TolC& T, const double* rays, int64_t n,
                                const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    if constexpr (!BATCHED) {
        if (sc.occupancy == 2 && sc.block != 64 && sc.block != 128 && !I.gr_dipole && !I.larmor)
            return launch_specialised(sc, I, T, rays, n, W, fin, ifin, st);
    } else {
        if (sc.block != 64 && sc.block != 128 && !I.gr_dipole && !I.larmor) {
            if (sc.occupancy == 2)
                return launch_batched_specialised<2>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
            return launch_batched_specialised<1>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
        }
    }
    if (sc.occupancy == 2) {
        switch (sc.block) {
            case 64: return launch_fwd_block<64, 2, BATCHED>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
            case 128: return launch_fwd_block<128, 2, BATCHED>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
            default: return launch_fwd_block<256, 2, BATCHED>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
        }
    }
    switch (sc.block) {
        case 64: return launch_fwd_block<64, 1, BATCHED>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
        case 128: return launch_fwd_block<128, 1, BATCHED>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
        default: return launch_fwd_block<256, 1, BATCHED>(sc, I, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
    }
}

int launch_trace_fwd(const rt_schedule& sc, const InstT<double>& I, const TolC& T, const double* rays, int64_t n,
                     const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    return launch_trace_variant<false>(sc, I, nullptr, nullptr, 0, T, rays, n, W, fin, ifin, st);
}

int launch_trace_fwd_batched(const rt_schedule& sc, const InstT<double>& I0, const InstT<double>* itab,
                             const int32_t* inst_of, int any_oblique, const TolC& T, const double* rays, int64_t n,
                             const FwdWs& W, double* fin, int32_t* ifin, hipStream_t st) {
    return launch_trace_variant<true>(sc, I0, itab, inst_of, any_oblique, T, rays, n, W, fin, ifin, st);
}

int launch_sample_batched(const InstT<double>* itab, const SeedT<double>* ctab, const int64_t* off, int32_t n_inst,
                          uint64_t seed, int64_t N, double* rays, int32_t* status, int32_t* inst_of, hipStream_t st) {
    hipLaunchKernelGGL(sample_batched_kernel, dim3(grid_for(N, 256, 8)), dim3(256), 0, st, itab, ctab, off, n_inst,
                       seed, N, rays, status, inst_of);
    return check_launch("sample_batched_kernel");
}

int launch_trace_init(const InstT<double>& I0, const InstT<double>* itab, const int32_t* inst_of, const TolC& T,
                      const double* rays, const int32_t* status, int64_t n, const FwdWs& W, double* fin,
                      int32_t* ifin, hipStream_t st) {
    hipLaunchKernelGGL(trace_keys_kernel, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, I0, itab, inst_of, rays,
                       status, n, W.keys, fin, ifin);
    int rc = check_launch("trace_keys_kernel");
    if (rc) return rc;
    rc = order_work_list(W, n, st);
    if (rc) return rc;
    hipLaunchKernelGGL(trace_init_kernel, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, I0, itab, inst_of, T, rays, n,
                       W.ctr, W.list, W.y0, W.h0, W.k1);
    return check_launch("trace_init_kernel");
}

}  // namespace rtd

namespace rtd {
int launch_bin(const double* fin, const int32_t* ifin, const double* w, int64_t n, const rt_bins* bins,
               const int64_t* inst_offset, int32_t n_inst, double* hist, double* cnt, double* over, void* ws,
               hipStream_t st) {
    int32_t ninst = inst_offset ? n_inst : 1;
    int64_t per = (int64_t)bins->n_theta * bins->n_psi * bins->n_omega;
    int64_t nbins = per * ninst;
    int zg = grid_for(nbins, 256, 4);
    hipLaunchKernelGGL(fill_kernel, dim3(zg), dim3(256), 0, st, hist, nbins, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3(zg), dim3(256), 0, st, cnt, nbins, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, over, (int64_t)2, 0.0);
    if (n == 0) return check_launch("fill_kernel");
    if (n > INT32_MAX) return fail(RT_EINVAL, "rt_bin_flux: n exceeds 2^31 - 1");
    BinWs B = carve_bin_ws(ws, n);
    int g1 = grid_for(n, 256, 8);
    hipLaunchKernelGGL(bin_keys_kernel, dim3(g1), dim3(256), 0, st, fin, ifin, n, bins->n_theta, bins->n_psi,
                       bins->n_omega, bins->d_omega, inst_offset, ninst, B.keys, w, over);
    const int64_t ntiles = (nbins + BIN_TILE - 1) / BIN_TILE;
    if (ntiles > PART_BUCKETS) {
        hipLaunchKernelGGL(bin_direct_kernel, dim3(grid_for(n, 256, 4)), dim3(256), 0, st, B.keys, w, n, hist, cnt);
        return check_launch("bin_direct_kernel");
    }
    int rc = partition_keys(B.keys, n, BIN_SHIFT, (int)ntiles, B.tab, B.start, B.list, nullptr, st);
    if (rc) return rc;
    // about 2048 workgroups over the tiles, none with fewer than ~256 rays on average
    int64_t slices = (2048 + ntiles - 1) / ntiles;
    const int64_t by_rays = n / (256 * ntiles);
    if (slices > by_rays) slices = by_rays;
    if (slices < 1) slices = 1;
    if (slices > 1024) slices = 1024;
    hipLaunchKernelGGL(bin_part_kernel, dim3((unsigned)ntiles, (unsigned)slices), dim3(256), 0, st, B.keys, w, B.list,
                       B.start, nbins, (int32_t)slices, hist, cnt);
    return check_launch("bin_part_kernel");
}
}  // namespace rtd

extern "C" int rt_bin_flux(const double* fin, const int32_t* ifin, const double* w, int64_t n, const rt_bins* bins,
                           const int64_t* inst_offset, int32_t n_inst, double* hist, double* cnt, double* over,
                           void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!bins || bins->n_theta <= 0 || bins->n_psi <= 0 || bins->n_omega <= 0 || !(bins->d_omega > 0.0))
        return fail(RT_EINVAL, "rt_bin_flux: invalid bins");
    if (n < 0) return fail(RT_EINVAL, "rt_bin_flux: negative n");
    if (inst_offset != nullptr && n_inst <= 0) return fail(RT_EINVAL, "rt_bin_flux: n_inst must be positive");
    int32_t ninst = inst_offset ? n_inst : 1;
    int64_t per = (int64_t)bins->n_theta * bins->n_psi * bins->n_omega;
    int64_t nbins = per * ninst;
    if (nbins > INT32_MAX) return fail(RT_EINVAL, "rt_bin_flux: too many bins");
    if (!hist || !cnt || !over) return fail(RT_EINVAL, "rt_bin_flux: null output");
    size_t need = rt_workspace_size(RT_OP_BIN, n);
    if (n > 0 && (!ws || ws_bytes < need)) return fail(RT_ENOWS, "rt_bin_flux: workspace too small");
    if (n > 0 && (!fin || !ifin || !w)) return fail(RT_EINVAL, "rt_bin_flux: null input");
    return launch_bin(fin, ifin, w, n, bins, inst_offset, n_inst, hist, cnt, over, ws, (hipStream_t)stream);
}


// ---------------------------------------------------------------------------
// rt_bin_flux_noalloc: the binning scratch in a static device array (one per device,
// resolved once per device and kept), for callers that cannot allocate
// ---------------------------------------------------------------------------
namespace {
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
// bin_ws_bytes(RT_NOALLOC_BIN_MAX_RAYS): keys and list, bucket starts, a full partition table
constexpr size_t NOALLOC_BIN_BYTES = 2 * al256(sizeof(int32_t) * (size_t)RT_NOALLOC_BIN_MAX_RAYS) +
                                     al256(sizeof(int32_t) * (PART_BUCKETS + 1)) +
                                     al256(sizeof(int32_t) * (size_t)PART_MAX_BLOCKS * PART_BUCKETS);
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BIN_BYTES];

// the array's address on the current device (host code never passes the array's name to
// a kernel: on the host it stands for no device address)
static void* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

extern "C" int rt_bin_flux_noalloc(const double* fin, const int32_t* ifin, const double* w, int64_t n,
                                   const rt_bins* bins, const int64_t* inst_offset, int32_t n_inst, double* hist,
                                   double* cnt, double* over, void* stream) {
    clear_error();
    if (n > (int64_t)RT_NOALLOC_BIN_MAX_RAYS)
        return fail(RT_EINVAL, "rt_bin_flux_noalloc: n exceeds RT_NOALLOC_BIN_MAX_RAYS (1048576 rays)");
    if (n >= 0 && bin_ws_bytes(n) > NOALLOC_BIN_BYTES)
        return fail(RT_EINVAL, "rt_bin_flux_noalloc: static workspace smaller than the binning needs");
    void* ws = scratch_on_current_device();
    if (ws == nullptr) return fail(RT_EHIP, "rt_bin_flux_noalloc: no address for the static workspace on this device");
    return rt_bin_flux(fin, ifin, w, n, bins, inst_offset, n_inst, hist, cnt, over, ws, NOALLOC_BIN_BYTES, stream);
}
