/* rt.h -- C ABI of the MI355X (gfx950) ray tracer for axion-photon conversion
 * around neutron stars (McDonald & Witte, "Generalized Ray Tracing for Axions
 * in Astrophysical Plasmas", arXiv:2309.08655).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments are DEVICE pointers to caller-owned, contiguous memory in
 *   structure-of-arrays layout: a "[F][n]" array holds field F of ray i at
 *   element F*n + i.  Struct arguments (rt_star, rt_tol, ...) are HOST memory,
 *   read during the call and not retained.
 * - Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *   NULL = the default stream).  No call allocates device memory, frees it or
 *   synchronises; scratch memory comes from a caller workspace whose size
 *   rt_workspace_size() reports.
 * - Return value: RT_OK (0) or a negative code.  Arguments are validated on the
 *   host before anything is launched; on error nothing is launched and
 *   rt_last_error() returns a message (thread-local).
 * - Per-ray outcomes are reported in status arrays (RT_ST_*), never as errors.
 * - Integrator units: lengths and times in km, covariant momentum in units of
 *   the axion energy at infinity w_inf = m_a sqrt(1 + v0^2) (so k_t = -1 at
 *   emission).  State order: (x, y, z, t, k_x, k_y, k_z, k_t), Cartesian chart
 *   of the Schwarzschild metric (x = r n with r the areal radius).
 * - Calls that overlap on one stream-ordered workspace race; distinct
 *   workspaces may run concurrently.
 */
#ifndef RT_H
#define RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RT_OK = 0, RT_EINVAL = -1, RT_EHIP = -2, RT_ENOWS = -3, RT_EUNSUPPORTED = -4 };

/* per-ray status */
enum { RT_ST_OK = 0, RT_ST_ESCAPED = 1, RT_ST_HIT_STAR = 2, RT_ST_NO_RESONANCE = 3,
       RT_ST_MAX_STEPS = 4, RT_ST_STEP_UNDERFLOW = 5, RT_ST_NONFINITE = 6, RT_ST_EXCISED = 7 };

enum { RT_PLASMA_ISO = 0, RT_PLASMA_ANISO = 1 };                /* Sec. 4.1 */
enum { RT_DENSITY_GJ = 0, RT_DENSITY_MAGNETAR = 1,              /* eqs. (GJDensity), (neMag) */
       RT_DENSITY_SPHERICAL = 2, RT_DENSITY_NONE = 3 };         /* test profiles */
enum { RT_WEIGHTS_UNIT = 0, RT_WEIGHTS_CONVERSION = 1, RT_WEIGHTS_CONST_B = 2 };
enum { RT_KDIR_ISOTROPIC = 0, RT_KDIR_OUTWARD = 1 };
enum { RT_SPEEDS_MONO = 0, RT_SPEEDS_MAXWELL = 1 };
/* rt_star.flags (bits):
   RT_FLAG_EXCISE_OPEN removes conversion on open magnetic field lines (Sec. 6:
     r / sin^2 theta_mag >= r_LC = c / Omega): such seeds get RT_ST_EXCISED and weight 0, such
     backward events weigh 0;
   the approximation variants (App. B; Sec. 6 eq. (reweight)), forward tracing only:
   RT_FLAG_FLAT_PROPAGATION seeds with curved initial conditions (static-frame momentum and
     local frequency) and traces with M = 0;
   RT_FLAG_RENORM_WEIGHTS sets P_ag = 1 and rescales each ray by
     R = (1 cm^-3 / n_a)(m_a / |k_a|)/sqrt(1 - r_s/r), i.e. w = C_k Vt |cos theta_n| m_a (1 cm^-3)/sqrt(A);
   RT_FLAG_THIN_SURFACE seeds on w_p = m_a instead of the foliation k^a = k^gamma; the photon
     keeps the axion's frequency and direction, |k| from the LO dispersion relation, and the
     weight is the un-cancelled |cos theta_n| v_a E P_ag;
   RT_FLAG_GR_DIPOLE replaces the flat dipole placed in the static frame by the static vacuum
     dipole of Schwarzschild (vector potential (mu sin^2 theta / r) G(r_s/r),
     G(x) = -3 [ln(1 - x) + x + x^2/2]/x^3), normalised to B0 at the surface pole: the field
     direction enters the LO Hamiltonian, its strength the conversion weights and the
     cyclotron depth; the Goldreich-Julian density keeps its printed form.  Everywhere
     (forward, backward, batched, adjoint);
   RT_FLAG_FINITE_LARMOR replaces the strong-field Hamiltonian (Sec. 4.1 eq. (StrongBHam)) by
     the cold magnetised plasma at finite magnetisation, eq. (DisRel) with eq. (Larmor):
     H = H_L / (w_L^2 w^2 k^2) = H_strong - (w^2 - w_p^2)(k^2 + w_p^2)^2 / (w_L^2 k^2), with
     k^2 = g^{mu nu} k_mu k_nu and w_L = e|B|/(m_e c) the electron cyclotron frequency of the
     dipole field; the resonance (photon on its shell at the axion's momentum), the seeds'
     momenta, the energy gradient of the weights and the traced rays follow it, while the
     conversion probability keeps eq. (CPAnisoCurved).  Anisotropic plasma only; seeding,
     forward tracing, binning and rt_flux_grad; not with RT_FLAG_THIN_SURFACE, the batched
     launch or the backward entry points (RT_EUNSUPPORTED).  The rays are meaningful where
     the plasma stays magnetised (w_L well above the plasma's share of the dispersion:
     the two magnetoionic modes do not meet), as everywhere inside r_max for the paper's
     stars. */
enum { RT_FLAG_EXCISE_OPEN = 1, RT_FLAG_FLAT_PROPAGATION = 2, RT_FLAG_RENORM_WEIGHTS = 4,
       RT_FLAG_THIN_SURFACE = 8, RT_FLAG_GR_DIPOLE = 16, RT_FLAG_FINITE_LARMOR = 32 };

/* Star, plasma and axion parameters (Sec. 5 fiducial set; Sec. 6 magnetar models). */
typedef struct rt_star {
    double B0_G;          /* polar surface dipole field [G] */
    double P_s;           /* rotation period [s] */
    double theta_m;       /* angle between magnetic and rotation axes [rad] */
    double M_Msun;        /* stellar mass [M_sun]; 0 = flat spacetime */
    double R_km;          /* stellar radius [km] */
    double m_a_eV;        /* axion mass [eV] */
    double g_agg_GeV;     /* axion-photon coupling [GeV^-1] */
    double v0_kms;        /* axion speed at infinity [km/s] */
    double rho_GeVcm3;    /* dark-matter density at infinity [GeV cm^-3] */
    double multiplicity;  /* charge multiplicity lambda */
    double psi_twist;     /* magnetar twist psi (RT_DENSITY_MAGNETAR) */
    double B_test_G;      /* constant |B_perp| used by RT_WEIGHTS_CONST_B [G] */
    int32_t plasma;       /* RT_PLASMA_* */
    int32_t density;      /* RT_DENSITY_* */
    int32_t weights;      /* RT_WEIGHTS_* */
    int32_t kdir;         /* RT_KDIR_*: axion directions isotropic or in the outward hemisphere */
    int32_t speeds;       /* RT_SPEEDS_*: axion momentum at infinity k0 = m_a v0 (Sec. 4.3 eq.
                             (fa_approx)) or Maxwellian with dispersion k0 (eq. (GaussianDist)) */
    int32_t flags;        /* RT_FLAG_* bits */
} rt_star;

/* Integrator tolerances: embedded DOPRI5 error test with scale atol + rtol max(|y|,|y_new|)
   over all 8 components; rays stop at r = r_max_km (located on the continuous extension). */
typedef struct rt_tol {
    double rtol, atol, r_max_km;
    int64_t max_steps;    /* accepted steps per ray before RT_ST_MAX_STEPS */
} rt_tol;

/* Sky binning (Sec. 2.2, the top-hat window D): n_theta bins of pi/n_theta in the polar
   angle, n_psi bins of 2 pi/n_psi in the co-rotating azimuth, n_omega bins of width
   d_omega in (w_f - 1) with the line centre w_f = 1 at the centre of bin n_omega/2. */
typedef struct rt_bins {
    int32_t n_theta, n_psi, n_omega;
    double d_omega;
} rt_bins;

/* Image plane of the backward tracer (Sec. 2.1): nx x ny square pixels of side
   2 half_width_km / nx centred on the line of sight at distance D_km, observer at polar
   angle incl and azimuth phi_o. */
typedef struct rt_image {
    double D_km, incl, phi_o, half_width_km;
    int32_t nx, ny;
} rt_image;

/* Launch schedule of the persistent tracing kernels (chosen by the autotuner). */
typedef struct rt_schedule {
    int32_t block;        /* threads per workgroup: 64, 128 or 256 */
    int32_t waves_per_cu; /* resident waves per CU requested (0 = occupancy limit) */
    int32_t refill_min;   /* idle lanes a wave waits for before refilling from the queue */
    int32_t occupancy;    /* register budget of the tracing kernels: 1 = one wave per SIMD (no
                             spills), 2 = two waves per SIMD (a few spills to scratch) */
    int32_t cross_batch;  /* forward tracing of the GJ density: crossings of the null surface a
                             wave lets wait before restarting them together (1..64; 0 = 8) */
    int32_t chunk;        /* queue chunk: work-list entries a wave claims at once and hands to
                             its idle lanes over several refills (64..65536); 0 = exactly the
                             idle lanes' worth at each refill (the default) */
} rt_schedule;

/* Number of doubles / int32 per final record (fin: "[RT_NFIN][n]", ifin: "[RT_NIFIN][n]"):
   fin  = x, y, z, t, k_x, k_y, k_z, k_t (final state), theta, phi, psi (co-rotating
          azimuth in [0, 2 pi)), omega (= -k_t), H, lambda, r, h_next
   ifin = accepted steps, rejected steps, status */
#define RT_NFIN 16
#define RT_NIFIN 3
/* backward event record: x, y, z, t, k_x, k_y, k_z, k_t, Doppler ratio (-k_t - 1),
   local frequency (-k_t / sqrt(A)) */
#define RT_NEV 10

enum { RT_OP_TRACE_FORWARD = 1, RT_OP_TRACE_BACKWARD = 2, RT_OP_BIN = 3, RT_OP_BATCHED = 4,
       RT_OP_FLUX_GRAD = 5, RT_OP_BACKWARD_POWER = 6 };

/* rt_sample_resonance -- seed forward rays on the resonance foliation and weight them
 * (Sec. 2.2 eq. (Power); Sec. 3 eqs. (Hypersurfaces), (ForwardTracingEquation1);
 *  Sec. 4.2 eq. (PowerCurved); Sec. 4.3 eq. (fa_approx); Sec. 4.4 eqs. (ProbIsoCurved),
 *  (CPAnisoCurved)).
 * Ray i (global index first + j) draws Philox4x32-10 uniforms with key = seed and counter
 * (i, instance, block); emission direction uniform in (cos theta, phi), axion direction
 * isotropic (or outward hemisphere), emission time uniform over one period; with
 * RT_SPEEDS_MAXWELL the sixth uniform gives |k_inf| by inverting the Maxwellian's
 * distribution function (Sec. 4.3 eq. (GaussianDist)), the ray's energy at infinity is
 * sqrt(m_a^2 + k_inf^2) (k_t = -that / (m_a sqrt(1 + v0^2))) and its focused density
 * n_inf |k_a| / k_inf.  The photon takes the axion's 4-momentum where the kinematic
 * matching k^a = k^gamma holds.
 * Output rays "[10][n]": x, y, z, t, k_x, k_y, k_z, k_t, w, r_c; status[n] = RT_ST_OK,
 * RT_ST_NO_RESONANCE or RT_ST_EXCISED (then w = 0; an excised ray keeps its r_c).  The unbiased power estimate is (1/n) sum w [eV^2].
 * Errors: RT_EINVAL for n < 0, null arrays or non-finite / out-of-range parameters. */
int rt_sample_resonance(const rt_star* star, uint64_t seed, int32_t instance, int64_t first, int64_t n,
                        double* rays, int32_t* status, void* stream);

/* rt_trace_forward -- integrate Hamilton's equations (Sec. 2 eq. (Hamilton)) with the
 * strong-field Hamiltonian (Sec. 4.1 eq. (StrongBHam)) from each seed to r = r_max with
 * adaptive FP64 Dormand-Prince 5(4), one ray per lane in a persistent work-queue kernel.
 * rays "[>=8][n]" (only the first 8 fields are read), status[n] (rays with status != OK are
 * copied through untraced).  Output fin "[RT_NFIN][n]", ifin "[RT_NIFIN][n]".
 * Workspace: rt_workspace_size(RT_OP_TRACE_FORWARD, n) bytes, device memory.
 * sched may be NULL (defaults).  Errors: RT_EINVAL, RT_ENOWS (workspace too small). */
int rt_trace_forward(const rt_star* star, const rt_tol* tol, const double* rays, const int32_t* status,
                     int64_t n, double* fin, int32_t* ifin, void* ws, size_t ws_bytes,
                     const rt_schedule* sched, void* stream);

/* rt_cyclotron_depth -- resonant cyclotron absorption of escaped forward rays (Sec. 6): the
 * photon is taken to move radially along its asymptotic direction from its final state; at
 * the radius where the electron cyclotron frequency of the dipole field equals the photon's
 * local frequency, tau = (pi/3) (w_p^2 / w) r.  rays "[>=10][n]" of rt_sample_resonance
 * (weight w = rays[8], emission radius r_c = rays[9]), fin/ifin of rt_trace_forward (device).
 * Output (device): tau[n] (0 for rays that do not escape, that have no resonance above the
 * surface, or that are emitted beyond it); r_cyc[n] the resonance radius [km] or -1 (may be
 * NULL); w_out[n] = w e^{-tau} (may be NULL), ready for rt_bin_flux.  Errors: RT_EINVAL. */
int rt_cyclotron_depth(const rt_star* star, const double* rays, const double* fin, const int32_t* ifin, int64_t n,
                       double* tau, double* r_cyc, double* w_out, void* stream);

/* rt_bin_flux -- top-hat sky/frequency binning of escaped rays (Sec. 2.2): hist and cnt are
 * "[n_theta][n_psi][n_omega]" (sum of w and ray count, both double, overwritten), over[2]
 * = (weight, count) of escaped rays outside the frequency range.  Bins are privatised in
 * LDS tiles and merged with FP64 atomics, so sums are exact up to summation order.
 * inst_offset: NULL for one instance, else a DEVICE array of n_inst + 1 ray offsets and
 * hist/cnt hold n_inst consecutive maps.  Workspace: rt_workspace_size(RT_OP_BIN, n). */
int rt_bin_flux(const double* fin, const int32_t* ifin, const double* w, int64_t n, const rt_bins* bins,
                const int64_t* inst_offset, int32_t n_inst, double* hist, double* cnt, double* over,
                void* ws, size_t ws_bytes, void* stream);

/* rt_bin_flux_noalloc -- rt_bin_flux for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * binning with no workspace argument.  Its scratch (every ray's bin key and tile-ordered
 * list entry, the partition table) lives in one static device array of the library, sized
 * for n <= RT_NOALLOC_BIN_MAX_RAYS rays (2^20 rays, 12.02 MiB), which every device the
 * library runs on holds until the process ends.  Arguments, results and errors are those
 * of rt_bin_flux; n above the maximum returns RT_EINVAL before anything is launched.  The
 * first call on a device resolves the array's address there (hipGetSymbolAddress; not a
 * stream operation) and keeps it; a failure returns RT_EHIP.  Every call on one device
 * shares that array, which keeps the last call's contents: calls that overlap on a device
 * (other streams, other threads) race, and the caller must serialise them.  Nothing in
 * the array has to start at zero: each call writes every entry it later reads. */
#define RT_NOALLOC_BIN_MAX_RAYS 1048576
int rt_bin_flux_noalloc(const double* fin, const int32_t* ifin, const double* w, int64_t n, const rt_bins* bins,
                        const int64_t* inst_offset, int32_t n_inst, double* hist, double* cnt, double* over,
                        void* stream);

/* rt_trace_backward -- trace the nx x ny parallel rays of an image plane backwards in the
 * worldline parameter (Sec. 2.1; Sec. 2.3 for the role of gravity) through every level
 * crossing k^gamma = k^a (sign change of G = g^{mu nu} k_mu k_nu + m_a^2, Sec. 3), until the
 * ray hits the star or recedes beyond 1.01 D.  The GJ density is integrated one smooth
 * piece at a time, as in rt_trace_forward: a step that crosses its null surface ends there,
 * its events searched only on the part taken.  k_t = -1 (monochromatic, Sec. 4.3), |k| from
 * the LO branch of eq. (AnisotropicDisp).  Events are sampled at 1/4, 1/2, 3/4 and 1 of
 * every accepted step and bisected on the continuous extension.
 * Output: ev "[K][RT_NEV][nx*ny]" (first K events per pixel, pixel index i*ny + j),
 * nev[nx*ny] (all crossings, may exceed K), fin/ifin as for rt_trace_forward.
 * Workspace: rt_workspace_size(RT_OP_TRACE_BACKWARD, nx*ny). */
int rt_trace_backward(const rt_star* star, const rt_tol* tol, const rt_image* image, int32_t K, double* ev,
                      int32_t* nev, double* fin, int32_t* ifin, void* ws, size_t ws_bytes,
                      const rt_schedule* sched, void* stream);

/* rt_trace_backward_rays -- as rt_trace_backward, for n rays through explicit points
 * (b1[q], b2[q]) [km] of the plane at distance D_km perpendicular to the line of sight
 * (inclination incl, azimuth phi_o) instead of a pixel grid: non-uniform sampling of the
 * asymptotic surface (Sec. 2.1), e.g. quadrature nodes of the image integral.  b1, b2:
 * device arrays [n]; outputs as for rt_trace_backward with ray index q.
 * Workspace: rt_workspace_size(RT_OP_TRACE_BACKWARD, n).  Errors: RT_EINVAL, RT_ENOWS. */
int rt_trace_backward_rays(const rt_star* star, const rt_tol* tol, double D_km, double incl, double phi_o,
                           const double* b1, const double* b2, int64_t n, int32_t K, double* ev, int32_t* nev,
                           double* fin, int32_t* ifin, void* ws, size_t ws_bytes, const rt_schedule* sched,
                           void* stream);

/* rt_backward_power -- the backward image sum of Sec. 2.1 eq. (BackPower), integrated over
 * frequency: each recorded production event adds P_ag f_a (Sec. 3) to its ray, with the
 * focused monochromatic axion density of Sec. 4.3 and P_ag of Sec. 4.4 (eqs.
 * (ProbIsoCurved), (CPAnisoCurved)); an event contributes w^3 sqrt(A) P_ag v_a n_c/(4 pi k^2)
 * [eV^4] per unit image area.  Events whose conversion length sqrt(2 pi v_a/|khat.dE|)
 * exceeds Lc_max_km are excluded (the IR cutoff of Sec. 4.4; Lc_max_km <= 0: no cutoff).
 * RT_WEIGHTS_CONST_B replaces |B_perp| by B_test_G; RT_WEIGHTS_UNIT is treated as
 * RT_WEIGHTS_CONVERSION.  Monochromatic axions only (RT_SPEEDS_MAXWELL: RT_EUNSUPPORTED; its
 * image would need a frequency integral over traced frequencies).
 * ev "[K][RT_NEV][n]", nev[n]: events of rt_trace_backward(_rays) (device; only the first
 * min(nev, K) events of a ray are stored, so only they count).  area: device [n] image area
 * element of each ray [km^2], or NULL for a uniform pixel_area_km2.
 * Output (device): wsum[n] = each ray's summed event weights [eV^4]; total[1] (may be NULL)
 * = sum_q area_q wsum_q / (hbar c)^2 = dP/dOmega [eV^2], reduced in a fixed order.
 * Workspace (only when total != NULL): rt_workspace_size(RT_OP_BACKWARD_POWER, n).
 * Errors: RT_EINVAL, RT_ENOWS. */
int rt_backward_power(const rt_star* star, const double* ev, const int32_t* nev, int64_t n, int32_t K,
                      double Lc_max_km, const double* area, double pixel_area_km2, double* wsum, double* total,
                      void* ws, size_t ws_bytes, void* stream);

/* Batched persistent launch (parameter scans): many star instances traced by one
 * persistent work-queue kernel.  Instances share plasma, density, weights and kdir; each
 * has its own parameters and ray count.  Instance k owns the global rays
 * [ray_offset[k], ray_offset[k+1]) and seeds ray i with Philox counter (i - ray_offset[k], k),
 * so its rays are identical to rt_sample_resonance(..., instance = k, first = 0, ...).  One
 * cost-ordered queue serves every instance (longest rays of all instances first); a lane
 * loads its ray's instance constants when it takes the ray. */
typedef struct rt_batch {        /* filled by rt_batch_prepare; plain host data */
    int32_t n_inst;
    int32_t any_oblique;
    int64_t n_rays;              /* N = ray_offset[n_inst] */
    int64_t n_bin_blocks;
    int32_t plasma, density;
    size_t ws_bytes;
} rt_batch;

/* Workspace bytes for a batch (device memory), from the HOST offsets array. */
size_t rt_batch_workspace_size(int32_t n_inst, const int64_t* ray_offset);

/* rt_batch_prepare -- validate the instances and upload their constant tables into the
 * workspace (HOST arrays stars[n_inst], ray_offset[n_inst+1]).  Synchronises `stream` once;
 * the host arrays may be released on return.  Not capturable; call it before capturing
 * rt_trace_batched.  Errors: RT_EINVAL (invalid or inconsistent instances), RT_ENOWS. */
int rt_batch_prepare(const rt_star* stars, int32_t n_inst, const int64_t* ray_offset, rt_batch* out, void* ws,
                     size_t ws_bytes, void* stream);

/* rt_trace_batched -- seed, order, trace (one persistent kernel over all instances),
 * finalise and bin every instance of a prepared batch.  Issues a fixed sequence of
 * kernels with no host synchronisation, allocation or memset, so it can be captured
 * into a hipGraph and replayed.  rays "[10][N]", status[N], fin "[RT_NFIN][N]",
 * ifin "[RT_NIFIN][N]", maps/cnt "[n_inst][n_theta][n_psi][n_omega]" (overwritten). */
int rt_trace_batched(const rt_batch* batch, uint64_t seed, const rt_tol* tol, const rt_bins* bins, double* rays,
                     int32_t* status, double* fin, int32_t* ifin, double* maps, double* cnt, void* ws,
                     size_t ws_bytes, const rt_schedule* sched, void* stream);

/* rt_flux_grad -- Gaussian-smoothed flux and its gradient with respect to the star
 * parameters p = (B0, P, theta_m, M, R, m_a), by a discretise-then-differentiate adjoint.
 *   F_j = (1/n) sum_{escaped i} w_i K(n_i . o_j),  K(c) = exp((c - 1)/sigma^2) / (2 pi sigma^2),
 * the forward estimator of Sec. 2.2 with the weights of Secs. 3-4, smoothed on the sky
 * so that it is differentiable; n_i is the arrival direction in the frame co-rotating
 * with the star (the direction that rt_trace_forward reports as (theta, psi)).
 * The derivative is that of the computed map: accepted DOPRI5 step sizes and each ray's
 * status frozen at the nominal p; resonance root, photon momentum and weight differentiated
 * through the seeding; the r = r_max crossing implicitly on the continuous extension; every
 * accepted step through its stages (Hamilton's equations, Sec. 2 eq. (Hamilton)).  Rays are
 * traced as rt_trace_forward traces them: for the GJ density one smooth piece at a time,
 * restarting where a step crosses the null surface g = 0; the restart point is
 * differentiated implicitly through g = 0 (with g's own dependence on Omega and theta_m).
 *   phase 0 (forward): seeds n rays (seed, instance 0), traces them with a checkpoint of
 *     (y, h, controller state, density piece) every ckpt_every accepted steps, writes flux[n_obs] (device)
 *     and, if ray_info != NULL, ray_info "[3][n]" = n_acc, n_rej, status (device).
 *     A ray that would need more than max_ckpt checkpoints ends as RT_ST_MAX_STEPS.
 *     Checkpoints go to a pool of ckpt_pool slots shared by all rays (a traced ray needs
 *     1 + (n_acc - 1) / ckpt_every of them, n_acc >= 1).  If ckpt_used != NULL, *ckpt_used (device int64)
 *     receives the number of slots the rays asked for.  The flux is valid either way; if
 *     the rays asked for more than ckpt_pool, the phase stores what fits and the reverse
 *     phase yields NaN: call phase 0 again with ckpt_pool >= *ckpt_used (the count depends
 *     only on the arguments, not on the pool or the schedule).
 *   phase 1 (reverse): given gbar[n_obs] (device), recomputes each segment from its
 *     checkpoint and sweeps back through the stages; writes grad[6] = sum_j gbar_j dF_j/dp
 *     (device) and, if grad_rays != NULL, each ray's share "[n][6]" (zero for rays that
 *     do not escape).  Needs the workspace of the phase-0 call of the same arguments,
 *     unchanged; phase-1 calls may be repeated with other gbar.
 * obs: HOST array "[n_obs][3]" of unit vectors, 1 <= n_obs <= 64; sigma > 0 [rad];
 * 1 <= ckpt_every <= 1024; max_ckpt >= 1; 1 <= ckpt_pool <= 2^31 - 1; weights
 * RT_WEIGHTS_CONST_B is not supported.
 * Workspace: rt_flux_grad_workspace_size(n, n_obs, ckpt_every, ckpt_pool) bytes (about
 * 120 n + 96 ckpt_pool + max(5.8 MB x ckpt_every, 264 n + 50 MB) + 4 MB: the reverse phase's
 * replay buffer shares its bytes with what only the forward phase uses).  Returns RT_OK, RT_EINVAL, RT_ENOWS,
 * RT_EUNSUPPORTED or RT_EHIP. */
int rt_flux_grad(const rt_star* star, const rt_tol* tol, uint64_t seed, int64_t n, const double* obs,
                 int32_t n_obs, double sigma, int32_t ckpt_every, int32_t max_ckpt, int64_t ckpt_pool, int32_t phase,
                 const double* gbar, double* flux, double* grad, double* grad_rays, int32_t* ray_info,
                 int64_t* ckpt_used, void* ws, size_t ws_bytes, void* stream);

size_t rt_flux_grad_workspace_size(int64_t n, int32_t n_obs, int32_t ckpt_every, int64_t ckpt_pool);

/* Workspace bytes needed by op (RT_OP_*) for n rays; RT_OP_FLUX_GRAD is
 * rt_flux_grad_workspace_size(n, 64, 64, 2 n + 1). */
size_t rt_workspace_size(int32_t op, int64_t n);

/* Kernel timing.  rt_timing(1) starts recording (and forgets earlier records): every
 * later launch of a persistent tracing kernel (trace_fwd_kernel of rt_trace_forward or
 * rt_trace_batched, trace_bwd_kernel of rt_trace_backward(_rays), the forward and reverse
 * kernels of rt_flux_grad) and of the event-weight kernel of rt_backward_power is bracketed by a HIP event pair recorded on the caller's
 * stream, up to 1024 launches; rt_timing(0) stops recording.  rt_kernel_times waits
 * for the recorded launches and writes up to max durations [ms] and kernel kinds
 * (RT_KERNEL_*) in launch order; returns the count.  This is a measurement aid with
 * one record list for the whole process (every thread, stream and device): the
 * library's only mutable global besides the thread-local error string.  Its state is
 * guarded by a mutex, so concurrent calls are safe and their launches interleave in
 * the list in the order they were issued; a launch still in flight on another thread
 * when rt_kernel_times runs is left out.  Recording must be off while a stream is
 * being captured into a graph. */
enum { RT_KERNEL_TRACE_FORWARD = 1, RT_KERNEL_TRACE_BATCHED = 2, RT_KERNEL_TRACE_BACKWARD = 3,
       RT_KERNEL_ADJOINT_FORWARD = 4, RT_KERNEL_ADJOINT_REVERSE = 5, RT_KERNEL_EVENT_POWER = 6 };
int rt_timing(int32_t on);
int32_t rt_kernel_times(double* ms, int32_t* kind, int32_t max);

/* Message of the last failed call on this thread ("" if none). */
const char* rt_last_error(void);

/* Library build string (compiler, target). */
const char* rt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
