/* CPU oracle: plain FP64 reference of the ray-tracing hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, constant table or generator with the GPU library; the two are
 * written independently from the paper (McDonald & Witte, "Generalized Ray
 * Tracing for Axions in Astrophysical Plasmas", arXiv:2309.08655).
 *
 * Conventions (all arrays are host memory, caller-owned):
 *   state y = (x, y, z, t, k_x, k_y, k_z, k_t): Cartesian Schwarzschild chart,
 *   lengths and times in km, covariant momentum in units of the axion energy
 *   at infinity (so k_t = -1 at emission).
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double B0_G;          /* polar surface field [G] */
    double P_s;           /* rotation period [s] */
    double theta_m;       /* magnetic inclination [rad] */
    double M_Msun;        /* stellar mass [solar masses] */
    double R_km;          /* stellar radius [km] */
    double m_a_eV;        /* axion mass [eV] */
    double g_agg_GeV;     /* axion-photon coupling [GeV^-1] */
    double v0_kms;        /* axion speed at infinity [km/s] */
    double rho_GeVcm3;    /* dark-matter density [GeV cm^-3] */
    double multiplicity;  /* charge multiplicity lambda */
    double psi_twist;     /* magnetar twist psi */
    double B_test_G;      /* constant |B_perp| for the zero-variance weight test */
    int32_t plasma;       /* 0 isotropic, 1 anisotropic (strong-B LO mode) */
    int32_t density;      /* 0 Goldreich-Julian, 1 magnetar, 2 spherical test, 3 none */
    int32_t weights;      /* 0 unit, 1 conversion, 2 conversion with constant |B_perp| */
    int32_t kdir;         /* 0 isotropic axion directions, 1 outward hemisphere */
    int32_t speeds;       /* 0 every axion at |k_inf| = m_a v0; 1 Maxwellian |k_inf|, dispersion k0 = m_a v0 */
    int32_t flags;        /* ORC_FLAG_* bits: 1 no conversion on open field lines (r / sin^2 theta_mag >= c/Omega);
                             2 flat propagation (curved initial conditions, M = 0 in the tracing);
                             4 renormalised weights (P_ag = 1 times R_i); 8 thin surface w_p = m_a;
                             16 the Schwarzschild vacuum dipole instead of the flat one;
                             32 finite magnetisation: the cold magnetised plasma response at the local
                             electron cyclotron frequency (Sec. 4.1 eqs. (DisRel), (Larmor)) instead of
                             its strong-field limit (anisotropic plasma, forward tracing) */
} orc_star;

typedef struct {
    double rtol, atol, r_max_km;
    int64_t max_steps;
} orc_tol;

enum { ORC_OK = 0, ORC_ESCAPED = 1, ORC_HIT_STAR = 2, ORC_NO_RESONANCE = 3,
       ORC_MAX_STEPS = 4, ORC_STEP_UNDERFLOW = 5, ORC_NONFINITE = 6, ORC_EXCISED = 7 };
enum { ORC_FLAG_EXCISE_OPEN = 1, ORC_FLAG_FLAT_PROPAGATION = 2, ORC_FLAG_RENORM_WEIGHTS = 4,
       ORC_FLAG_THIN_SURFACE = 8, ORC_FLAG_GR_DIPOLE = 16, ORC_FLAG_FINITE_LARMOR = 32 };

/* number of doubles per final record and their order */
#define ORC_NFIN 16  /* y_f[8], theta, phi, psi, omega, H_f, lam_f, r_f, h_last */
#define ORC_NIFIN 3  /* n_acc, n_rej, status */
#define ORC_NEV 10   /* event record: y[8], doppler, local frequency */

int orc_constants(double* out, int n);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_uniforms(uint64_t seed, int32_t instance, int64_t i, double u[6]);

double orc_wp2(const orc_star* s, const double x[3], double t);
void orc_bfield(const orc_star* s, const double x[3], double t, double B[3]);
double orc_hamiltonian(const orc_star* s, const double y[8]);
void orc_grad_h(const orc_star* s, const double y[8], double g[8]);
void orc_inverse_metric(const orc_star* s, const double x[3], double gi[9]);

/* seeds: rays[10][n] = x,y,z,t,kx,ky,kz,kt,w,r_c ; status[n] */
int orc_sample(const orc_star* s, uint64_t seed, int32_t instance, int64_t first, int64_t n,
               double* rays, int32_t* status, int nthreads);
/* root of the resonance function along direction nhat at time t0 for axion direction khat */
double orc_resonance_radius(const orc_star* s, const double nhat[3], const double khat[3], double t0);
/* local photon frequency (units of w_inf) of the LO branch at covariant spatial k: eq.
   (AnisotropicDisp) '+', or with ORC_FLAG_FINITE_LARMOR the root of eq. (DisRel) that
   continues it */
double orc_energy_aniso(const orc_star* s, const double x[3], double t, const double k[3]);

/* forward trace: rays[10][n] as produced by orc_sample (w and r_c unused);
   status_in[n]; fin[ORC_NFIN][n]; ifin[ORC_NIFIN][n].  kinks != 0: for the GJ density,
   one smooth piece at a time, cut and restarted at every crossing of the null surface
   (the forward-tracing definition); kinks = 0: the density |g| as it stands, as the
   adjoint's discretised map integrates it */
int orc_trace_forward(const orc_star* s, const orc_tol* tol, const double* rays, const int32_t* status_in,
                      int64_t n, double* fin, int32_t* ifin, int nthreads, int kinks);
/* same, backward in the worldline parameter (for the time-reversal check) */
int orc_trace_reverse(const orc_star* s, const orc_tol* tol, const double* rays, int64_t n,
                      double lam_stop_abs, double* fin, int32_t* ifin, int nthreads);

/* histogram: hist[nt][np][nw] (sum of w), cnt likewise, over[2] = {under/over-range weight, count} */
int orc_bin(const double* fin, const int32_t* ifin, const double* w, int64_t n, int32_t nt, int32_t np,
            int32_t nw, double dw, double* hist, double* cnt, double* over);

/* backward image: events ev[K][ORC_NEV][n], nev[n], fin[ORC_NFIN][n], ifin[ORC_NIFIN][n];
   pixels (i, j) with i in [i0, i0+ni*stride) step stride, likewise j */
int orc_trace_backward(const orc_star* s, const orc_tol* tol, double D_km, double incl, double phi_o,
                       double half_width_km, int32_t nx, int32_t ny, int32_t i0, int32_t j0, int32_t stride,
                       int32_t ni, int32_t nj, int32_t K, double* ev, int32_t* nev, double* fin,
                       int32_t* ifin, int nthreads);

/* backward rays through explicit image-plane points (b1, b2) [km]; wsum[n] = sum over the
   ray's recorded production events of the event weight dP/dOmega per unit image area
   [eV^4] (Sec. 2.1 eq. (BackPower) with the Sec. 4.3-4.4 f_a and P_ag), events with
   conversion length above Lc_max_km excluded when Lc_max_km > 0 */
int orc_backward_rays(const orc_star* s, const orc_tol* tol, double D_km, double incl, double phi_o,
                      const double* b1, const double* b2, int64_t n, int32_t K, double Lc_max_km, double* wsum,
                      double* ev, int32_t* nev, double* fin, int32_t* ifin, int nthreads);
/* resonant cyclotron optical depth of Sec. 6 for each escaped forward ray (fin, ifin as
   written by orc_trace_forward, r_emit[n] = emission radii): tau[n] (0 for other rays) */
int orc_cyclotron_depth(const orc_star* s, const double* fin, const int32_t* ifin, const double* r_emit, int64_t n,
                        double* tau, double* r_cyc);
/* whether x (at time t) lies on an open field line of the rotating dipole */
int orc_open_field(const orc_star* s, const double* x, double t);

/* x = (|k_inf|/k0)^2 at quantile u of the Maxwellian of Sec. 4.3 eq. (GaussianDist) */
double orc_maxwell_x(double u);
/* the weight of one production event at state y[8] (and its conversion length [km]) */
int orc_event_weight(const orc_star* s, const double* y, double Lc_max_km, double* w, double* Lc);

/* integrator pins: problem 0 = harmonic oscillator y'' = -y (state 8: pairs),
   problem 1 = exponential growth y' = y.  Returns final state and dense samples. */
int orc_dopri_test(int32_t problem, double rtol, double atol, double t_end, double* y_end,
                   int64_t* n_acc, int64_t* n_rej, double h_fixed, double* dense_err);

/* smoothed flux and its forward-mode derivative with respect to
   (B0, P, theta_m, M, R, m_a); steps frozen at the nominal run.  Rays are traced as
   orc_trace_forward does with kinks != 0 (the GJ density one smooth piece at a time),
   restart points carrying the implicit derivative of g(y(theta)) = 0.  If fray/dray are
   not NULL they receive each ray's share (w K / n and its derivative; zero for rays
   that do not escape) and ray_status each ray's status. */
int orc_flux_fwdmode(const orc_star* s, const orc_tol* tol, uint64_t seed, int64_t n,
                     const double* obs /*[n_obs][3]*/, int32_t n_obs, double sigma,
                     double* flux /*[n_obs]*/, double* dflux /*[n_obs][6]*/, double* fray /*[n][n_obs] or NULL*/,
                     double* dray /*[n][n_obs][6] or NULL*/, int32_t* ray_status /*[n] or NULL*/, int nthreads);
/* smoothed flux with a replayed step sequence (for frozen-step finite differences);
   hseq[n][max_steps] step sizes recorded by a nominal run when record != 0 */
int orc_flux_replay(const orc_star* s, const orc_tol* tol, uint64_t seed, int64_t n,
                    const double* obs, int32_t n_obs, double sigma, int32_t record, int32_t max_rec,
                    double* hseq, int32_t* nseq, int32_t* stat, double* flux, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
