/*
 * glasma_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded FP64 CPU reference of the boost-invariant SU(3)
 * Glasma evolved on a transverse lattice, coupled to a colored-particle-in-cell
 * solution of Wong's equations (Avramescu et al., "Heavy quark kappa and jet
 * qhat transport coefficients in the Glasma early stage of heavy-ion
 * collisions", Hard Probes 2023).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the HIP library.
 *
 * Conventions (all quantities in lattice units, a = 1, g absorbed in fields):
 *   site index          x = ix + N*iy, periodic in both directions
 *   3x3 complex matrix  18 doubles, row-major, (re, im) interleaved
 *   link array   U      [2][N*N][18]   direction 0 = x, 1 = y
 *   algebra array       [..][8]        components X^a = 2 Tr(T^a X), T^a = lambda^a/2
 *   E array             [2][N*N][8]
 *   phi, pi arrays      [N*N][8]
 *   site-field array F  [N*N][6][8]    order Ex, Ey, Ez, Bx, By, Bz (local frame)
 *   particle arrays     cell [np][2] int32, off [np][2], eta [np], p [np][3]
 *                       = (px, py, P_eta), Q [np][8], p0 [np][3] = (px0, py0, pz0_lab),
 *                       species [np] int32
 *   series              [nspecies][4] = (sum dpx^2, sum dpy^2, sum dpz^2, n_active)
 *
 * Return codes: 0 ok, -1 bad argument, -3 matching did not converge.
 */
#ifndef GLASMA_ORACLE_H
#define GLASMA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- SU(3) algebra helpers (exposed for the pins) ---------------------- */
void orc_generator(int a, double *T18);                 /* T^a as a 3x3 matrix   */
double orc_dsym(int a, int b, int c);                   /* d_abc = 2Tr({Ta,Tb}Tc) */
void orc_expi(const double *x8, double *U18);           /* exp(i x^a T^a)         */
void orc_expm(const double *A18, double *out18);        /* exp of any 3x3 matrix  */
void orc_proj(const double *M18, double *x8);           /* components of [M]_X    */

/* ---- counter-based random numbers (Philox4x32-10, Salmon et al. 2011) -- */
void orc_philox(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]);
double orc_u53(uint32_t lo, uint32_t hi);               /* uniform in (0,1)       */

/* ---- initial conditions ------------------------------------------------ */
/* Gaussian MV charges of one (nucleus, sheet): rho [N*N][8], variance sigma^2. */
void orc_mv_charges(int N, double sigma, uint64_t seed, int nucleus, int sheet,
                    double *rho);
/* Complex 1-D DFT by recursive radix-2/3 decimation; sign -1 forward. */
int orc_fft(int n, double *data_re_im, int sign);
/* Solve (-Lap + m2) out = src on the periodic N x N lattice (one real plane). */
int orc_poisson(int N, double m2, const double *src, double *out);
/* Same with a UV regulator: Fourier modes with lattice momentum squared
 * 4 sin^2(pi kx/N) + 4 sin^2(pi ky/N) > uv2 are removed (uv2 <= 0: none). */
int orc_poisson_uv(int N, double m2, double uv2, const double *src, double *out);
/* Wilson line of one nucleus, V = prod_s exp(-i Lambda_s), V [N*N][18]. */
int orc_wilson_line(int N, double sigma, double m2, int n_sheets, uint64_t seed,
                    int nucleus, double *V);
int orc_wilson_line_uv(int N, double sigma, double m2, double uv2, int n_sheets, uint64_t seed,
                       int nucleus, double *V);
/* Pure-gauge nucleus links U_i(x) = V(x) V^dag(x+i), Un [2][N*N][18]. */
void orc_nucleus_links(int N, const double *V, double *Un);
/* Solve [(UA+UB)(1+U^dag)]_X = 0 for one link; returns iterations or -3. */
int orc_match_link(const double *UA, const double *UB, double *U, double tol,
                   int max_iter, double *res_out);
/* Initial longitudinal field pi0 [N*N][8] from matched and nucleus links. */
void orc_pi0(int N, const double *U, const double *UA, const double *UB,
             double *pi0);
/* Whole initial condition: state at step 1 (U^1, phi^1; E^{1/2}, pi^{1/2}). */
int orc_init_glasma(int N, double sigma, double m2, int n_sheets, uint64_t seed,
                    double dtau, double *U, double *E, double *phi, double *pi,
                    double *max_res_out);
int orc_init_glasma_uv(int N, double sigma, double m2, double uv2, int n_sheets, uint64_t seed,
                       double dtau, double *U, double *E, double *phi, double *pi,
                       double *max_res_out);

/* ---- field evolution --------------------------------------------------- */
/* Forces at time tau: dE/dtau [2][N*N][8], dpi/dtau [N*N][8]. */
void orc_forces(int N, double tau, const double *U, const double *phi,
                double *FE, double *Fpi);
/* One leapfrog step n -> n+1 (n >= 1), in place.  If F is non-null the site
 * fields at tau_n are written there.  If reunit_period > 0 nothing changes
 * (the oracle never reunitarizes); the argument is reserved. */
void orc_field_step(int N, int n, double dtau, double *U, double *E,
                    double *phi, double *pi, double *F);
/* The same step evaluated only at listed sites, reading whole-lattice inputs;
 * outputs per listed site: U_new [ns][2][18], E_new [ns][2][8], phi_new [ns][8],
 * pi_new [ns][8], F [ns][6][8]. */
void orc_field_step_sites(int N, int n, double dtau, const double *U,
                          const double *E, const double *phi, const double *pi,
                          int ns, const int *sites, double *U_new, double *E_new,
                          double *phi_new, double *pi_new, double *F);
/* Energy per unit rapidity at tau, split in (E_T, E_L, B_T, B_L) terms:
 * E_T = sum Tr E_i^2 / tau, E_L = tau sum Tr pi^2,
 * B_T = sum Tr(Phi_{+i}-phi)^2 / tau, B_L = 2 tau sum (3 - Re Tr P). */
void orc_energy(int N, double tau, const double *U, const double *E,
                const double *phi, const double *pi, double out[4]);
/* Gauss-law residual G(x) [N*N][8]. */
void orc_gauss(int N, const double *U, const double *E, const double *phi,
               const double *pi, double *G);

/* ---- particles ---------------------------------------------------------- */
/* Initialise np particles of one species (stream 2 + species_id). kind 0:
 * heavy quark, |p_T| = p0 with uniform azimuth; kind 1: jet along +x. */
void orc_particles_init(int N, uint64_t seed, int species_id, int kind,
                        double p0, int np, int *cell, double *off, double *eta,
                        double *p, double *Q, double *p0v);
/* One particle step n -> n+1 for particles with n >= nform[species].
 * U, phi are U^n, phi^n; F the site fields at tau_n.  Adds the broadening
 * sums at tau_{n+1/2} to series [nspecies][4] (not cleared here). */
void orc_particle_step(int N, int n, double dtau, const double *U,
                       const double *phi, const double *F, int np, int *cell,
                       double *off, double *eta, double *p, double *Q,
                       const double *p0v, const int *species, int nspecies,
                       const double *mass, const int *nform, double *series);

/* ---- whole run ---------------------------------------------------------- */
/* Initial Glasma + particles, then n_steps coupled steps starting at n = 1.
 * series_out [n_steps][nspecies][4]; the final fields and particles are
 * returned in the caller's arrays (particle arrays must be sized sum(np)). */
int orc_run(int N, double sigma, double m2, int n_sheets, uint64_t seed,
            double dtau, int n_steps, int nspecies, const int *kind,
            const double *mass, const double *p0, const int *nform,
            const int *np, double *U, double *E, double *phi, double *pi,
            int *cell, double *off, double *eta, double *p, double *Q,
            double *p0v, int *species, double *series_out);

#ifdef __cplusplus
}
#endif
#endif
