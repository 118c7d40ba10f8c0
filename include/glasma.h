/*
 * glasma.h -- C-ABI of the MI355X (gfx950) library for the boost-invariant
 * SU(3) Glasma coupled to a colored-particle-in-cell solution of Wong's
 * equations (Avramescu et al., "Heavy quark kappa and jet qhat transport
 * coefficients in the Glasma early stage of heavy-ion collisions", Hard
 * Probes 2023).
 *
 * The calls follow the paper's statement of the problem:
 *   gl_init_glasma          MV color sources -> Glasma at tau = 0+   (Sec. 1 "Glasma")
 *   gl_evolve_fields        classical Yang-Mills on links, Eq. (1)    (Sec. 1 "Glasma")
 *   gl_push_particles       Wong's equations, Eq. (2), CPIC colors    (Sec. 1 "Probes in Glasma")
 *   gl_broadening / gl_kappa / gl_qhat   <dp_i^2>, Eq. (3)            (Sec. 2)
 *
 * Conventions
 *   - Every function returns gl_status (0 = GL_OK, negative = error) and never
 *     throws.  gl_last_error() returns a thread-local message for the last
 *     error on the calling thread.
 *   - Units at the boundary are GeV and fm.  Inside, a = 1 and g is absorbed
 *     into the fields (gA -> A).
 *   - Device memory is owned by the caller.  gl_required_bytes() gives the
 *     size of one workspace; the caller allocates it (256-byte aligned) and
 *     passes it to gl_event_create(); it must outlive the event.  The library
 *     allocates no device memory of its own.
 *   - All device work is ordered on the hipStream_t given at creation (passed
 *     as void*).  Calls that return host data synchronise that stream.
 *   - An event is not thread-safe; distinct events on distinct streams are
 *     independent.
 *
 * Array layouts used by the host-side getters/setters (all FP64, host memory,
 * structure of arrays, site index x = ix + N*iy):
 *   U    [2][18][N*N]  link U_i(x), i = 0 (x) or 1 (y); 18 = row-major 3x3,
 *                      real and imaginary parts interleaved per entry
 *   E    [2][8][N*N]   E_i^a(x) = 2 Tr(T^a E_i(x)), T^a = lambda^a/2
 *   phi  [8][N*N]      A_eta components
 *   pi   [8][N*N]      E_eta components
 *   F    [6][8][N*N]   local-frame site fields Ex, Ey, Ez, Bx, By, Bz at tau_n
 *   particles: cell [2][n] int32, off [2][n], eta [n], p [3][n] = (px, py, P_eta
 *   = tau^2 p^eta), Q [8][n], p0 [3][n] = (px, py, pz_lab) at formation,
 *   species [n] int32, in creation order.
 *
 * Time grid: tau_n = n * dtau with dtau = dtau_over_a * a.  After
 * gl_init_glasma the state is at n = 1 (U^1, phi^1; E, pi at tau_{1/2}).
 * One field step takes n -> n+1; one particle step does too.
 */
#ifndef GLASMA_H
#define GLASMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gl_status;
#define GL_OK        0
#define GL_EINVAL   (-1)   /* bad argument                                 */
#define GL_ESTATE   (-2)   /* call not allowed in the event's current state */
#define GL_ENOTCONV (-3)   /* a link of the initial-condition matching did not converge */
#define GL_ENUMERIC (-4)   /* non-finite value found by the diagnostics    */
#define GL_EDEVICE  (-5)   /* a HIP runtime call failed                    */
#define GL_ENOMEM   (-6)   /* workspace too small                          */

#define GL_MAX_SPECIES 16

typedef struct gl_event gl_event;

/* Lattice and run description. */
typedef struct {
    int32_t N;              /* transverse sites per direction, 2 <= N <= 1024, N = 2^a 3^b for MV init */
    double  L_fm;           /* transverse box size; a = L/N */
    double  dtau_over_a;    /* leapfrog step in lattice units (the paper's runs: 1/8) */
    int32_t precision;      /* 64 (FP64 fields/particles) or 32 (FP32 fields/particles, FP64 sums) */
    int32_t reunit_every;   /* FP32 only: re-unitarise links when n % reunit_every == reunit_every-1; 0 = never */
    int32_t max_steps;      /* capacity of the broadening series (rows) */
    int64_t max_particles;  /* particle capacity over all species (padding included by the library);
                               at most gl_max_particles(precision), 19173888 (FP64) or 33554176
                               (FP32); GL_EINVAL above */
    int32_t static_correlator; /* nonzero: reserve the static-quark accumulators (gl_static_start) */
    int32_t lightlike_correlator; /* nonzero: reserve the lightlike-jet accumulators (gl_lightlike_start) */
} gl_lattice_desc;

/* MV-model description (Sec. 1 "Glasma"): per-sheet charge variance
 * (g^2 mu)^2 / (n_sheets a^2), infrared regulator m in the Poisson solve, and
 * an optional UV regulator: Fourier modes whose lattice momentum
 * 2 sqrt(sin^2(pi kx/N) + sin^2(pi ky/N)) / a exceeds uv_cut_GeV are dropped
 * (0: no cut), which makes the initial fields independent of the lattice
 * spacing once a is fine enough. */
typedef struct {
    double  g2mu_GeV;
    double  m_ir_GeV;
    int32_t n_sheets;
    double  uv_cut_GeV;
} gl_mv_desc;

/* Particle species (Sec. 2, toy initialisation). */
#define GL_KIND_HEAVY_QUARK 0   /* |p_T| = p0 with uniform azimuth */
#define GL_KIND_JET         1   /* p = (p0, 0, 0) along +x        */
typedef struct {
    double  mass_GeV;
    double  p0_GeV;
    int32_t kind;
    double  tau_form_fm;    /* < 0: 1/(2 m_T) with m_T = sqrt(m^2 + p0^2) */
} gl_species_desc;

typedef struct {
    double gauss_max;        /* max |G^a(x)| of the Gauss-law residual */
    double gauss_rel;        /* gauss_max / max |E^a|                   */
    double unitarity_max;    /* max |U U^dag - 1| entry                 */
    double energy[4];        /* (E_T, E_L, B_T, B_L) per unit rapidity, lattice units, at the stored times */
    double casimir2_dev;     /* max |Q^aQ^a - 4| over the particles     */
    double casimir3_dev;     /* max |d_abc Q^aQ^bQ^c - 10/3| over the particles */
    int32_t nonfinite;       /* 1 if any NaN/Inf in the fields          */
} gl_diag;

/* Workspace size for an event.  Pure function. */
gl_status gl_required_bytes(const gl_lattice_desc *desc, size_t *bytes);

/* Largest max_particles an event of this precision (64 or 32) accepts: the
 * particle record, in 16-byte chunk planes over all slots, must stay within
 * 32-bit byte offsets.  Pure function; GL_EINVAL for another precision. */
gl_status gl_max_particles(int32_t precision, int64_t *max_particles);

/* Create an event on a caller-owned workspace and stream (hipStream_t). */
gl_status gl_event_create(const gl_lattice_desc *desc, void *workspace, size_t bytes,
                          void *stream, gl_event **out);
/* Free the event's host state (and its graphs and timing events, after the
 * stream is done with them).  Work already queued on the stream may still
 * read and write the workspace: the caller frees the workspace only after
 * that work has completed (synchronise the stream, or order the release after
 * it).  An event held by a batch is destroyed only after the batch. */
void gl_event_destroy(gl_event *ev);

/* MV sources -> Glasma (Sec. 1): charges drawn on the device from Philox4x32-10
 * (key = seed, counter = (site, 4*sheet + j, nucleus, 0)), Poisson solve,
 * Wilson lines, matching of the two nuclei, initial longitudinal field and
 * the first half step.  Returns GL_ENOTCONV if a link did not converge. */
gl_status gl_init_glasma(gl_event *ev, const gl_mv_desc *mv, uint64_t seed);

/* Same from caller-supplied charges rho (device, FP64) laid out
 * [2][n_sheets][8][N*N] in lattice units (no UV cut). */
gl_status gl_init_glasma_from_charges(gl_event *ev, const double *rho_dev, int32_t n_sheets,
                                      double m_ir_GeV);

/* Add n particles of one species (Sec. 2 toy model); draws from Philox with
 * counter (i, j, 2 + species_id, 0).  Species ids are 0, 1, ... in call order. */
gl_status gl_add_species(gl_event *ev, const gl_species_desc *sp, int64_t n, uint64_t seed,
                         int32_t *species_id);

/* Fields only: n_steps leapfrog steps.  GL_ESTATE if particles are behind
 * the field time (a gl_push_particles is due). */
gl_status gl_evolve_fields(gl_event *ev, int32_t n_steps);
/* One particle step tau_n -> tau_{n+1} with the field snapshot at tau_n;
 * must follow gl_evolve_fields(ev, 1) when the event has particles. */
gl_status gl_push_particles(gl_event *ev);
/* Hot path: n_steps x (one field step + one particle step). */
gl_status gl_run(gl_event *ev, int32_t n_steps);

/* Observables of one species (Sec. 2, Eq. (3)).
 * gl_broadening rows: (tau_fm, <dpx^2>, <dpy^2>, <dpz^2>, n_active) in GeV^2,
 *   at the half steps tau_{n+1/2} where the species is active.
 * gl_kappa rows: (tau_fm, tau - tau_form, kappa_T, kappa_L) in GeV^2/fm at tau_n.
 * gl_qhat rows: (tau_fm, qhat_y, qhat_z) in GeV^2/fm at tau_n.
 * cap is the row capacity of out; *n_rows receives the row count. */
gl_status gl_broadening(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows);
gl_status gl_kappa(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows);
gl_status gl_qhat(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows);
/* Raw FP64 series [rows][GL_MAX_SPECIES][4] = (sum dpx^2, sum dpy^2, sum dpz^2,
 * n_active) in lattice units; row k holds tau_{k+1+1/2}. */
gl_status gl_series(gl_event *ev, double *out, int32_t cap_rows, int32_t *n_rows);

/* Same derivative as gl_kappa on a host series of one species, for callers
 * that hold their own series: series [rows][4] (lattice units), rate out
 * [rows][3] (lattice units); rows before formation are set to 0. */
gl_status gl_rates_from_series(const double *series, int32_t rows, double dtau,
                               double *rates);

/* Event statistics of the broadening (Sec. 2: <dp_i^2> is averaged over the
 * particle trajectories and over Glasma events; the paper's scans are
 * curves of it and of its derivative with that averaging).  series holds,
 * for each of n_events >= 2 events, the raw series of one species as
 * gl_series gives it, [n_events][rows][4] = (sum dpx^2, sum dpy^2, sum dpz^2,
 * n_active) in lattice units, on the same time grid (row k: tau_{k+1+1/2}).
 * The components are A = dp_x^2 + dp_y^2 (transverse) and B = dp_z^2
 * (longitudinal) for kind GL_KIND_HEAVY_QUARK, A = dp_y^2 and B = dp_z^2 for
 * GL_KIND_JET (a jet along x).  Per row with active particles, out [cap][14]
 * receives (tau_{k+1+1/2} [fm], tau_{k+1} [fm], <A>, err, <B>, err, <B>/<A>,
 * err, d<A>/dtau, err, d<B>/dtau, err, d<A + B>/dtau, err): the broadenings
 * in GeV^2 pooled over all events (sum over events of the sums over their
 * count), the anisotropy ratio, the rates kappa_T, kappa_L (heavy quarks) or
 * qhat_y, qhat_z (jets) in GeV^2/fm as the central difference of gl_kappa /
 * gl_qhat, and the total rate (the paper's total kappa or qhat); each
 * with its delete-one jackknife error sqrt((n-1)/n sum_i (f_(i) - mean f_(.))^2)
 * over the events.  out may be null to query n_rows.  dtau_fm and a_fm: the
 * step and lattice spacing in fm.  GL_EINVAL for bad arguments or events
 * whose active rows differ.  Host-only. */
gl_status gl_scan_statistics(const double *series, int32_t n_events, int32_t rows, int32_t kind, double dtau_fm,
                             double a_fm, double *out, int32_t cap, int32_t *n_rows);

/* Diagnostics of the current state (FP64 reductions on the device): the
 * Gauss-law residual, unitarity, the energy terms, and the two Casimirs of
 * the particle charges, which Eq. (2) conserves (Sec. 1 "Probes in Glasma":
 * q2 = Q^aQ^a = 4 and q3 = d_abc Q^aQ^bQ^c = 10/3 for <Q^aQ^b> = delta^ab/2,
 * <Q^aQ^bQ^c> = d^abc/4).  GL_ENUMERIC, with *out filled, when a field value
 * is not finite. */
gl_status gl_diagnostics(gl_event *ev, gl_diag *out);

/* Failure detection inside gl_run.  With period K >= 1 every K-th step (and
 * the last step of the call) checks the whole field state for non-finite
 * values on the device, and the series rows the call wrote are checked at
 * its end; gl_run then synchronises the stream and returns GL_ENUMERIC,
 * naming the first step at which a non-finite value was seen, if any was.
 * The run itself is not cut short (the device does not stop), so the state
 * at return is that of the full call.  0 (default) switches the checks off. */
gl_status gl_set_check_period(gl_event *ev, int32_t every);

/* Graph replay inside gl_run.  With G >= 1 gl_run records each whole block of
 * G coupled steps from the event's stream into a HIP graph and launches that
 * graph.  Blocks alternate between two executable graphs: the one due waits
 * on the host for its previous launch (two blocks back) to finish, then is
 * updated in place when the launches match or instantiated anew when they do
 * not (a block whose sort or series flush falls elsewhere).  Steps left over (fewer than
 * G) are launched directly, and so is every step while kernel timing
 * (gl_profile_enable) or the finite checks are on.  The launches and their
 * results are those of direct stepping, bit for bit.  Needs an event created
 * on a stream other than the null stream (GL_EINVAL otherwise).  0 (default)
 * launches every step directly and frees the graphs (after the stream is done
 * with them).  A recording or launch
 * error returns GL_EDEVICE and leaves the event uninitialised. */
gl_status gl_set_graph_steps(gl_event *ev, int32_t steps);
/* Graphs launched by gl_run since the event was created, and how many of them
 * had to be instantiated (the rest updated one of the two in place). */
gl_status gl_graph_stats(const gl_event *ev, int64_t *launches, int64_t *instantiations);

/* Iteration cap and residual tolerance of the matching Newton solve of the
 * initial condition (defaults 100 and 1e-13; max_iter >= 1, tol > 0).  A link
 * whose residual is not below tol after max_iter iterations makes
 * gl_init_glasma return GL_ENOTCONV. */
gl_status gl_set_match_params(gl_event *ev, int32_t max_iter, double tol);

/* Checkpoint and restore (bitwise resume).  gl_checkpoint writes, to a file
 * of the host, everything a later call needs to continue the event exactly
 * as if it had not stopped: the field state (and, when a particle step is
 * due, the site fields and the state at tau_n that the push reads), the particles in their device order with their ids,
 * the species table, the broadening series and formation sums, the sort
 * phase, and the static-quark and lightlike-jet accumulators with their
 * series when running.  Not saved: the Wilson lines of the initial
 * condition (gl_get_wilson_line, gl_dipole need a new gl_init_glasma) and
 * the kernel-timing state.  gl_restore reads such a file into an event
 * created with an identical gl_lattice_desc (GL_EINVAL otherwise, for a
 * file that is not a checkpoint of this format or is truncated, and for one
 * whose step counters, cadences or species counts are out of range or do not
 * fill the used particle slots; after such a refusal the event is left
 * uninitialised); the event's previous contents are replaced.  Both synchronise the stream.  GL_ESTATE for an
 * uninitialised event (checkpoint) or an event held by a batch (restore). */
gl_status gl_checkpoint(gl_event *ev, const char *path);
gl_status gl_restore(gl_event *ev, const char *path);

/* Host <-> device state transfer in the layouts above (tests, checkpoints).
 * The device keeps the first two rows of each link and rebuilds the third as
 * the complex conjugate of their cross product (exact for SU(3)):
 * gl_set_state expects SU(3) links and stores rows 0 and 1 of each;
 * gl_get_state returns all 18 values with the third row so rebuilt. */
gl_status gl_set_state(gl_event *ev, const double *U, const double *E, const double *phi,
                       const double *pi, int64_t n);
gl_status gl_get_state(gl_event *ev, double *U, double *E, double *phi, double *pi,
                       int64_t *n);
/* Site fields F^n of the last field step (valid while a particle step is due
 * or right after it). */
gl_status gl_get_site_fields(gl_event *ev, double *F);
/* Replace all particles; species table given as desc + per-particle species
 * (any order; the getters return this order).  nform per species is derived
 * from tau_form. */
gl_status gl_set_particles(gl_event *ev, int32_t n_species, const gl_species_desc *sp,
                           int64_t n, const int32_t *cell, const double *off,
                           const double *eta, const double *p, const double *Q,
                           const double *p0, const int32_t *species);
gl_status gl_get_particles(gl_event *ev, int64_t cap, int64_t *n, int32_t *cell, double *off,
                           double *eta, double *p, double *Q, double *p0, int32_t *species);
/* Particles are kept ordered by cell in device memory so that the push
 * gathers neighbouring site fields; they are re-sorted (stable, so the result
 * is deterministic) after every `every` particle steps and whenever particles
 * are added.  0 disables the periodic re-sort.  Default 16.  The host getters
 * always return particles in creation order. */
gl_status gl_set_sort_period(gl_event *ev, int32_t every);

/* Per-species formation step index and mass in lattice units. */
gl_status gl_species_info(gl_event *ev, int32_t species, int32_t *nform, double *mass_lat);

/* Wilson line V of one nucleus after gl_init_glasma: [18][N*N], FP64. */
gl_status gl_get_wilson_line(gl_event *ev, int32_t nucleus, double *V);
/* Saturation scale of the MV Wilson lines (reading of "Q_s = 2 GeV", which
 * the paper states without a conversion to g^2 mu): the dipole correlator
 * D(r) = (1/3) <Re Tr V(x) V^dag(x+r)>, averaged over the sites and the two
 * lattice directions, and Q_s defined by D(sqrt(2)/Q_s) = exp(-1/2).
 * gl_dipole writes D[0..rmax] (1 <= rmax <= N/2) of the stored Wilson line
 * of one nucleus (after gl_init_glasma).  gl_saturation_scale averages Q_s
 * over both nuclei, r interpolated linearly between lattice separations;
 * GL_ENUMERIC if D stays above exp(-1/2) up to N/2.  gl_calibrate_g2mu
 * searches g^2 mu (starting from mv->g2mu_GeV, or Q_s/0.6 if it is 0) so
 * that Q_s averaged over n_seeds MV draws (seeds seed .. seed+n_seeds-1)
 * equals qs_target_GeV within 0.1 %, with mv's sheets and regulators; it
 * overwrites the stored Wilson lines and leaves the field state alone. */
gl_status gl_dipole(gl_event *ev, int32_t nucleus, int32_t rmax, double *D);
gl_status gl_saturation_scale(gl_event *ev, double *qs_GeV);
gl_status gl_calibrate_g2mu(gl_event *ev, const gl_mv_desc *mv, double qs_target_GeV, uint64_t seed,
                            int32_t n_seeds, double *g2mu_out, double *qs_out);

/* MV charges of one (nucleus, sheet) drawn exactly as gl_init_glasma draws
 * them: [8][N*N] FP64, lattice units, for standard deviation sigma. */
gl_status gl_draw_charges(gl_event *ev, uint64_t seed, int32_t nucleus, int32_t sheet,
                          double sigma, double *rho);

/* Static quarks (Sec. 2, Eq. (4)): a quark of infinite mass keeps its site
 * and its colour charge, so its momentum change is the time integral of the
 * colour-electric field; with <Q^a Q^b> = delta^ab / 2 the broadening is
 * (1/2) sum_a (I_i^a)^2, I_i^a(x) = sum_n dtau E_i^a(x, tau_n), averaged over
 * the sites (a quark at every site).  E_i are the local-frame site fields
 * the particles read.  gl_static_start clears the FP64 accumulators and
 * accumulates from the first step at or after tau_start_fm (not before the
 * current step); the event must be created with static_correlator != 0.
 * Every later field step of the event (gl_evolve_fields, gl_run; not the
 * batched stepping) adds its step.
 * gl_static_broadening returns rows (tau_{n+1/2} [fm], <dp_x^2>, <dp_y^2>,
 * <dp_z^2> [GeV^2], sites) for the accumulated steps; out [cap][5] may be
 * null to query n_rows.  Errors: GL_ESTATE without the accumulators or before
 * initialisation, GL_EINVAL for a short output. */
gl_status gl_static_start(gl_event *ev, double tau_start_fm);
gl_status gl_static_broadening(gl_event *ev, double *out, int32_t cap, int32_t *n_rows);

/* Lightlike jets (Sec. 2, Eq. (5)): a jet with p_x -> infinity started at
 * the centre of every site x0 moves along +x at the speed of light (at step
 * n0 + k it sits in the cell x0 + floor(k dtau + 1/2), the NGP rule of the
 * particle push) and feels the colour force F_x = E_x, F_y = E_y - B_z,
 * F_z = E_z + B_y of the local-frame site fields, parallel transported to
 * its start with the product W of the x links it crossed (each at its
 * crossing step): I_i^a(x0) = sum_n dtau [W F_i W^dag]^a, FP64, and the
 * broadening is (1/2) sum_a (I_i^a)^2 averaged over the start sites.
 * gl_lightlike_start resets W to the identity and I to zero and starts at
 * the first step at or after tau_start_fm (not before the current step);
 * the event must be created with lightlike_correlator != 0.  Later field
 * steps of the event add theirs.  gl_lightlike_broadening returns rows
 * (tau_{n+1/2} [fm], <dp_x^2>, <dp_y^2>, <dp_z^2> [GeV^2], sites) like
 * gl_static_broadening; the same errors. */
gl_status gl_lightlike_start(gl_event *ev, double tau_start_fm);
gl_status gl_lightlike_broadening(gl_event *ev, double *out, int32_t cap, int32_t *n_rows);

/* Kernel timing with HIP events: period 0 switches it off, period p >= 1
 * times every p-th launch of each kernel class (a sample, so that the event
 * records barely perturb the run).  The single-kernel classes (0, 2, 4) take
 * the events with the launch itself (hipExtLaunchKernelGGL), at the kernel's
 * start and end, which times the kernel alone; classes 1 and 3 record them
 * on the event's stream around the launch, which also counts the dispatch
 * gap before it.  gl_profile_read synchronises
 * the stream and returns, per kernel class (0 field step, which also writes
 * the site fields when the event has particles or correlators, 1 static
 * quark and lightlike jet accumulation, 2 particle push, 3 series
 * reduction: one launch reduces the partial rows of up to 16 pushes, 4 the
 * particle push that also moves the particles to a newly sorted order, once
 * per sort period within gl_run), the summed milliseconds and the launch
 * counts since the last read, then clears them; ms and launches hold
 * GL_PROF_KERNELS entries.  Creates HIP events only (no device memory). */
#define GL_PROF_KERNELS 5
gl_status gl_profile_enable(gl_event *ev, int32_t period);
gl_status gl_profile_read(gl_event *ev, double *ms, int64_t *launches);

/* Lattice spacing in fm and GeV^-1, and the current step index. */
gl_status gl_event_info(gl_event *ev, double *a_fm, double *dtau_lat, int64_t *n);
/* Block until the event's stream is idle. */
gl_status gl_sync(gl_event *ev);

/* ---- batches of events (many uneven events in one launch per phase) ------
 * A batch steps events of equal precision, dtau and step index in lock-step
 * with flattened multi-event kernels: one launch per phase walks a table of
 * (event, tile) or (event, particle block) work items.  The step loop is
 * captured once into a hipGraph (graph_steps steps, default 32 = two particle
 * sort periods, so that the ping-pong parities return) and replayed; steps
 * that do not fill a graph run as ordinary launches.  The batch snapshots the
 * events, so while it exists it holds them: the calls that step, initialise
 * or change an event (gl_init_glasma*, gl_add_species, gl_set_particles,
 * gl_set_state, gl_restore, gl_evolve_fields, gl_push_particles, gl_run,
 * gl_set_sort_period, gl_static_start, gl_lightlike_start) return GL_ESTATE
 * for a held event, and an event can be held by one batch at a time.  The
 * getters work (gl_batch_run keeps the step index, buffers and series of its
 * events up to date); gl_batch_destroy releases the events, which can then
 * be used again.  Destroy the batch before its events.  The caller owns the
 * batch workspace (gl_batch_required_bytes, 256-byte aligned). */
typedef struct gl_batch gl_batch;
gl_status gl_batch_required_bytes(gl_event *const *evs, int32_t n_events, size_t *bytes);
gl_status gl_batch_create(gl_event *const *evs, int32_t n_events, void *workspace, size_t bytes,
                          void *stream, gl_batch **out);
void gl_batch_destroy(gl_batch *b);
/* Pick the field-kernel tile shape in sites (0: 32x4, 1: 64x2, 2: 16x8) and the
 * persistent grid (0: one workgroup per tile, k: k workgroups per compute
 * unit) by timing the field phases on this batch (they are idempotent, so
 * the state does not change), or read the choice from cache_json when it
 * holds this batch's key (device, precision, lattice sizes, particle count);
 * the choice is written back to cache_json.  cache_json may be NULL. */
gl_status gl_batch_autotune(gl_batch *b, const char *cache_json);
/* Set the configuration by hand (grid_mult as above, at most 64; sort_every
 * 0: never sort; graph_steps 0: no graph; graph_steps must be even and a
 * multiple of 2*sort_every).  GL_EINVAL otherwise.  A cached choice that
 * gl_batch_autotune finds out of its own range (shape, grid_mult above 8) is
 * ignored and the batch timed again. */
gl_status gl_batch_config(gl_batch *b, int32_t shape, int32_t grid_mult, int32_t sort_every,
                          int32_t graph_steps);
gl_status gl_batch_info(gl_batch *b, int32_t *shape, int32_t *tile_x, int32_t *tile_y,
                        int32_t *grid_mult, int32_t *graph_steps);
/* n_steps coupled steps of every event of the batch.  Failure handling: an
 * event whose broadening series turns non-finite at a step (a NaN or Inf
 * momentum, or fields gone non-finite where its particles are) is masked
 * from that step on: its field and particle work is skipped and its state
 * and series after that step are not meaningful, while the other events
 * run on unaffected.  At the end of the call every event's field state is
 * checked as well, and the call synchronises the batch stream and returns
 * GL_ENUMERIC if any event failed (gl_batch_status names them). */
gl_status gl_batch_run(gl_batch *b, int32_t n_steps);
/* Per event of the batch (in creation order), the first step at which it
 * failed, or -1. */
gl_status gl_batch_status(gl_batch *b, int32_t *fail_step);

/* ---- learned surrogate ------------------------------------------------------
 * Fully connected network n_in -> width (x depth hidden layers, SiLU) -> n_out
 * with BF16 weights and activations, FP32 accumulation on the matrix cores
 * (MFMA), FP32 master weights and Adam.  Inputs are scaled to [-1, 1] with
 * (in_lo, in_hi), outputs standardised with (out_mean, out_std), both inside
 * the kernels.  Parameters are one flat FP32 vector: W_1 [out][in], ...,
 * W_L, then b_1, ..., b_L.  X, Y are device FP32 arrays [n][n_in], [n][n_out].
 * The caller owns the workspace (gl_mlp_required_bytes; max_samples bounds n
 * of gl_mlp_train). */
typedef struct gl_mlp gl_mlp;
typedef struct {
    int32_t n_in, width, depth, n_out;
    int32_t max_batch;
} gl_mlp_desc;
gl_status gl_mlp_required_bytes(const gl_mlp_desc *d, int64_t max_samples, size_t *bytes);
gl_status gl_mlp_create(const gl_mlp_desc *d, int64_t max_samples, void *workspace, size_t bytes,
                        void *stream, uint64_t seed, gl_mlp **out);
void gl_mlp_destroy(gl_mlp *m);
gl_status gl_mlp_set_scaling(gl_mlp *m, const float *in_lo, const float *in_hi,
                             const float *out_mean, const float *out_std);
/* Optional per-output power of one input: the network then models
 * Y_c / X_col^powers[c] (standardised), and inference multiplies it back
 * (col < 0: off).  Used to factor out the Q_s scaling of the observables. */
gl_status gl_mlp_set_output_power(gl_mlp *m, int32_t col, const float *powers);
/* Minibatch Adam (beta 0.9, 0.999) for `epochs` passes over n samples in
 * shuffled whole batches; loss_per_epoch (host, may be NULL) receives the
 * mean standardised MSE of each epoch. */
gl_status gl_mlp_train(gl_mlp *m, const float *X, const float *Y, int64_t n, int32_t epochs,
                       int32_t batch, float lr, uint64_t seed, float *loss_per_epoch);
gl_status gl_mlp_infer(gl_mlp *m, const float *X, float *Y, int64_t n);
/* Inference that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same outputs as gl_mlp_infer, bit for bit, with its
 * staging and activation buffers in a fixed 4 MiB device array of the library
 * instead of the model's workspace.  X [n][n_in], Y [n][n_out] are device
 * FP32 arrays of the caller; rows go through in passes of as many as fit
 * (about 4000 at width 256).  The device of the model's stream must be the
 * current device; the array's address on that device is looked up on the
 * first call there.  Every call on one device uses that device's one array,
 * so calls that overlap on a device (concurrent streams or threads) race.
 * GL_EINVAL for a network too wide for 64 rows to fit (width above about
 * 16 000) or a stream of another device; launches only, no allocation. */
gl_status gl_mlp_infer_noalloc(gl_mlp *m, const float *X, float *Y, int64_t n);
/* One forward/backward pass on n <= max_batch samples (no update): gradients
 * of the standardised MSE to host grads [n_params], loss to *loss. */
gl_status gl_mlp_grads(gl_mlp *m, const float *X, const float *Y, int32_t n, float *grads,
                       float *loss);
/* The surrogate's answer or the solver (the surrogate falls back to the
 * solver, which also judges its error).  gl_mlp_set_trust stores a trust
 * region: the box [lo, hi] of the inputs the network was trained on (host
 * arrays of n_in), the allowed values of one discrete input column
 * (class_col, n_classes values, matched within class_tol), bins of one
 * continuous column (bin_col, n_bins + 1 increasing edges, the last bin
 * closed), and err [n_classes][n_bins], the network's error measured on
 * held-out solver runs of each cell; cells whose err exceeds err_max are not
 * trusted.  gl_surrogate_query takes n query rows X [n][n_in] (host FP32)
 * and sets *verdict to GL_SURROGATE_NETWORK when every row lies in the box,
 * in a known class and bin, in a trusted cell: then Y [n][n_out] (host)
 * receives the network's outputs (computed on the device through the
 * model's workspace, like gl_mlp_infer).  Otherwise *verdict is
 * GL_SURROGATE_OUTSIDE_DOMAIN or GL_SURROGATE_UNTRUSTED, Y is not written,
 * and the caller runs the solver.  GL_ESTATE without a trust table.
 * Synchronises the model's stream. */
#define GL_SURROGATE_NETWORK 0
#define GL_SURROGATE_OUTSIDE_DOMAIN 1
#define GL_SURROGATE_UNTRUSTED 2
gl_status gl_mlp_set_trust(gl_mlp *m, const float *lo, const float *hi, int32_t class_col, int32_t n_classes,
                           const float *classes, float class_tol, int32_t bin_col, int32_t n_bins,
                           const float *bin_edges, const float *err, float err_max);
gl_status gl_surrogate_query(gl_mlp *m, const float *X, int64_t n, float *Y, int32_t *verdict);
/* Read (get) and/or write (set) the FP32 parameters (host arrays). */
gl_status gl_mlp_params(gl_mlp *m, float *get, const float *set, int64_t *n_params);
const char *gl_mlp_last_error(void);

/* ---- measurement ---------------------------------------------------------------
 * The bandwidth a kernel of this library reaches on the device, as the
 * ceiling next to the 8 TB/s peak for the roofline fractions: reps timed
 * launches (after one untimed) of a streaming kernel over caller device
 * buffers in 16-byte accesses, kind 0 copy src -> dst, 1 read src (the
 * workgroups write one 16-byte word each to dst), 2 write dst (a fill); blocks
 * workgroups of 256 lanes.  variant (0 .. GL_STREAM_VARIANTS-1): 0 one vector
 * per lane and pass, interleaved workgroups; 1 four vectors per lane; 2 the
 * same non-temporal; 3 four vectors, each workgroup one contiguous share; 4
 * the same non-temporal; 5 eight vectors, non-temporal.  bytes: the size
 * streamed (a multiple of 16, 16-byte aligned buffers); dst_bytes: the size
 * of dst (at least bytes, or 16 * blocks for a read).  *ms_avg receives the
 * mean milliseconds per launch (HIP events on stream).  Errors: GL_EINVAL,
 * GL_EDEVICE (message from gl_stream_last_error). */
#define GL_STREAM_VARIANTS 6
gl_status gl_stream_probe(int32_t kind, int32_t variant, int32_t blocks, const void *src, void *dst, size_t bytes,
                          size_t dst_bytes, int32_t reps, void *stream, double *ms_avg);
const char *gl_stream_last_error(void);

const char *gl_status_string(gl_status s);
const char *gl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GLASMA_H */
