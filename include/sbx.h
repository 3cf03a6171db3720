/*
 * sbx.h -- C ABI of the MI355X nested-grid particle-mesh field solve.
 *
 * Method: Bien, Brandt & Just (2012), "Simulating sinking satellites with
 * Superbox-10", Sec. 2: nearest-grid-point mass assignment (Eq. 7), the
 * isolated-boundary potential by a zero-padded 3D FFT convolution with the
 * Green's function of Eq. 2 (Eqs. 1-5), force differencing with the Taylor
 * terms of Eq. 8, the five grids per galaxy with their grid-selection rule
 * (Sec. 2.1, Fig. 2), flattened grids (Sec. 2.2.2, Eq. 9), individual masses
 * (Sec. 2.2.1) and the leapfrog of Eq. 6.
 *
 * Conventions shared by every entry point
 *   - Return value: SBX_OK (0) or a negative sbx_status.  No exception or
 *     abort crosses the ABI.  sbx_last_error() gives a message for the last
 *     failing call on the calling thread.
 *   - Host pointers are borrowed for the duration of the call only.  Device
 *     pointers passed to sbx_poisson_solve are borrowed for that call and must
 *     stay valid until the work on the plan's stream has finished.
 *   - The context owns every device buffer it allocates; sbx_destroy frees
 *     them.  A context is not thread-safe: calls on one context must not
 *     overlap.
 *   - Grids are stored x-fastest: element (ix, iy, iz) of an N^3 grid is at
 *     (iz * N + iy) * N + ix.
 *   - Particle arrays on the host are n x 3 row-major (x, y, z per particle).
 *   - Units: G is a parameter; lengths and masses are the caller's.  The
 *     potential the API reports is the physical one, phi = -Phi, where
 *     Phi = +G sum M H is the positive field of Eq. 1; accelerations are
 *     +grad Phi as in Eq. 8.
 *   - Readings of points the paper leaves open: cell length l = 2R/(N-4)
 *     (usable cells [2, N-3] per axis, Table 3); z cell length q*l; cell of
 *     Eq. 7 = floor(((x - c) * gamma + N/2) + 0.5) in float64 with each
 *     operation rounded; membership by the spheroidal radius
 *     (dx^2 + dy^2) + (dz/q)^2 < R^2; H(0,0,0) = H(1,0,0) unless h0_mode
 *     is 1 (cell mean of 1/r) or 2 (zero); velocities are staggered,
 *     v = v(t - dt/2).
 */
#ifndef SBX_H
#define SBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBX_OK = 0,
  SBX_EINVAL = -1,   /* bad argument (NULL, size, NaN, negative mass, ...)   */
  SBX_ENOMEM = -2,   /* device or host allocation failed                     */
  SBX_EDEVICE = -3,  /* HIP runtime error (no device, launch failure, ...)   */
  SBX_EQCRIT = -4,   /* flattening below q_crit of Eq. 9                     */
  SBX_ESTATE = -5,   /* call out of order (e.g. step before build_grids)     */
  SBX_EPARITY = -6   /* a self-check of the method failed: the FP64 transform
                        of the mirrored Green's function (Eq. 5) is not real
                        to rounding (max|Im| / max|Re| above 1e-10)          */
} sbx_status;

typedef enum { SBX_FP32 = 0, SBX_FP64 = 1 } sbx_prec;
typedef enum { SBX_CENTRE_FIXED = 0, SBX_CENTRE_COM = 1, SBX_CENTRE_DENSITY = 2 } sbx_centring;

/* Particle classes relative to one galaxy's grids (Sec. 2.1 list of grids). */
typedef enum { SBX_CORE = 0, SBX_RING = 1, SBX_OUTER = 2, SBX_LOST = 3 } sbx_class;

/* One grid geometry: n cells per axis (power of two, 8..256), half-extent R
 * of the usable region, flattening q in (0, 1] of the z cell length. */
typedef struct {
  int32_t n;
  double R;
  double q;
} sbx_level;

/* Grids of one galaxy (Sec. 2.1, Fig. 2).
 * n_levels = 3: lv[0] inner (grid 1), lv[1] middle (grids 2 and 3), lv[2]
 *   outer = the fixed global grid (grids 4 and 5), centred at outer_centre.
 *   The inner and middle levels follow the galaxy centre: `centre` when
 *   centring = SBX_CENTRE_FIXED, the centre of mass of the galaxy's live
 *   particles (recomputed every step) when SBX_CENTRE_COM, the galaxy's
 *   density maximum when SBX_CENTRE_DENSITY (recomputed at every solve,
 *   starting from the centre of the previous solve, `centre` for the first
 *   one): the galaxy's live particle masses are binned on the N^3 cells
 *   (Eq. 7) of the inner grid placed at that centre as exact integers
 *   floor(m 2^s), s = 62 - e - b with m_max < 2^e over all particles and b
 *   the bit length of the particle count; the densest cell (ties: lowest
 *   (z, y, x) index) and the FP64 mass centre of the galaxy's live particles
 *   in its 3x3x3 block of cells give the new centre (the previous one is
 *   kept when no particle is on the grid).  Costs an N^3 array of 64-bit
 *   integers per galaxy.
 * n_levels = 1: one isolated grid lv[0], fixed at `centre`, holding every
 *   particle (centring must be SBX_CENTRE_FIXED). */
typedef struct {
  int32_t n_levels;
  sbx_level lv[3];
  int32_t centring;
  double centre[3];
  double outer_centre[3];
} sbx_hierarchy;

typedef struct {
  int32_t prec;     /* sbx_prec: arithmetic of grids, FFT, forces, particles */
  double G;         /* gravitational constant                                 */
  int32_t h0_mode;  /* H(0,0,0), singular in Eq. 2: 0 = H(1,0,0) = 1/l
                       (default), 1 = mean of 1/r over the cell (closed form
                       of a uniform prism; 2.3800774/l in a cubic cell),
                       2 = 0                                                  */
  int32_t taylor;   /* 1 = full Eq. 8, 0 = central differences only           */
  int32_t device;   /* HIP device ordinal                                     */
  void* stream;     /* hipStream_t to run on, or NULL for a private stream    */
} sbx_config;

/* FP64 diagnostics (per particle component id 0..7). */
typedef struct {
  double ekin[8];     /* sum 1/2 m |v_sync|^2, v_sync = v + dt/2 a(t)       */
  double epot[8];     /* 1/2 sum m phi(x), phi = -Phi at the particle       */
  double L[8][3];     /* sum m x cross v_sync about the origin              */
  double disc_sigR;   /* component 0 of galaxy 0: sigma_R about galaxy 0's  */
  double disc_sigz;   /*   centre, and sigma_z                              */
  int64_t n_lost;     /* particles flagged lost                             */
  int64_t n_live[8];  /* live particles per component                       */
} sbx_diag;

typedef struct sbx_ctx sbx_ctx;
typedef struct sbx_poisson sbx_poisson;
typedef struct sbx_batch sbx_batch;

/* Message of the last failing call on this thread ("" if none). */
const char* sbx_last_error(void);

/* Host-only check of a set of hierarchies (nesting, q in (0,1], Eq. 9
 * q >= q_crit = max(R1/R2, 4/(N-4) * R3/R2) for the middle level, q < 1 only
 * for galaxy 0, several galaxies share one global outer level).  Needs no GPU.
 * Returns SBX_EQCRIT below q_crit, SBX_EINVAL otherwise when invalid. */
sbx_status sbx_validate_hierarchies(int32_t n_galaxies, const sbx_hierarchy* h);

/* q_crit of Eq. 9 (host-only). */
double sbx_q_crit(int32_t n, double R_core, double R_out, double R_sys);

/* ---- context: particles, grids, forces, steps ---------------------------- */

/* Create a context on cfg->device.  *out receives the handle. */
sbx_status sbx_create(const sbx_config* cfg, sbx_ctx** out);
void sbx_destroy(sbx_ctx* ctx);

/* Copy n particles from the host (x, v: n*3; m: n; comp, gal: n; comp in
 * 0..7, gal < n_galaxies of build_grids).  Converted to the context precision
 * on the device.  Masses must be finite and >= 0.  Lost flags are cleared. */
sbx_status sbx_load_particles(sbx_ctx* ctx, int64_t n, const double* x, const double* v,
                              const double* m, const int8_t* comp, const int8_t* gal);

/* As sbx_load_particles, from device memory of the context's device (same
 * layouts; e.g. the storage of torch tensors).  The arrays are read on the
 * context stream: work that produced them must be ordered before the call
 * (same stream, or synchronised).  They are validated on the device (first
 * bad particle reported, SBX_EINVAL); pointers that are not device memory of
 * the context's device are rejected with SBX_EINVAL.  Borrowed for the call
 * only. */
sbx_status sbx_load_particles_device(sbx_ctx* ctx, int64_t n, const double* x, const double* v,
                                     const double* m, const int8_t* comp, const int8_t* gal);

/* Borrow the particle storage of the caller (e.g. torch tensors) instead
 * of copying it in.  All arrays are device memory of the context's device;
 * x, v, m are in the context precision (float for SBX_FP32, double for
 * SBX_FP64) and laid out as structures of arrays: x[k * n + i] is coordinate
 * k of particle i (a 3 x n row-major array), v likewise (v(t - dt/2)), m[n];
 * comp, gal: n int8 as in sbx_load_particles; lost: n uint8 (0 = live), read
 * and written by the library.  Steps move x and v and set lost in place on
 * the context stream; getters copy from them.  The storage is borrowed until
 * sbx_destroy or the next sbx_load_particles*, sbx_bind_device_particles or
 * sbx_load: the caller keeps it alive and orders its own work on it with the
 * context stream.  Bound particles are never reordered (the cell sort, a
 * performance setting only, is skipped), and a context holding them cannot
 * join a batch.  Validated on the device as sbx_load_particles_device
 * (SBX_EINVAL); x, v and lost must not overlap any other array (SBX_EINVAL).
 * Lost flags are taken as given. */
sbx_status sbx_bind_device_particles(sbx_ctx* ctx, int64_t n, void* x, void* v, void* m,
                                     int8_t* comp, int8_t* gal, uint8_t* lost);

/* Validate the hierarchies and build the Green's tables (Sec. 2.1: the
 * transformed H is computed once): H of Eq. 2 on lags 0..N, mirrored to
 * (2N)^3 by Eq. 5, transformed by an FP64 FFT, scaled by G/(2N)^3 and stored
 * on (N+1)^3 (it is real and even per axis).  Allocates the grids.
 * SBX_EQCRIT below q_crit, SBX_EPARITY if a transformed table is not real to
 * rounding (max|Im| / max|Re| > 1e-10), SBX_ENOMEM, SBX_EINVAL. */
sbx_status sbx_build_grids(sbx_ctx* ctx, int32_t n_galaxies, const sbx_hierarchy* h);
/* (1 <= n_galaxies <= 8; every galaxy's grids are solved and summed into the
 * forces of all particles, Sec. 2.1: the number of galaxies is not fixed.) */

/* One field solve at the current positions, no motion: loss test, centres,
 * mass assignment, the isolated solves, Eq. 8 with the grid-selection rule.
 * acc (n*3) and pot (n, physical phi) are host outputs; either may be NULL.
 * Lost particles get zeros. */
sbx_status sbx_compute_forces(sbx_ctx* ctx, double* acc, double* pot);

/* nsteps integration cycles of Eq. 6 with constant dt (stream-ordered, does
 * not synchronise).  When diag_every > 0 the FP64 diagnostics are taken at the
 * start of every diag_every-th step and appended to the context's log. */
sbx_status sbx_step(sbx_ctx* ctx, double dt, int32_t nsteps, int32_t diag_every);

/* Read back positions, velocities (v(t - dt/2)) and lost flags (any may be
 * NULL).  Synchronises the context stream. */
sbx_status sbx_get_particles(sbx_ctx* ctx, double* x, double* v, uint8_t* lost);

/* As sbx_get_particles, into device memory of the context's device (written
 * on the context stream; the call returns when the writes are done). */
sbx_status sbx_get_particles_device(sbx_ctx* ctx, double* x, double* v, uint8_t* lost);

/* Centres used by the last solve: n_galaxies * 3 doubles. */
sbx_status sbx_get_centres(sbx_ctx* ctx, double* centres);

/* Class of every particle relative to galaxy `galaxy` and its cell on level
 * `level` (idx: n*3 int32, cls: n int8; either may be NULL), at the current
 * positions and the centres of the last solve (or the fixed centres). */
sbx_status sbx_get_indices(sbx_ctx* ctx, int32_t galaxy, int32_t level, int32_t* idx,
                           int8_t* cls);

/* Grid `which` of galaxy `galaxy` after the last solve, as N^3 float64.
 * kind 0 = cell masses, 1 = field Phi (positive, Eq. 1).  Three levels:
 * which 0 = grid 1 (core, inner level), 1 = grid 3 (ring, middle level),
 * 2 = grids 2+3 (core and ring, middle level), 3 = grid 5 (outer, global
 * level), 4 = grids 4+5 (all, global level).  One level: which 0 only.
 * kind 1 is valid after sbx_compute_forces (sbx_step reuses the buffers). */
sbx_status sbx_get_grid(sbx_ctx* ctx, int32_t galaxy, int32_t which, int32_t kind, double* out);

/* FP64 diagnostics at the current state (a solve without motion). */
sbx_status sbx_diagnostics(sbx_ctx* ctx, double dt, sbx_diag* out);

/* Number of entries in the diagnostics log of sbx_step, and a copy of up to
 * max entries (oldest first).  Synchronises. */
sbx_status sbx_diag_log(sbx_ctx* ctx, int32_t max, sbx_diag* out, int32_t* count);

/* Differentiable segment: nsteps integration cycles from the current state
 * (no reordering inside), then the reverse mode of the discrete cycles, with
 * (x, v) checkpoints every ckpt_every steps and the positions between
 * checkpoints recomputed.  Loss L = sum over the live particles of component
 * sel_comp of galaxy sel_gal of 1/2 m v_z^2, with v the staggered velocity
 * after the last kick.  Outputs (host, caller's particle order, any may be
 * NULL): loss (1), grad_m = dL/dm (n), grad_x = dL/dx (n*3) and
 * grad_v = dL/dv (n*3) at the start of the segment.  Nearest-grid-point
 * cells are piecewise constant, so dL/dx holds the in-cell (Eq. 8 offset)
 * part only.  Each reverse cycle re-solves the fields from the particles that
 * took part in that cycle (live after its start-of-step loss test, Sec. 2.1):
 * a particle lost during the segment is not in the loss, but its dL/dm
 * collects the fields of the cycles before its loss.
 * Fixed centres only (SBX_EINVAL otherwise).  Leaves the context at the
 * final state, as sbx_step would.  FP64 adjoint state in both precisions. */
sbx_status sbx_adjoint_segment(sbx_ctx* ctx, double dt, int32_t nsteps, int32_t ckpt_every,
                               int32_t sel_comp, int32_t sel_gal, double* loss, double* grad_m,
                               double* grad_x, double* grad_v);

/* As sbx_adjoint_segment with grad_m, grad_x, grad_v in device memory of the
 * context's device (loss stays a host pointer). */
sbx_status sbx_adjoint_segment_device(sbx_ctx* ctx, double dt, int32_t nsteps, int32_t ckpt_every,
                                      int32_t sel_comp, int32_t sel_gal, double* loss,
                                      double* grad_m, double* grad_x, double* grad_v);

/* Disc diagnostics of the paper's analysis (Sec. 4.2, 5.2-5.4).
 * The disc is the live particles of component `comp` of galaxy `galaxy`;
 * positions are taken relative to that galaxy's centre at the last solve
 * (its given centre before any solve) and velocities (the stored staggered
 * v) relative to the disc's mass-weighted mean velocity.
 *   - Radial bins of equal particle numbers: particles ordered by cylindrical
 *     R (ties in the caller's particle order), bin k holding n / n_bins
 *     particles plus one for k < n % n_bins.  Per bin (unweighted means):
 *     mean R, mean circular velocity (mean v_phi), RMS z.
 *   - Heat: sum of 1/2 m |v - vbar_c(R) phi|^2 over the disc, vbar_c linearly
 *     interpolated between the bins' mean radii, constant beyond the ends.
 *   - In the annulus R_lo <= R < R_hi: sigma_R, sigma_phi, sigma_z about the
 *     annulus means, sigma_tot^2, and the vertical density profile: mass in
 *     n_z equal bins of z over [-z_max, z_max) over (annulus area x bin
 *     width).
 * Every sum is reduced in a fixed order except the profile bins.  Outputs on
 * the host: bin_r, bin_vc, bin_rms_z (n_bins each) and rho_z (n_z), any may
 * be NULL.  SBX_EINVAL for a bad query (1 <= n_bins <= 2048,
 * 1 <= n_z <= 1024, z_max > 0, 0 <= R_lo < R_hi), SBX_ESTATE without disc
 * particles. */
typedef struct {
  int32_t n_bins;
  double annulus[2];
  int32_t n_z;
  double z_max;
  int32_t comp, galaxy;
} sbx_disc_query;

typedef struct {
  double e_heat;
  double sig_R, sig_phi, sig_z, sig_tot2;
  double bulk_v[3];
  int64_t n_disc, n_annulus;
} sbx_disc_result;

sbx_status sbx_disc_analysis(sbx_ctx* ctx, const sbx_disc_query* q, sbx_disc_result* out,
                             double* bin_r, double* bin_vc, double* bin_rms_z, double* rho_z);

/* Fourier coefficients of the disc's surface density in annular bins
 * (Sec. 5.6): for bin k = [k dR, (k+1) dR), dR = r_max / n_rbins, and
 * m = 0..m_max, A_m = (1/S_k) sum over the bin's particles of M exp(-i m phi)
 * with phi the polar angle about the galaxy centre and S_k the bin area.
 * Same disc selection and centre as sbx_disc_analysis.  coeff (host):
 * n_rbins * (m_max + 1) * 2 doubles, (re, im) at (k * (m_max + 1) + m) * 2.
 * Sums in a fixed order.  SBX_EINVAL unless 1 <= n_rbins <= 65536,
 * r_max > 0, 0 <= m_max <= 16. */
sbx_status sbx_disc_modes(sbx_ctx* ctx, int32_t comp, int32_t galaxy, int32_t n_rbins, double r_max,
                          int32_t m_max, double* coeff);

/* Merge grid 5 of all galaxies into one solve (1) or solve it per galaxy (0,
 * the default); applied at the next sbx_build_grids.  Each class's sum of
 * Sec. 2.1 contains grid 5 (core: grids 1 + 3 + 5, ring: 2 + 3 + 5, outer:
 * 4 + 5), so by linearity of Eq. 1 the sum over galaxies of their grid-5
 * potentials is the potential of the summed grid-5 masses, read once per
 * particle: n_galaxies * 4 + 1 solves per step instead of n_galaxies * 5.
 * The build then fails with SBX_EINVAL unless there are at least two
 * galaxies, all with three levels.  In sbx_get_grid, which 3 of galaxy 0 is
 * the summed grid 5 (which 3 of the others stays zero) and which 4 is grid 4
 * alone.  sbx_adjoint_segment rejects a merged context (SBX_EINVAL). */
sbx_status sbx_set_outer_merge(sbx_ctx* ctx, int32_t merge);

/* Mass assignment form (Sec. 2.1; Eq. 7 cells).  on = 0 (the default):
 * cell masses are floating-point sums in the context's precision, added in
 * an order that varies between runs (atomics).  on = 1: fixed-point sums.
 * Every mass enters as the integer floor(m 2^s), s = 62 - e - b, where the
 * largest particle mass of the context is below 2^e and b is the bit length
 * of its particle count, so that every cell total fits in 62 bits; the
 * integers are summed exactly and each cell mass is (sum converted to
 * float64 with one rounding) * 2^-s, then rounded to the context's
 * precision.  Cell masses are then independent of the order of the adds
 * and equal the oracle's fixed-point assignment bit for bit.  Nothing else
 * in a step depends on the order of additions except the FP64 sums of the
 * centre of mass and of the density-maximum centre, which run in particle
 * order: runs are bitwise reproducible with fixed centres, or with the
 * reorder off (sbx_set_sort_interval 0; the reorder's slot reservation
 * leaves the particles of one cell in a varying order).  Each mass loses
 * less than 2^-s (for 8.5M equal masses of 6.6e-7 that is 3.5e-18, 5e-12
 * relative).  Costs one 8-byte accumulator per mass-grid
 * cell and a conversion pass per assignment.  Takes effect for the next
 * assignment; kept by sbx_save / sbx_load.  SBX_ESTATE while the context
 * belongs to a batch (the contexts of a batch must share the form,
 * SBX_EINVAL from sbx_batch_create otherwise). */
sbx_status sbx_set_deterministic_deposit(sbx_ctx* ctx, int32_t on);

/* Reorder the particles in device memory by the cell of their finest grid
 * every `every` steps (at the start of the step; 0 = never; default 4).  A
 * performance setting only: every output is returned in the caller's
 * particle order. */
sbx_status sbx_set_sort_interval(sbx_ctx* ctx, int32_t every);

/* Checkpoint files (Sec. 3.1 and 4.1: models are evolved in isolation, kept
 * and reused).  sbx_save writes the whole state of a context: precision, G,
 * h0_mode, taylor, the hierarchies, the outer-merge, mass assignment and
 * sort settings, the
 * step count and last dt, the centres of the last solve (the state density-
 * maximum centring continues from), and the particles in the caller's order
 * (x, staggered v, m, comp, gal, lost).  The diagnostics log is not saved.
 * Synchronises.  SBX_ESTATE without grids or particles, SBX_EINVAL when the
 * file cannot be written.
 * sbx_load restores such a file into a context created with the same
 * precision, G, h0_mode and taylor setting (SBX_EINVAL otherwise, and for
 * a file that is not a version 1 or 2 checkpoint, truncated or corrupt): it
 * rebuilds the grids and Green's tables, loads the particles (owned copies)
 * with their lost flags, and restores the step count, dt, centres and
 * settings.  Stepping on from a loaded state gives what stepping the saved
 * context would have given, up to summation orders (bit for bit with fixed
 * centres when the mass assignment is fixed-point or every cell total is
 * exact, e.g. dyadic masses; centre-of-mass sums run in particle order,
 * which a load resets to the caller's). */
sbx_status sbx_save(sbx_ctx* ctx, const char* path);
sbx_status sbx_load(sbx_ctx* ctx, const char* path);

/* Block until all work queued on the context stream has finished. */
sbx_status sbx_sync(sbx_ctx* ctx);

/* Particles held (live and lost) and galaxies built; either may be NULL. */
sbx_status sbx_get_counts(sbx_ctx* ctx, int64_t* n, int32_t* n_galaxies);

/* Number of live particles (synchronises). */
sbx_status sbx_count_live(sbx_ctx* ctx, int64_t* live);

/* ---- batches: independent instances stepped together ---------------------- */

/* Group n (1..32) contexts -- same device and precision, grids built,
 * particles loaded, all fresh or all stepped together -- so that every phase
 * of a step is one launch over all of them (the FFT passes: one launch per
 * distinct grid size) and a step is one replay of a captured HIP graph (two
 * graphs: with and without the cell sort).  Uneven sizes are fine: grids of
 * 8..256 cells, any particle counts.  The contexts stay owned by the caller;
 * while in the batch they are stepped only through it (sbx_step, forces,
 * loading and rebuilding return SBX_ESTATE) and their getters need
 * sbx_batch_sync after sbx_batch_step.  stream: hipStream_t or NULL.  The
 * sort interval is taken from the first context. */
sbx_status sbx_batch_create(sbx_ctx* const* ctxs, int32_t n, void* stream, sbx_batch** out);

/* nsteps integration cycles of every instance; dt: one value per context in
 * the order of creation (NULL keeps the previous values, initially each
 * context's last dt).  Stream-ordered, does not synchronise.  No diagnostics
 * records are taken in batch steps. */
sbx_status sbx_batch_step(sbx_batch* b, const double* dt, int32_t nsteps);

/* Wait for the batch's work and hand its state back to the contexts. */
sbx_status sbx_batch_sync(sbx_batch* b);

/* Sort interval of the batch (as sbx_set_sort_interval; default 4). */
sbx_status sbx_batch_set_sort_interval(sbx_batch* b, int32_t every);

/* Synchronise and release the contexts (they can be stepped alone again). */
void sbx_batch_destroy(sbx_batch* b);

/* ---- tracing: per-phase timing with HIP events ---------------------------- */

/* Phases: 0 step start (not a kernel), 1 zero grids, 2 loss test and centres,
 * 3 mass assignment, 4 fwd_x, 5 fwd_y, 6 z pass with the Green multiply,
 * 7 inv_y, 8 inv_x (the five FFT passes of all solves of a step), 9 force,
 * kick and drift, 10 particle reordering. */
#define SBX_N_PHASES 11

/* Start recording an event after every phase launched on the context stream
 * (at most max_marks events; later marks are dropped).  Synchronises. */
sbx_status sbx_profile_begin(sbx_ctx* ctx, int32_t max_marks);

/* Stop recording, synchronise, and return per phase the summed GPU time in
 * milliseconds (out_ms) and the number of launches (out_count); arrays of
 * n_phases >= SBX_N_PHASES entries. */
sbx_status sbx_profile_end(sbx_ctx* ctx, int32_t n_phases, double* out_ms, int64_t* out_count);

/* ---- standalone isolated Poisson solves (Eqs. 1-5) ------------------------ */

/* Plan for isolated solves on one geometry (n, R, q) in precision prec.
 * Builds the Green's table as sbx_build_grids does (h0_mode as in
 * sbx_config; SBX_EPARITY as in sbx_build_grids). */
sbx_status sbx_poisson_create(int32_t n, double R, double q, double G, int32_t h0_mode,
                              int32_t prec, int32_t device, void* stream, sbx_poisson** out);
void sbx_poisson_destroy(sbx_poisson* p);

/* Solve `batch` independent grids: rho and phi are device pointers to
 * batch * n^3 elements of the plan precision (x-fastest per grid, grids
 * back to back); phi = Phi of Eq. 1 for cell masses rho.  rho and phi may be
 * the same buffer.  batch <= 64.  Stream-ordered on the plan's stream. */
sbx_status sbx_poisson_solve(sbx_poisson* p, int32_t batch, const void* rho, void* phi);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * sbx_poisson_solve, but the work arrays, the solve descriptors and the work
 * counters live in a fixed work space of 96 MiB (100663296 bytes) that each
 * GPU the library runs on holds until the process ends; the call launches
 * kernels only (no hipMalloc, hipFree, memset, copy or synchronisation) and
 * returns without waiting.  The plan (made by sbx_poisson_create, which sets
 * the work space up on its device) supplies the Green's table and stream;
 * the caller passes rho and phi as for sbx_poisson_solve.  SBX_EINVAL when
 * the batch needs more than the work space: each grid takes 5 N^3 + 20 N^2
 * complex values of the plan precision (plus a few hundred bytes per call),
 * so one 128^3 solve fits in FP32 (82.5 MiB), four 64^3 solves in FP64 and
 * nine in FP32.  Every call on a GPU uses
 * that GPU's one work space: calls that overlap in time on one GPU (other
 * streams, other threads, other plans) race and must be ordered by the
 * caller.  The work counters are cleared at the start of each call by a
 * kernel, so stale contents of an earlier call do not matter. */
sbx_status sbx_poisson_solve_noalloc(sbx_poisson* p, int32_t batch, const void* rho, void* phi);

/* The stored transformed Green's function, (n+1)^3 float64, index
 * (kx * (n+1) + ky) * (n+1) + kz, scaled by G/(2n)^3; rel_imag receives
 * max|Im| / max|Re| of the FP64 transform before folding (may be NULL). */
sbx_status sbx_poisson_green(sbx_poisson* p, double* out, double* rel_imag);

/* Device bytes the plan holds. */
int64_t sbx_poisson_bytes(sbx_poisson* p);

/* Line schedule of the FFT passes of every solve (Eqs. 3-5): a line of
 * length L = 2n is transformed with 16 or 32 values per thread (radix 16,
 * then L/16, then 2 if L/16 > 16; or radix 32, then L/32).  In FP32, lines of
 * 128 points and more (n >= 64) have both, and the launch-shape tuner times
 * both the first time a precision, grid size and solve count is planned.
 * v = 16 or 32 pins that schedule for every plan made from now on, in every
 * context and standalone plan of the process (plans already made keep
 * theirs); v = 0 (the default) lets the tuner choose.  Lengths with one
 * schedule ignore the pin.  SBX_EINVAL for other values. */
sbx_status sbx_set_fft_schedule(int32_t v);

/* Form of the solves (Eqs. 3-5).  form = 5: five passes of line
 * transforms (x, y, z with the Green's multiply, inverse y, inverse x).
 * form = 3: where one z plane's half spectrum fits in the 160 KB of LDS of
 * a compute unit (32 <= n <= 128; at n = 128 half a plane per block), three
 * passes: the x and y transforms of one plane in one block, the z pass,
 * and the inverse y and x transforms of one plane in one block, so the
 * x-transformed planes never go to device memory (about 30% fewer bytes
 * per solve); each padded length-2n line transform is done as two
 * length-n transforms of its even and odd frequencies (at n = 128
 * the forward plane pass takes the even and the odd x frequencies of a
 * plane in two blocks, with 256 or 512 threads; the inverse takes the even
 * and the odd rows of a plane in two blocks with 256 or 512 threads, or in
 * FP32 also a whole plane with 1024).  form = 0 (the
 * default): the tuner times both the first time a precision, grid size and
 * solve count is planned and keeps the faster.  Like the schedule pin,
 * process-wide, for plans made from now on; sizes without the plane form
 * use five passes whatever the pin.  SBX_EINVAL for other values. */
sbx_status sbx_set_fft_form(int32_t form);

/* Block size of the plane-fused passes (form 3, Eqs. 3-5) for plans made
 * from now on: 256, 512 or 1024 threads, or 0 (the default: the tuner times
 * every block size a pass has and keeps the fastest).  At n = 128, 256
 * and 512 run the half-plane passes (two blocks per plane), and 1024 the
 * whole-plane inverse (FP32 only); the forward pass there has no 1024 and, like
 * every pass without the pinned size, is still tuned over its own.
 * Process-wide, like the other pins.  SBX_EINVAL for other values. */
sbx_status sbx_set_plane_threads(int32_t nt);

/* The launch shapes the tuner has chosen so far in this process, one line
 * per precision, grid size, solve count and pass ("fp32 N=128 x5 form=5
 * zpass nt=256 grid=1024 v=16"; grid=tiles: one block per tile; the plane
 * passes of form 3 are "plane_fwd nt=512" and "plane_inv nt=512"), and
 * where both forms were timed, one more line with the tuner's time of the
 * whole solve set in each ("... timed five-pass 0.247 ms, plane 0.233 ms").
 * Writes at most cap bytes including a terminating NUL into out (may be
 * NULL when cap is 0) and returns the length of the whole report. */
int64_t sbx_fft_tuning_report(char* out, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* SBX_H */
