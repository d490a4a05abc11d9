/*
 * relpic.h -- C ABI of the MI355X (gfx950) electromagnetic PIC step for
 * relativistic beams.
 *
 * Method: Xu et al., "On numerical errors to the fields surrounding a
 * relativistically moving particle in PIC codes".  One step is the PIC cycle
 * of Sec. 1: charge-conserving current deposit with the quadratic B-spline
 * shape, Maxwell field advance (Eq. 1) with the Yee operators (Eq. 14) or the
 * customized axial operator of Sec. 3 / App. C, field gather, and the
 * relativistic Boris push.
 *
 * Conventions
 *   Units: c = 1, d_t E = curl B - J, div E = rho (Eqs. 1, 5).
 *   Lattice (node = integer index): E1 (i1+1/2,i2,i3), E2 (i1,i2+1/2,i3),
 *     E3 (i1,i2,i3+1/2), B1 (i1,i2+1/2,i3+1/2), B2 (i1+1/2,i2,i3+1/2),
 *     B3 (i1+1/2,i2+1/2,i3); J like E; rho at nodes.  In 2D i3 is absent.
 *   Field arrays exchanged with the caller are dense, x1 fastest:
 *     index = i1 + n1 * (i2 + n2 * i3), with i1 counted from the first cell
 *     of the (possibly moving) window.
 *   Particle positions are (cell, offset): cell = nearest node (x1 global,
 *     i.e. counted from the window's starting position at t = 0), offset in
 *     [-1/2, 1/2) in cell units; momenta u = gamma * beta.
 *   Axial operators (App. C):
 *     d+ f_i = (1/dx1) sum_{l=1..M} C_l (f_{i+l} - f_{i-l+1})   (E -> B)
 *     d- f_i = (1/dx1) sum_{l=1..M} C_l (f_{i+l-1} - f_{i-l})   (B -> E)
 *     M = 1, C_1 = 1 is Yee.  x2 and x3 always use the Yee difference.
 *
 * Ownership: every pointer argument is caller-owned; the library copies what
 * it needs before returning.  Host pointers are host memory unless a name
 * says "device".  Handles are not thread-safe: one handle per host thread and
 * stream.  No C++ exception or abort crosses this boundary; every call
 * returns a relpic_status and relpic_last_error() describes the last failure
 * on the calling thread.
 */
#ifndef RELPIC_H
#define RELPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RELPIC_OK = 0,
  RELPIC_EINVAL = 1,    /* malformed argument or descriptor */
  RELPIC_EUNSTABLE = 2, /* time step violates the operators' Courant limit */
  RELPIC_ERANGE = 3,    /* particle or index outside the grid / capacity */
  RELPIC_ENOMEM = 4,    /* device or host allocation failed */
  RELPIC_EDEVICE = 5,   /* HIP runtime error, or a kernel raised the error word */
  RELPIC_ESTATE = 6     /* call not valid in the object's current state */
} relpic_status;

typedef enum { RELPIC_FP32 = 0, RELPIC_FP64 = 1 } relpic_precision;

typedef enum { RELPIC_BC_PERIODIC = 0, RELPIC_BC_WINDOW = 1 } relpic_bc;

typedef enum {
  RELPIC_E1 = 0, RELPIC_E2, RELPIC_E3,
  RELPIC_B1, RELPIC_B2, RELPIC_B3,
  RELPIC_J1, RELPIC_J2, RELPIC_J3
} relpic_field;

/* Grid.  ndim 2 or 3; n[d], dx[d] for d < ndim (others ignored); dt the time
 * step.  bc1 is the x1 boundary: periodic, or a window moving along +x1 at
 * window_speed (units of c) that advances one cell each time
 * floor(steps * window_speed * dt / dx1) grows; fields outside the window are
 * zero and particles whose cell leaves [2, n1 - 3] of the window are dropped.
 * x2 and x3 are periodic. */
typedef struct {
  int ndim;
  int64_t n[3];
  double dx[3];
  double dt;
  int bc1;
  double window_speed;
} relpic_grid;

/* Axial operators (App. C).  M coefficients C[0..M-1] (C_1..C_M) of the
 * operator on E (d+, Faraday's law: [k]_E1); M = 1 with C = NULL or C[0] = 1
 * is Yee.  MB coefficients CB[0..MB-1] of the operator on B (d-, Ampere's
 * law: [k]_B1; it is also the divergence of Gauss's law and of the
 * continuity equation); MB = 0 (a zero-initialized struct) uses C for both,
 * Sec. 3's choice [k]_E1 = [k]_B1.  Sec. 3 also allows [k]_E1 != [k]_B1 with
 * [k]_E1 [k]_B1 = [k1]_t^2: e.g. MB = 1, CB = {1} (Yee on B) with C from
 * relpic_fit_operator(..., RELPIC_FIT_E_WITH_YEE_B, ...).  Whenever the
 * operator on B is wider than two points the library also applies the
 * current correction J1 <- G * J1 (G the inverse of the telescoped d-
 * stencil) so that the discrete Gauss law holds with that divergence; with
 * Yee on B none is needed.  The shorter operator is zero-padded to the
 * longer one's width. */
typedef struct {
  int M;
  const double *C;
  int MB;
  const double *CB;
} relpic_solver;

/* Targets of the App. C fit. */
enum {
  RELPIC_FIT_TIME = 0,         /* [k]_1 = [k1]_t (the same operator on E and B) */
  RELPIC_FIT_E_WITH_YEE_B = 1  /* [k]_E1 = [k1]_t^2 / [k]_Yee (operator on E when B uses Yee) */
};

typedef void *(*relpic_alloc_fn)(size_t bytes, void *user);
typedef void (*relpic_free_fn)(void *device_ptr, void *user);

/* Device binding.  stream is a hipStream_t (NULL = the null stream).  If alloc
 * is non-NULL all device memory comes from alloc/free (e.g. PyTorch's caching
 * allocator); otherwise hipMalloc/hipFree. */
typedef struct {
  int device;
  void *stream;
  relpic_alloc_fn alloc;
  relpic_free_fn free;
  void *user;
} relpic_device;

typedef struct relpic_sim relpic_sim;

/* FP64 diagnostics (a7), computed on the GPU in FP64 in either precision.
 * w_field = 1/2 sum (E^2 + B^2) dV; w_kin = sum over alive macro-particles of
 * (Q / (q/m)) (gamma - 1); gauss_max = max |d- . E - rho - rho_bg| over the
 * interior nodes (customized divergence for M > 1; the window's 2M + 2 edge
 * cells are excluded); rho_max = max |rho| of the particles (the scale for
 * gauss_max); charge = sum rho dV of the particles. */
typedef struct {
  int64_t step;
  int64_t window_start;
  int64_t n_alive;
  double time;
  double w_field;
  double w_kin;
  double gauss_max;
  double rho_max;
  double charge;
  int32_t error_word; /* bit 0: a particle moved more than one cell; bit 1: NaN momentum */
} relpic_diag;

/* App. C: constrained least-squares fit of M axial coefficients to the
 * leapfrog operator [k1]_t = sin(k1 dt/2)/(dt/2) at kappa = dx1/dt, with
 * consistency order p (even), super-Gaussian weight FWHM wk1 (in units of
 * k_g1) and exponent nsg.  C_out: caller-owned, length M.  max_rel_err_out
 * (nullable): max relative symbol error for k1 dx1/2 <= 1. */
relpic_status relpic_fit_coefficients(double kappa, int M, int p, double wk1, double nsg, double *C_out,
                                      double *max_rel_err_out);

/* The same fit to another target (RELPIC_FIT_TIME or RELPIC_FIT_E_WITH_YEE_B);
 * max_rel_err_out is then the error against that target. */
relpic_status relpic_fit_operator(double kappa, int M, int p, double wk1, double nsg, int target, double *C_out,
                                  double *max_rel_err_out);

/* Create a simulation.  Returns RELPIC_EUNSTABLE if
 * (dt/2)^2 * max_k sum_d [k]_d^2 >= 1 for the chosen operators. */
relpic_status relpic_create(const relpic_grid *grid, const relpic_solver *solver, relpic_precision prec,
                            const relpic_device *dev, relpic_sim **out);

relpic_status relpic_destroy(relpic_sim *sim);

/* Add a particle species with charge-to-mass ratio q_over_m (electrons: -1),
 * charge Q of one macro-particle and room for `capacity` particles (at most
 * 2^32 bytes per particle array: 2^30 particles in FP32, 2^29 in FP64;
 * RELPIC_EINVAL beyond).
 * q_over_m = 0 gives a ballistic species: its momenta never change (no
 * force), it still deposits current, and its kinetic energy is not counted
 * in the diagnostics. */
relpic_status relpic_add_species(relpic_sim *sim, double q_over_m, double Q, int64_t capacity, int *species_id);

/* Append n particles (host arrays): cell [n][ndim] int32, offset [n][ndim]
 * in [-1/2, 1/2), u [n][3].  Rounded to FP32 in FP32 mode.  RELPIC_ERANGE if
 * a cell lies outside the grid (window: outside [2, n1 - 3] of the current
 * window) or the capacity is exceeded. */
relpic_status relpic_load_particles(relpic_sim *sim, int species, int64_t n, const int32_t *cell,
                                    const double *offset, const double *u);

/* Plasma injection at every window shift into the slab at window cell n1 - 3:
 * ppc[d] particles per cell per dimension on a regular sub-lattice
 * (offsets (a + 1/2)/ppc - 1/2), momenta uth * N(0,1) per component drawn
 * from splitmix64 stream `seed` (counter = running injected-particle index *
 * 3 + component, Box-Muller on consecutive uniforms).  The index and the
 * particle ids count a slab's particles in row order (x2 fastest, then x3,
 * the sub-lattice point fastest within a cell); a species sorted by tiles
 * stores them in its tile order instead. */
relpic_status relpic_set_injection(relpic_sim *sim, int species, const int *ppc, double uth, uint64_t seed);

/* Immobile background charge density (node-centred, dense layout above,
 * window-relative), added to rho in the Gauss diagnostic. */
relpic_status relpic_set_background_rho(relpic_sim *sim, const double *rho, int64_t count);

/* Enqueue nsteps PIC steps on the bound stream (asynchronous). */
relpic_status relpic_step(relpic_sim *sim, int64_t nsteps);

/* Wait for the bound stream; returns RELPIC_EDEVICE if a kernel set the error word. */
relpic_status relpic_sync(relpic_sim *sim);

/* Copy a field to host FP64 (synchronizing); count must equal n1*n2*n3. */
relpic_status relpic_read_field(relpic_sim *sim, relpic_field f, double *host, int64_t count);

/* Overwrite a field from host FP64 (synchronizing). */
relpic_status relpic_write_field(relpic_sim *sim, relpic_field f, const double *host, int64_t count);

/* Device address and element size (4 or 8) of a field array in storage
 * order; with the moving window the x1 index of storage is (global mod n1). */
relpic_status relpic_field_device_ptr(relpic_sim *sim, relpic_field f, void **device_ptr, int *elem_bytes);

/* Copy particles of a species to host (synchronizing).  cell [cap][ndim]
 * (x1 global), offset [cap][ndim], u [cap][3], alive [cap], id [cap]
 * (nullable: the particle's load order within the species, injected
 * particles numbered after); *n_out = number of particle slots (alive or
 * dropped).  Slots are in the library's current (cell-sorted) order. */
relpic_status relpic_read_particles(relpic_sim *sim, int species, int64_t cap, int32_t *cell, double *offset,
                                    double *u, uint8_t *alive, int64_t *id, int64_t *n_out);

/* Particle sort (a2).  The push kernel deposits through per-workgroup LDS
 * tiles and sums wavefronts of particles that share a cell, which pays off
 * when particles are stored in cell order.  Species are sorted by cell
 * (dropped particles removed) before the first step after a load, and every
 * `interval` steps if interval > 0 (default 25: particles that drift into
 * other cells slowly break the order up).  Sorting synchronizes the stream. */
relpic_status relpic_sort_particles(relpic_sim *sim);
relpic_status relpic_set_sort_interval(relpic_sim *sim, int64_t interval);

/* Fused field update (a5), 3D grids only.  The leapfrog of Eq. 1 advances E
 * from step n to n + 1 and B from n + 1/2 to n + 3/2 in one pass over the
 * grid when no window shift falls between them (and to n + 1 at the end of a
 * relpic_step call): E^{n+1} = E^n + dt (curl- B^{n+1/2} - J^{n+1/2}), then
 * B^{n+3/2} = B^{n+1/2} - dt curl+ E^{n+1}, reading and writing each field
 * once (12 words per cell instead of 18).  The results are those of the
 * separate updates up to floating-point contraction.  It needs whole x1
 * lines in one workgroup (n1 <= 512, n1 >= 2 x the staged halo: 2 for Yee,
 * 32 for M = 16, 64 otherwise), n2 even, and a
 * second set of E arrays (3 n1 n2 n3 values, allocated at creation when the
 * grid qualifies; the E buffers alternate between the two sets, so device
 * pointers from relpic_field_device_ptr for E are valid only until the next
 * relpic_step).  On by default where supported; enable = 1 on a grid that
 * does not qualify returns RELPIC_EINVAL.  *active (may be null) receives
 * whether the fused update is in use. */
relpic_status relpic_set_fused_fields(relpic_sim *sim, int enable, int *active);

/* Current filter (f1): the 5-pass low-pass filter with which Secs. 2.2-3 and
 * Table 2 quote the self-force F1 (quadratic shape plus filter).  Reading:
 * npass passes of the binomial (1/4, 1/2, 1/4) along x1 and one compensating
 * pass (-c/4, 1 + c/2, -c/4), symbol cos^(2 npass)(k1 dx1/2) (1 + c
 * sin^2(k1 dx1/2)); npass = 4, c = 5 reproduces all three printed filtered
 * self-forces.  Applied every step to J1 (after the J1 correction), J2 and
 * J3 on each x1 line the particles deposited on, before the E update; a line
 * is zero beyond a moving window's ends and wraps when x1 is periodic.  The
 * same filter is applied to the density of relpic_diagnostics, so that
 * gauss_max measures Gauss's law for the filtered density, which the filtered
 * current conserves.  npass = 0 turns the filter off (the default); npass
 * in 0..16, c finite when npass > 0, n1 at most 4096 (RELPIC_EINVAL
 * otherwise).  Single runs only: batches and the adjoint run unfiltered. */
relpic_status relpic_set_current_filter(relpic_sim *sim, int npass, double comp);

/* Self-consistent initial fields of the loaded charges streaming along x1 at
 * beta (Sec. 2.1's fields in terms of the charge density, ultra-relativistic
 * limit), so that a relativistic beam does not start in zero fields (which
 * leaves a static image of opposite charge behind and radiates the sudden
 * start).  For axial operators with [k]_E1 [k]_B1 = [beta k1]_t^2 the
 * transverse field of every x1 slice is the lattice transverse Poisson field
 * of that slice's charge (-lap_perp phi = rho, Yee x2/x3 differences,
 * periodic), E_perp = -grad_perp phi, E1 = -(1 - beta^2) d1 phi, B = beta x E
 * on B's lattice points (B3 at i1 + 1/2 from the E2 of i1 and i1 + 1).  rho
 * is every species' charge at the current positions.  The part of a
 * slice's charge that is uniform over x2 and x3 has no such field and is
 * left out: the fields are exact for a beam whose slice charge is
 * neutralized (e.g. by a co-moving, transversely uniform ballistic species
 * of opposite charge), which is how a periodic transverse grid stands in for
 * open space.  Overwrites E and B; only before the first step (else
 * RELPIC_ESTATE); 0 < beta <= 1.  Synchronizing. */
relpic_status relpic_init_beam_fields(relpic_sim *sim, double beta);

/* FP64 diagnostics (synchronizing). */
relpic_status relpic_diagnostics(relpic_sim *sim, relpic_diag *out);

/* Current step count and window start (host-side bookkeeping, no sync). */
relpic_status relpic_get_step(relpic_sim *sim, int64_t *step, int64_t *window_start);

/* Half-width of the FIR J1 correction along x1 (0 for Yee). */
relpic_status relpic_correction_halfwidth(relpic_sim *sim, int *halfwidth);

/* Per-kernel timing with HIP events recorded on the bound stream around every
 * launch (adds a small gap between launches; off by default).  Kernel classes:
 * 0 push+deposit, 1 J1 correction, 2 B update (curl E), 3 E update (curl B),
 * 4 window shift and injection, 5 current added to E inside the deposit box
 * (or, after a fused update, cleared there), 6 merge of the push workgroups'
 * deposit boxes, 7 fused E and B update, 8 current filter. */
#define RELPIC_NUM_KERNEL_CLASSES 9
typedef struct {
  int64_t launches[RELPIC_NUM_KERNEL_CLASSES];
  double total_ms[RELPIC_NUM_KERNEL_CLASSES];
} relpic_profile;

/* Enable (1) or disable (0) per-kernel timing; enabling clears the totals. */
relpic_status relpic_profile_enable(relpic_sim *sim, int on);

/* Synchronize and return the totals accumulated since enabling. */
relpic_status relpic_profile_read(relpic_sim *sim, relpic_profile *out);

/* The push+deposit launches (class 0) of one species alone, accumulated
 * since enabling: number of launches and total time in ms (synchronizing). */
relpic_status relpic_profile_read_species(relpic_sim *sim, int species, int64_t *launches, double *total_ms);

/* ---- Batched many-run path ------------------------------------------------
 *
 * A batch advances many independent 2D runs with a periodic x1 boundary,
 * each with its own grid (n1, n2, dx1, dx2), time step and axial operator
 * (Yee or customized, its own M and C_l) and its own particles, as one
 * launch per phase of the step over all runs; the launches between two
 * particle sorts are recorded once into a HIP graph and replayed.  Every run
 * computes what a single relpic_sim with the same descriptors computes (the
 * per-cell and per-particle device code is shared).
 *
 * Each run is a relpic_sim owned by the batch (relpic_batch_run): species,
 * particle loads, field reads and writes and diagnostics use the single-run
 * calls on that handle.  Calling relpic_step on a run handle is allowed; the
 * batch notices and rebuilds its tables at its next step.  Runs may not use
 * plasma injection.
 *
 * Field kernels work on tiles of 128 x1 cells (one thread each) that march
 * through a range of x2 rows: shape 0, 1, 2 = 4, 8, 16 rows per tile, chosen
 * per run.  The default is 8 rows; relpic_batch_autotune measures and picks. */
typedef struct relpic_batch relpic_batch;

/* Create nruns runs from grids[nruns] and solvers[nruns] (NULL: all Yee),
 * with the validation of relpic_create per run.  RELPIC_EINVAL unless every
 * grid is 2D with bc1 = RELPIC_BC_PERIODIC. */
relpic_status relpic_batch_create(int nruns, const relpic_grid *grids, const relpic_solver *solvers,
                                  relpic_precision prec, const relpic_device *dev, relpic_batch **out);

/* Destroys the batch and its run handles. */
relpic_status relpic_batch_destroy(relpic_batch *batch);

/* Run handle (owned by the batch, valid until relpic_batch_destroy). */
relpic_status relpic_batch_run(relpic_batch *batch, int run, relpic_sim **sim);

/* Enqueue nsteps steps of every run on the bound stream (asynchronous).  The
 * first step after particle loads sorts them (synchronizing); particles are
 * re-sorted every graph_steps steps (every 20 with graphs off). */
relpic_status relpic_batch_step(relpic_batch *batch, int64_t nsteps);

/* Wait for the stream; RELPIC_EDEVICE if a kernel set the error word. */
relpic_status relpic_batch_sync(relpic_batch *batch);

/* Steps per recorded graph (even; 0 = launch every kernel directly).
 * Default 20. */
relpic_status relpic_batch_set_graph_steps(relpic_batch *batch, int steps);

/* Tile shape per run (shape[nruns], values 0..2; NULL keeps the current
 * shapes) and the field kernels' grid: grid_workgroups = 0 launches one
 * workgroup per tile, a positive multiple of 8 launches that many
 * persistent workgroups that loop over the tiles. */
relpic_status relpic_batch_set_tiling(relpic_batch *batch, const int *shape, int grid_workgroups);
relpic_status relpic_batch_get_tiling(relpic_batch *batch, int *shape, int *grid_workgroups);

/* Autotuner report (times are per launch of the B update, in ms). */
typedef struct {
  double ms_uniform[3];    /* every run on shape 0, 1, 2; one workgroup per tile */
  double ms_model;         /* per-run shapes from the fitted per-tile cost of each shape */
  double ms_persistent[2]; /* best assignment on 4096 and 8192 persistent workgroups (0: not tried) */
  double ms_chosen;
  int choice;              /* 0..2: uniform shape, 3: per-run model */
  int grid_workgroups;     /* field-kernel grid chosen */
  int runs_per_shape[3];
} relpic_batch_tune;

/* Time the B update (curl E) of the whole batch under each uniform tile
 * shape, fit a cost per tile for each shape, give every run the shape whose
 * modelled cost (tiles x cost per tile) is lowest, time that, then try
 * persistent grids; keep the fastest.  reps launches per timing.  Leaves the
 * simulation state unchanged (the timed launches write only the B buffer
 * that is free between calls).  Synchronizing. */
relpic_status relpic_batch_autotune(relpic_batch *batch, int reps, relpic_batch_tune *out);

/* relpic_read_field on one run. */
relpic_status relpic_batch_read_field(relpic_batch *batch, int run, relpic_field f, double *host, int64_t count);

/* ---- Adjoint of the field advance ------------------------------------------
 *
 * Gradient of a field loss with respect to the axial coefficients C_1..C_M
 * (customized operator of Sec. 3 / App. C; M = 1 is Yee's C_1), by
 * reverse-mode differentiation of the field advance (Eq. 1 with the axial
 * operators) and of the J1 correction G = K^-1, with time-step checkpoints.
 *
 * The run: a 2D periodic grid, fields zero at t = 0, one ballistic species
 * (constant momenta, so the deposited current does not depend on C), nsteps
 * steps.  With b_n = B^{n-1/2}, e_n = E^n and B^n = (b_n + b_{n+1}) / 2:
 *   L = sum_{n=1..nsteps} dx1 dx2 dt * sum over points outside the box of
 *       E1^2 (at E1's points) + (E2 - B3c)^2 (at E2's points (i1, i2 + 1/2)),
 * where B3c(i1) = (B^n_3(i1 - 1) + B^n_3(i1)) / 2 is B3 moved onto E2's point
 * and the box of step n has centre (x1 + v1 n dt, x2) and half-widths
 * (half1, half2), physical units, not wrapped.  E2 - B3 is the transverse
 * force on a beta = 1 particle, zero for the bunch's own field in the
 * continuum; outside the box it measures the numerical field. */
typedef struct {
  double x1, x2;       /* box centre at t = 0 */
  double v1;           /* box velocity along x1 (units of c) */
  double half1, half2; /* half-widths */
} relpic_loss_box;

typedef struct relpic_adj relpic_adj;

/* grid: 2D, bc1 periodic.  C0: M coefficients used to validate the set-up
 * (M in 1..8).  checkpoint_every: steps between stored field states (the
 * backward pass recomputes each segment from its checkpoint). */
relpic_status relpic_adj_create(const relpic_grid *grid, int M, const double *C0, relpic_precision prec,
                                const relpic_device *dev, int64_t nsteps, int checkpoint_every,
                                const relpic_loss_box *box, relpic_adj **out);
relpic_status relpic_adj_destroy(relpic_adj *adj);

/* The ballistic species: n particles of charge Q each (layout as in
 * relpic_load_particles).  Once per adjoint object. */
relpic_status relpic_adj_load_particles(relpic_adj *adj, double Q, int64_t n, const int32_t *cell,
                                        const double *offset, const double *u);

/* Run the nsteps forward with coefficients C[M] from the initial state and
 * return the loss (synchronizing).  RELPIC_EUNSTABLE if C breaks the Courant
 * limit. */
relpic_status relpic_adj_forward(relpic_adj *adj, const double *C, double *loss);

/* dL/dC_l, l = 1..M, at the coefficients of the last forward call
 * (synchronizing); RELPIC_ESTATE without a forward call. */
relpic_status relpic_adj_backward(relpic_adj *adj, double *dLdC);

/* The simulation the adjoint runs on (owned by it): fields after the last
 * forward call. */
relpic_status relpic_adj_sim(relpic_adj *adj, relpic_sim **sim);

/* ---- k-space field of a streaming charge (FP64, on the GPU) -----------------
 *
 * Sec. 2, Eq. 13 (general beta through Eqs. 8-9): the on-axis E1 of a point
 * charge q moving at beta along x1 through a 2D grid with the Yee transverse
 * operator and the axial operators C_1..C_M on E and CB on B (Yee: M = 1,
 * C = NULL or {1}; X = [beta k1']_t^2 - [k]_E1 [k]_B1, prefactor i/[k]_B1),
 * particle on a node, in the steady state of an infinite grid.  The k1
 * integral runs over the zones nu = -nu_max..nu_max of the aliased density
 * (App. A) with the k2 integral in closed form (App. D, causal pole
 * prescription).  Computed in FP64 by quadrature on the device. */
typedef struct {
  int M;           /* operator on E: [k]_E1 */
  const double *C;
  double kappa;    /* dx1 / dt (> 1) */
  double r;        /* dx2 / dx1 */
  double beta;     /* 0 < beta <= 1 */
  int shape_order; /* B-spline order of the deposit along x1 (2: quadratic) */
  int tpow;        /* power of the transverse density factor 1 - sin^2(k2 dx2/2)/2:
                      0 for the paper's linear transverse shape, 1 for a quadratic
                      deposit, 2 for a quadratic deposit and gather */
  int nu_max;      /* alias zones (the paper uses 1) */
  int MB;          /* operator on B, [k]_B1 (MB = 0: the same as on E) */
  const double *CB;
} relpic_kspace;

/* out[i] = E1 dx1 / q at the E1 point i1_rel[i] cells ahead of the particle
 * (E1 sits at i1 + 1/2, so i1_rel = 0 is half a cell ahead, -1 half a cell
 * behind).  Synchronizing; dev may be NULL (device 0, null stream, hipMalloc). */
relpic_status relpic_kspace_e1(const relpic_kspace *q, const relpic_device *dev, int64_t npts, const double *i1_rel,
                               double *out);

/* Self-force F1 dx1 / q^2 in the paper's convention (Eqs. 19, 25): the field
 * weighted by the gather's unaliased shape of order gather_order. */
relpic_status relpic_kspace_self_force(const relpic_kspace *q, const relpic_device *dev, int gather_order,
                                       double *out);

/* E1 at any E1 point of a 2D or a 3D grid (Eq. 9 with the x2 and x3
 * integrals; off axis, Sec. 2.2 gives only i2 = 0 and notes the other rows
 * follow from the same integral).  ndim = 2: out[k] = E1 dx1 / q at
 * (i1_rel[k] + 1/2, i2[k]) relative to the particle's node (i3 and r3
 * unused, i3 may be NULL); ndim = 3: out[k] = E1 dx1^2 / q at (i1_rel[k] +
 * 1/2, i2[k], i3[k]), q->r = dx2/dx1, r3 = dx3/dx1 > 0.  The transverse
 * operators are Yee's and tpow applies to each transverse direction; the
 * axial operators, beta, shape and zones as for relpic_kspace_e1 (with i2 =
 * 0 in 2D it returns the same quantity).  FP64 quadrature: in 3D the x3
 * integral is in closed form and the x2 integral a tanh-sinh rule inside
 * every k1 node (about 1e7 integrand evaluations per point).  npts <= 2^20;
 * |i2|, |i3| <= 100000.  Synchronizing; dev may be NULL. */
relpic_status relpic_kspace_field(const relpic_kspace *q, const relpic_device *dev, int ndim, double r3, int64_t npts,
                                  const double *i1_rel, const int32_t *i2, const int32_t *i3, double *out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): relpic_kspace_e1
 * without any device or host heap allocation.  Same arguments and results
 * (the same panels and kernel); dev may be NULL (device 0, null stream) but
 * must carry no allocator callbacks.  Its device scratch (quadrature panels,
 * point phases, per-point results: 88 KiB) is a static array of the library,
 * one copy per GPU, held until the process ends; limits: npts <= 4096
 * (RELPIC_EINVAL beyond) and at most 1024 quadrature panels (RELPIC_ERANGE
 * beyond; lower nu_max).  Every call on a GPU shares that GPU's scratch:
 * calls that overlap on one GPU (two host threads or two streams) race.
 * Nothing in the scratch needs clearing (each call writes every value it
 * reads).  Synchronizing. */
relpic_status relpic_kspace_e1_noalloc(const relpic_kspace *q, const relpic_device *dev, int64_t npts,
                                       const double *i1_rel, double *out);

/* ---- Self-force and line-out against the k-space field (Sec. 2.2, Eq. 19) ---
 *
 * EB[6 k + c] (caller-owned, count x 6 doubles) = E1, E2, E3, B1, B2, B3 at
 * particle slot first + k of a species (slots in relpic_read_particles
 * order), interpolated at the particle's position with the push's quadratic
 * B-spline, each component from its own staggered points, at the current
 * step (E^n and B^n), in FP64.  The self-force on a particle of charge Q is
 * Q (E + v x B); for a charge moving along x1 it is F1 = Q E1 (Eq. 19
 * measures the same quantity in k space).  Dropped particles give zeros.
 * Synchronizing.  RELPIC_ERANGE if the slots exceed the species. */
relpic_status relpic_gather_particles(relpic_sim *sim, int species, int64_t first, int64_t count, double *EB);

/* The simulated on-axis E1 around one particle next to the k-space
 * prediction for the same points (Eq. 13 in 2D; in 3D Eq. 9 with both
 * transverse integrals, relpic_kspace_field at r3 = dx3/dx1, and the values
 * are E1 dx1^2 / Q instead of E1 dx1 / Q).  The particle (slot
 * `slot` of `species`) must sit on an x1 node (|offset1| <= 1e-6, else
 * RELPIC_ERANGE; a beta = 1 charge returns to a node every kappa steps when
 * kappa is an integer).  For each k, sim_out[k] = E1 dx1 / Q at the E1
 * point i1_rel[k] cells ahead of the particle's cell on its x2 row (E1 sits
 * at i1 + 1/2), and theory_out[k] = relpic_kspace_e1 of q at the same
 * point; the residual is their difference.  q must describe this run: its
 * M, C, kappa (= dx1/dt) and r (= dx2/dx1) equal the simulation's (else
 * RELPIC_EINVAL); beta, shape_order, tpow and nu_max are the caller's.
 * Window runs: every point inside the window (else RELPIC_ERANGE).
 * npts <= 4096.  Synchronizing. */
relpic_status relpic_e1_residual(relpic_sim *sim, int species, int64_t slot, const relpic_kspace *q, int64_t npts,
                                 const int32_t *i1_rel, double *sim_out, double *theory_out);

const char *relpic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RELPIC_H */
