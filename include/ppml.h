/*
 * ppml.h -- C ABI of the MI355X solver for the operator-splitting PPML
 * scheme of Kulikov & Vorobyov, "Using the PPML approach for constructing a
 * low-dissipation, operator-splitting scheme for numerical simulations of
 * hydrodynamic flows" (arXiv:1607.01105).
 *
 * The problem follows the paper's statement (Sec. 2, eqs. (1)-(4)): the
 * unknowns are the densities of mass rho, momentum rho*v, total energy
 * rho*E and internal energy rho*eps of an ideal gas with p = (gamma-1) rho eps,
 * on a uniform Cartesian mesh, optionally in a fixed external potential Phi,
 * advanced with the CFL time step of Sec. 2.1.  One step = Eulerian stage
 * (acoustic Riemann problem on parabolas, pressure and force terms, no
 * advection; Sec. 2.1-2.2) + Lagrangian stage (upwind parabolic advection
 * with the 9-point transverse velocity; Sec. 2.3) + total-energy correction
 * (Sec. 2.4), optionally preceded by the self-gravity potential solve
 * (Sec. 2.5).  Every step runs in HIP kernels on the caller's stream (the
 * self-gravity transforms as rocBLAS GEMMs on the same stream).
 *
 * Conventions shared by every function:
 *  - Return value: PPML_OK (0) or a negative ppml_status.  Nothing throws
 *    across the ABI.  ppml_last_error() gives a thread-local detail string.
 *  - Memory: the caller owns all device memory and the HIP stream; the
 *    library borrows the pointers for the lifetime of the grid and owns only
 *    the small opaque host object (and short-lived staging buffers inside
 *    the set/get calls).
 *  - Device state layout (structure of arrays, x fastest, C order
 *    [z][y][x]): F = 3 + ndim fields of n[0]*n[1]*n[2] values of the storage
 *    type (float for PPML_FP32, double for PPML_FP64), in the order
 *    rho, rho*vx [, rho*vy [, rho*vz]], rho*E, rho*eps.
 *  - Host arrays are FP64, interior cells only, C order [z][y][x].
 *  - Asynchrony: ppml_step only enqueues work; functions that return values
 *    to the host (get_*, totals, sync) synchronize the stream first.
 */
#ifndef PPML_H
#define PPML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PPML_OK = 0,
    PPML_EINVAL = -1,     /* bad descriptor, argument or initial state      */
    PPML_ENOMEM = -2,     /* staging allocation failed                      */
    PPML_EHIP = -3,       /* a HIP runtime call failed                      */
    PPML_ENONFINITE = -4, /* a step produced rho <= 0, eps <= 0 or NaN/Inf  */
    PPML_EBUDGET = -5,    /* request exceeds the memory budget              */
    PPML_ESTATE = -6      /* call not valid in the object's current state   */
} ppml_status;

typedef enum { PPML_FP32 = 0, PPML_FP64 = 1 } ppml_precision;

/* Boundary conditions (the paper names periodic, outflow, reflecting and
 * inflow boundaries in its tests; their ghost-cell form is a reading:
 * periodic = wrap, outflow = copy of the nearest interior cell, reflect =
 * mirror image with the wall-normal momentum negated, inflow = the prescribed
 * state of the face (ppml_desc.inflow) in every ghost cell; three ghost layers
 * per side, filled axis by axis x, y, z, so a cell that is a ghost along
 * several axes follows the last of them). */
typedef enum { PPML_PERIODIC = 0, PPML_OUTFLOW = 1, PPML_REFLECT = 2, PPML_INFLOW = 3 } ppml_bc;

/* Conserved fields (Sec. 2, eqs. (1)-(4)). */
typedef enum { PPML_RHO = 0, PPML_MX = 1, PPML_MY = 2, PPML_MZ = 3, PPML_ETOT = 4, PPML_EINT = 5 } ppml_field;

/* Fixed external potential whose gradient enters the momentum and energy
 * equations (eqs. (2)-(3)):
 *   PPML_POT_LOG:     Phi = v0^2/2 ln(rc^2 + X^2 + Y^2 + Z^2/q^2), X = x - cx, ...
 *                     pot = {v0, rc, q, cx, cy, cz}
 *   PPML_POT_UNIFORM: Phi = gx x + gy y + gz z;  pot = {gx, gy, gz}
 *   PPML_POT_HALO:    the dark-matter halo of Sec. 4, density
 *                     rho0 / (1 + (r/r0)^2) out to the halo radius rh (r from
 *                     (cx, cy, cz)); grad Phi = G M(r) / r^2 (radial, outward)
 *                     with M(r) = 4 pi rho0 r0^3 (u - atan u), u = min(r, rh)/r0;
 *                     pot = {G rho0, r0, rh, cx, cy, cz}, r0, rh > 0; 3-D
 *                     grids, stepped alone (not in a batch)                */
typedef enum { PPML_POT_NONE = 0, PPML_POT_LOG = 1, PPML_POT_UNIFORM = 2, PPML_POT_HALO = 3 } ppml_potential;

/* Descriptor flags.  PPML_FLAG_FIRST_ORDER: piecewise-constant states in both
 * stages instead of parabolas -- the first-order scheme of Sec. 2.1 that the
 * paper compares against (its shock-tube comparison).
 * PPML_FLAG_ISOTHERMAL: the isothermal approximation the paper adopts for its
 * galactic disks (Sec. 4, gamma = 1): pressure p = iso_cs^2 rho and sound
 * speed iso_cs in the Riemann problem and the CFL step.  The isothermal model
 * has no energy equation: rho E and rho eps are still stored (set from the
 * given p with gamma as usual) and carried by the same updates -- with
 * gamma = 1 the eps equation loses its work term -- but feed nothing back;
 * the vacuum branch of Sec. 2.4, which acts on them, is off. */
enum { PPML_FLAG_FIRST_ORDER = 1, PPML_FLAG_ISOTHERMAL = 2 };

typedef struct {
    int32_t ndim;          /* 1, 2 or 3                                             */
    int32_t prec;          /* ppml_precision of the stored state and the stencil    */
    int64_t n[3];          /* interior cells per axis; 1 for axes >= ndim           */
    double lo[3], hi[3];   /* domain extents; cell size h[d] = (hi-lo)/n            */
    double gamma;          /* ratio of specific heats, > 1                          */
    double cfl;            /* Courant number, 0 < cfl < 1 (the paper uses 0.2)      */
    int32_t bc_lo[3];      /* ppml_bc of the low face of each axis                  */
    int32_t bc_hi[3];      /* ppml_bc of the high face                              */
    double vacuum_ratio;   /* Sec. 2.4 vacuum threshold relative to the initial
                              mean density (the paper: five orders, 1e-5)            */
    int32_t potential;     /* ppml_potential                                        */
    int32_t flags;         /* PPML_FLAG_* bits; 0 = the paper's PPML scheme          */
    double pot[8];         /* potential parameters (see ppml_potential)             */
    int32_t tile;          /* work-group tile shape of the stage kernels: index in
                              the list of ppml_tile_shape (0 = default); changes
                              the speed only, never the results                  */
    int32_t self_gravity;  /* 1: add the force of the gas's own potential (Sec. 2.5,
                              see below); 0: none.  Needs ndim = 3, cubic cells and
                              the origin off the centres of the shell cells     */
    double inflow[6][5];   /* ghost state (rho, vx, vy, vz, p) of face 2*axis+side
                              (side 0 low, 1 high) where that face is PPML_INFLOW;
                              rho, p > 0; converted like ppml_set_primitive   */
    double grav_G;         /* gravitational constant G of Delta Phi = 4 pi G rho
                              (used when self_gravity = 1; > 0)                  */
    double iso_cs;         /* sound speed of PPML_FLAG_ISOTHERMAL (> 0)             */
} ppml_desc;

/* Self-gravity (Sec. 2.5, the Poisson solver).  Before each step's Eulerian
 * stage the potential of the current density is found from the 27-point
 * finite-difference Poisson equation (weights -38/9, 4/9, 1/9, 1/36;
 * right-hand side 4 pi G h^2 rho) on the interior cells, with the values of
 * a one-cell shell around the box taken from the two-term multipole
 * expansion about the coordinate origin (monopole and quadrupole; the
 * quadrupole with MacCullagh's factor 1/2) and moved to the right-hand side;
 * the Dirichlet problem is solved exactly by sine transforms along each axis
 * (sums and differences of mirror cells, then products with the half-size
 * odd- and even-mode sine matrices on the matrix cores), division by the
 * stencil's eigenvalues and the inverse transforms.  The force terms of
 * eqs. (2)-(3) then use the central difference of the potential across each
 * cell, added to any fixed potential's gradient.  The scratch area grows by
 * the potential, two work arrays of the grid's size, the shell terms of the
 * outer layer of cells and the sine tables (see ppml_scratch_bytes).  Grids with self-gravity step alone, not in a
 * batch. */

/* Work-group tile shapes of the stage kernels for grids of ndim dimensions:
 * ppml_tile_count returns how many there are (>= 1) or PPML_EINVAL;
 * ppml_tile_shape gives the x and y extent of shape `variant` (a work group
 * of tx*ty threads owns a tx x ty column of cells; 3-D kernels march it
 * along z).  Used by the autotuner, which times the shapes on the caller's
 * workload; every shape computes bit-identical results. */
int ppml_tile_count(int32_t ndim);
int ppml_tile_shape(int32_t ndim, int32_t variant, int32_t *tx, int32_t *ty);

typedef struct ppml_grid ppml_grid;

/* Bytes of device memory the caller must provide for the state
 * ((3+ndim) * cells * sizeof(storage type)) and for the scratch area (the
 * Eulerian-stage output, the control block and reduction partials).
 * Returns 0 for an invalid descriptor. */
size_t ppml_state_bytes(const ppml_desc *d);
size_t ppml_scratch_bytes(const ppml_desc *d);

/* Create a grid on the current HIP device.  state_dev and scratch_dev are
 * device pointers of at least ppml_state_bytes / ppml_scratch_bytes bytes,
 * 256-byte aligned; hip_stream is a hipStream_t (NULL = default stream).
 * The state is undefined until ppml_set_primitive or ppml_set_conserved.
 * Errors: PPML_EINVAL (descriptor: ndim, n >= 1, reflect needs n >= 3,
 * gamma > 1, 0 < cfl < 1, extents, enums), PPML_EHIP. */
int ppml_create(const ppml_desc *d, void *state_dev, void *scratch_dev, void *hip_stream, ppml_grid **out);

/* Set the state from primitive variables at cell centres (Sec. 2): e = p/(gamma-1),
 * rho*E = e + rho |v|^2 / 2, computed in FP64 on the device and rounded to the
 * storage type.  vy / vz may be NULL (zero); components of axes >= ndim are
 * ignored.  Resets the time to 0, the step count to 0, records the FP64 mean
 * density for the vacuum threshold and computes the first CFL maxima.
 * Errors: PPML_EINVAL (NULL rho/p, rho <= 0 or p <= 0 or non-finite values),
 * PPML_ENOMEM, PPML_EHIP. */
int ppml_set_primitive(ppml_grid *g, const double *rho, const double *vx, const double *vy, const double *vz,
                       const double *p);

/* Set the conserved fields directly (checkpoint restore): f[ppml_field]
 * host arrays, entries of unused momentum axes may be NULL.  rho_mean0 > 0
 * sets the vacuum reference density (<= 0: mean of the given rho); t sets
 * the time.  Errors as ppml_set_primitive. */
int ppml_set_conserved(ppml_grid *g, const double *const *f, double rho_mean0, double t);

/* Enqueue nsteps steps.  dt_fixed > 0: use that time step; otherwise the CFL
 * step tau = cfl * min_d h_d / (max|v| + max c) of the current state (maxima
 * taken separately, Sec. 2.1).  t_stop > 0: clip the step so the run ends at
 * t_stop; steps after that are no-ops.  Asynchronous: errors of the step
 * itself are reported by the next synchronizing call.  Calls of 32 steps or
 * more replay a HIP graph of 32 steps (captured once per grid on a private
 * stream, launched on the grid's stream) unless per-step timing is on or
 * the grid has self-gravity; the results are the same bits.
 * Errors: PPML_EINVAL (nsteps < 0), PPML_ESTATE (state never set), PPML_EHIP. */
int ppml_step(ppml_grid *g, int32_t nsteps, double dt_fixed, double t_stop);

/* Synchronize and read the time, the last time step and the number of
 * steps taken (any pointer may be NULL).  Returns PPML_ENONFINITE if a step
 * produced a non-physical value. */
int ppml_get_time(ppml_grid *g, double *t, double *dt_last, int64_t *steps);

/* Synchronize and read the current maxima of |v| and of c over the cells. */
int ppml_max_speeds(ppml_grid *g, double *vmax, double *cmax);

/* Synchronize and copy one conserved field to host_out (FP64, cells values):
 * field 0 rho, 1 .. 3 rho v (x, y, z), 4 rho E, 5 rho eps -- the densities
 * the scheme of Sec. 2 evolves, rho eps being the internal energy carried
 * beside the total for the correction of Sec. 2.4.  Layout as for the
 * setters: interior cells, C order [z][y][x].
 * Errors: PPML_EINVAL (field of an unused axis), PPML_ENOMEM, PPML_EHIP. */
int ppml_get_conserved(ppml_grid *g, int32_t field, double *host_out);

/* Self-gravity potential (Sec. 2.5): synchronize, solve for the potential of
 * the current state and copy it to host_out as FP64, shell included:
 * (n[0]+2)(n[1]+2)(n[2]+2) values, C order [k+1][j+1][i+1] (index 0 and
 * n+1 along an axis are the shell).  Errors: PPML_EINVAL (NULL output,
 * self-gravity off), PPML_ESTATE (state never set), PPML_ENOMEM, PPML_EHIP. */
int ppml_get_potential(ppml_grid *g, double *host_out);

/* Synchronize and return the FP64 sums over all cells of the six conserved
 * densities (unused momentum axes give 0): the totals of mass, momentum and
 * total energy whose conservation the divergence form of Sec. 2 gives on
 * periodic grids (Sec. 2.4 discusses the total-energy one).  The summation
 * order is fixed, so repeated calls on the same state give identical bits. */
int ppml_totals(ppml_grid *g, double out[6]);

/* Synchronize the grid's stream; PPML_ENONFINITE if a step produced a
 * non-physical state (rho <= 0 or eps <= 0 after the energy correction of
 * Sec. 2.4) or a non-finite value. */
int ppml_sync(ppml_grid *g);

/* Destroy the host object (does not free caller memory). */
int ppml_destroy(ppml_grid *g);

/* Static description of the status code; thread-local detail of the last error. */
const char *ppml_strerror(int status);
const char *ppml_last_error(void);

/* Per-kernel timing of ppml_step, for benchmarks.  ppml_set_timing(g, cap)
 * with cap > 0 creates HIP events for up to cap steps and makes ppml_step
 * record an event before the Eulerian kernel, between the two stage kernels
 * and after the Lagrangian kernel on the grid's stream (steps beyond cap
 * are not timed); cap = 0 turns timing off and releases the events.
 * ppml_get_timing synchronizes, returns the summed kernel durations in
 * milliseconds (event-to-event on the same stream) and the number of steps
 * timed, and starts a new accumulation.  Errors: PPML_EINVAL, PPML_EHIP. */
int ppml_set_timing(ppml_grid *g, int32_t cap);
int ppml_get_timing(ppml_grid *g, double *ms_euler, double *ms_lagr, int64_t *nsteps);

/* As ppml_get_timing, with the self-gravity solve of each timed step (moments,
 * boundary values, transforms; 0 without self-gravity) split off:
 * ms[0] = gravity, ms[1] = Eulerian kernel, ms[2] = Lagrangian kernel. */
int ppml_get_timing_split(ppml_grid *g, double ms[3], int64_t *nsteps);

/* ---- Batches: many independent grids stepped together ------------------
 * A batch steps all its grids in the same kernel launches (one Eulerian and
 * one Lagrangian launch per step and dimensionality present; the launch
 * chains of different dimensionalities run concurrently on streams the
 * batch forks from its stream and joins back), optionally recorded once into
 * a HIP graph and replayed.  Each grid keeps its own
 * time step (Sec. 2.1 CFL condition of its own state), time, maxima and
 * error word, so a grid's results are the same alone and in any batch.
 * Grids keep their caller-owned memory; the batch owns two small tables
 * (device and pinned host, capacity entries).  All grids of a batch share
 * one precision.  Batch calls synchronize the batch stream before changing
 * membership or staging step counts. */
typedef struct ppml_batch ppml_batch;

/* Create a batch of up to capacity grids that steps on hip_stream (must not
 * be the legacy NULL stream when graphs are used).  budget_bytes > 0 caps the
 * summed state + scratch bytes of the admitted grids.
 * Errors: PPML_EINVAL, PPML_ENOMEM, PPML_EHIP. */
int ppml_batch_create(int32_t capacity, size_t budget_bytes, void *hip_stream, ppml_batch **out);

/* Admit a grid whose state is set; *slot receives its slot.  While admitted
 * the grid is stepped only by the batch (ppml_step returns PPML_ESTATE); its
 * get/set/totals/time/sync calls still work and, when the grid has a stream
 * of its own, first wait for the batch stream's queued work.  Errors: PPML_EBUDGET (budget or capacity
 * exhausted), PPML_ESTATE (already in a batch, state not set), PPML_EINVAL
 * (other device or precision). */
int ppml_batch_admit(ppml_batch *b, ppml_grid *g, int32_t *slot);

/* Remove the grid in slot from the batch (after the batch's queued work). */
int ppml_batch_retire(ppml_batch *b, int32_t slot);

/* Enqueue nsteps steps for every admitted grid; steps_per_slot (indexed by
 * slot, may be NULL) gives each grid's own count in [0, nsteps]: a grid stops
 * after its count (its remaining launches are no-ops).  dt_fixed and t_stop
 * as in ppml_step.  use_graph != 0 records the launches of nsteps steps into a
 * HIP graph (re-recorded after membership or nsteps change) and replays it.
 * Errors: PPML_EINVAL, PPML_EHIP. */
int ppml_batch_step(ppml_batch *b, int32_t nsteps, const int32_t *steps_per_slot, double dt_fixed, double t_stop,
                    int32_t use_graph);

/* Synchronize; PPML_ENONFINITE if any admitted grid flagged a non-physical state. */
int ppml_batch_sync(ppml_batch *b);

/* Number of admitted grids and their summed state + scratch bytes. */
int ppml_batch_info(ppml_batch *b, int32_t *count, size_t *bytes_in_use);

/* Tile shape (ppml_tile_shape index) of the batch's launches for grids of
 * ndim dimensions (default 0).  Allowed only while no grid of that
 * dimensionality is admitted; results do not depend on it.
 * Errors: PPML_EINVAL (ndim or variant), PPML_ESTATE. */
int ppml_batch_set_tile(ppml_batch *b, int32_t ndim, int32_t variant);

/* Destroy the batch (admitted grids become free-standing again). */
int ppml_batch_destroy(ppml_batch *b);

/* ---- Allocation-free stepping -------------------------------------------
 * For callers that cannot allocate memory: code under HIP graph capture
 * (with t_out and steps_out NULL), tight serving loops, harnesses that forbid
 * hipMalloc.  One call does what ppml_create on state_dev, ppml_set_conserved
 * of the state already on the device, ppml_step and ppml_get_time do, with
 * the same kernels and the same results, but allocates nothing: no device or
 * host memory, no host object, no graph.  The grid's work area (the
 * Eulerian-stage output, the control block and the totals partials: the
 * ppml_scratch_bytes of the descriptor) lies in a fixed area inside the
 * library, PPML_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on
 * that GPU until the process ends.
 *   state_dev: the conserved state in the layout above (ppml_state_bytes,
 *              256-byte aligned), caller-owned, advanced in place;
 *   rho_mean0: vacuum reference density (Sec. 2.4); <= 0: the mean of the
 *              state's density;
 *   t0:        time of the state; nsteps, dt_fixed, t_stop as in ppml_step
 *              (steps launched one by one on hip_stream);
 *   t_out, steps_out: when either is non-NULL the call synchronizes the
 *              stream and returns the time and the number of steps taken
 *              (PPML_ENONFINITE if a step produced a non-physical state);
 *              when both are NULL it only enqueues.
 * Every call on a GPU shares that GPU's work area, which keeps the last
 * call's contents (each call starts by rewriting everything it reads), so
 * calls that overlap on one GPU (other streams or threads) race: the caller
 * serializes them.  Errors: PPML_EINVAL (descriptor, self-gravity, a work
 * area above PPML_NOALLOC_SCRATCH_BYTES, NULL or misaligned state, nsteps < 0,
 * non-finite arguments), PPML_EHIP, PPML_ENONFINITE. */
#define PPML_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ppml_step_noalloc(const ppml_desc *d, void *state_dev, double rho_mean0, double t0, int32_t nsteps,
                      double dt_fixed, double t_stop, void *hip_stream, double *t_out, int64_t *steps_out);

/* Library version (major*10000 + minor*100 + patch). */
int ppml_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PPML_H */
