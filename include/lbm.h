/*
 * lbm.h -- C ABI of the MI355X (gfx950) two-phase lattice Boltzmann step
 * (D2Q9; D3Q19 and D3Q27 for 3-D lattices, see lbm_params.nz and lattice3).
 *
 * The operation is one time step of the lattice Boltzmann equation for a
 * liquid-vapour fluid driven by a chemical potential, in the two forms of
 * Z. Guo, "Well-balanced lattice Boltzmann equation for two-phase flows",
 * arXiv:2012.11075:
 *
 *   LBM_STANDARD       Sec. II: Eq. (2) with the equilibrium of Eq. (3), the
 *                      forcing term of Eq. (5) and the potential-form force
 *                      F = grad(cs2 rho) - rho grad(mu) (Eq. 6);
 *   LBM_WELL_BALANCED  Sec. III: Eq. (2) with the equilibrium of Eq. (24),
 *                      the force F = -rho grad(mu) of Eq. (25) and the
 *                      forcing term of Eq. (26).
 *
 * Both use rho and the half-force velocity of Eq. (4), the chemical potential
 * mu = mu0(rho) - kappa lap(rho) with the double-well mu0 of Eqs. (36)-(37),
 * isotropic central differences for grad and lap (Sec. II, the ICS of
 * Eq. 19 and its 9-point Laplacian companion), BGK collision with relaxation
 * time tau, and streaming f_i(x + c_i, t + 1) = f*_i(x, t) on a lattice that
 * is periodic in x and y.  Lattice units: dx = dt = c = 1, cs2 = 1/3.
 * Velocities are numbered as in the paper: c0 = (0,0), c1 = (1,0),
 * c2 = (0,1), c3 = (-1,0), c4 = (0,-1), c5 = (1,1), c6 = (-1,1),
 * c7 = (-1,-1), c8 = (1,-1).
 *
 * Memory and ownership
 *   - The caller owns every host array and the device workspace.  The library
 *     allocates no device memory; it owns only its host-side context structs
 *     and HIP graph objects (a batch also a second stream and two events),
 *     which the destroy calls free.
 *   - Host field arrays are dense, row-major double[ny][nx] (element (x, y)
 *     at index y*nx + x); 3-D: double[nz][ny][nx].  Population arrays are
 *     double[9][ny][nx]; 3-D: double[q][nz][ny][nx], q = 19 or 27.
 *   - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *     void*; NULL is the default stream).  lbm_step and lbm_batch_run are
 *     asynchronous; calls that return host data synchronise that stream.
 *   - A context (or batch) is not thread-safe; distinct ones are independent.
 *     Two contexts must not share workspace memory.
 *
 * Errors: every call returns an lbm_status; lbm_last_error() gives a message
 * for the last failing call on that context (or, for a NULL context, on the
 * calling thread).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* bad argument (sizes, tau <= 1/2, NULL, non-finite) */
  LBM_ENOSPACE = -2,    /* workspace or arena too small */
  LBM_EHIP = -3,        /* a HIP runtime call failed */
  LBM_ENONFINITE = -4,  /* observe found NaN/Inf or rho <= 0 (state kept) */
  LBM_ESTATE = -5,      /* call out of order (e.g. step before init) */
  LBM_EBUSY = -6        /* no free batch slot */
} lbm_status;

/* LBM_STANDARD: the standard LBE of Sec. II (equilibrium Eq. 3, force Eq. 6,
 * forcing term Eq. 5).  LBM_WELL_BALANCED: Sec. III (Eqs. 24-26).
 * LBM_STANDARD_EQ_FORCING: the standard LBE with the other forcing term the
 * paper names after Eq. (5), F_i = (c_i - u).F feq_i / (cs2 rho); same
 * equilibrium, force, observe pass and FP32 shift as LBM_STANDARD.  Single
 * lattices, 2-D (either force stencil) and 3-D, and batch slots, in either
 * precision. */
typedef enum {
  LBM_STANDARD = 0,
  LBM_WELL_BALANCED = 1,
  LBM_STANDARD_EQ_FORCING = 2
} lbm_scheme;

/* LBM_FP64: populations stored and updated in double precision.
 * LBM_FP32_SHIFTED: populations stored as float g_i = f_i - s_i and updated
 * in single precision, with s_i = feq_i(rho_ref, u = 0) of the scheme in use
 * (under WB rho_ref - (1 - w_0) rho0 for i = 0 and w_i rho0 otherwise,
 * Eq. 24; w_i rho_ref under the standard scheme); mass, kinetic energy and
 * max|u| are accumulated in double precision. */
typedef enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1 } lbm_precision;

typedef struct {
  int32_t nx, ny;   /* lattice size, each >= 1 */
  double tau;       /* BGK relaxation time (Eq. 2), > 1/2 */
  double beta;      /* double-well height (Eq. 36), >= 0 */
  double kappa;     /* gradient coefficient in mu = mu0 - kappa lap rho, >= 0 */
  double rho_l;     /* saturation liquid density (Eq. 36) */
  double rho_v;     /* saturation vapour density (Eq. 36) */
  double rho0;      /* constant rho0 of the WB equilibrium (Eq. 24); the paper uses 0 */
  double rho_ref;   /* reference density of the FP32 shift; ignored for FP64 */
  int32_t precision;   /* lbm_precision */
  int32_t shift_all;   /* FP32 only: 1 = shift every scheme by w_i rho_ref */
  int32_t force_stencil; /* gradients of the force (and of Eq. 26): 0 the
                          * isotropic central scheme of Sec. II; 1 the
                          * fourth-order form grad - (1/6) grad(lap), the
                          * higher-order discretisation discussed after
                          * Eq. (23) (FP64 or FP32-shifted, ny <= 65535, not
                          * in batches, block widths 256 and 512) */
  int32_t nz;            /* lattice depth: 0 or 1 for the 2-D D2Q9 lattice;
                          * > 1 for the 3-D lattice (D3Q19 or D3Q27, see
                          * lattice3) of the same method (Eqs. 24 and 26
                          * hold for general dimension; here D = 3).  3-D lattices run in FP64 or
                          * FP32-shifted storage with the central force
                          * stencil, single lattices only, ny and
                          * nz <= 65535, a z-plane of populations
                          * (q * ny * nx * element bytes, q = 19 or 27, nx
                          * rounded up to 32) below 4 GiB; one kernel per step.  Fields
                          * are then double[nz][ny][nx]. */
  int32_t lattice3;      /* velocity set of a 3-D lattice: 0 or 19 for
                          * D3Q19, 27 for D3Q27 (the 19 velocities and the
                          * 8 corners (+-1, +-1, +-1); weights 8/27, 2/27,
                          * 1/54, 1/216, and the gradient and Laplacian
                          * weighted with them).  Must be 0 on 2-D
                          * lattices.  D3Q27 tiles: block 256, depth 1..2. */
} lbm_params;

typedef struct {
  int64_t step;           /* steps taken since lbm_init / lbm_set_populations */
  double max_u;           /* max over nodes of |u| (Eq. 4 velocity) */
  double mass;            /* sum over nodes of rho */
  double kinetic_energy;  /* (1/2) sum rho |u|^2, the E(t) of Sec. IV.A */
  int32_t nonfinite;      /* 1 if any rho or u is NaN/Inf, or rho <= 0 */
  double momentum[3];     /* sum over nodes of rho u (x, y, z; z is 0 in 2-D).
                           * Eq. (2) moves the populations' momentum by the
                           * summed force of Eq. (6)/(25) each step, which
                           * vanishes in the continuum but not on the lattice
                           * away from equilibrium */
} lbm_observation;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

/* ---------------------------------------------------------- single instance */

/* Bytes of device workspace a context with these parameters needs (two
 * population copies, a field staging area and reduction partials).  Returns
 * 0 if the parameters are invalid. */
size_t lbm_workspace_bytes(const lbm_params* params);

/* Create a context over a caller-owned device workspace of `bytes` bytes
 * (256-byte aligned).  `hip_stream` is the hipStream_t all work goes to.
 * On success *out owns host state only; the workspace must outlive it. */
lbm_status lbm_create(const lbm_params* params, void* dev_workspace, size_t bytes,
                      void* hip_stream, lbm_ctx** out);

/* Set f(0) = feq(rho, u) of `scheme` (Eq. 3 or Eq. 24) from host fields.
 * ux and uy may both be NULL (u = 0).  Rejects non-finite values and
 * rho <= 0 with LBM_EINVAL.  Resets the step counter.  Synchronous. */
lbm_status lbm_init(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy,
                    lbm_scheme scheme);

/* Advance n >= 0 time steps of Eq. (2) with `scheme`, asynchronously on the
 * context stream.  Changing the scheme keeps the populations (for FP32 only
 * the storage shift is converted, an exact constant offset). */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n, lbm_scheme scheme);

/* Fields of the current state, with the same device code the step uses:
 * rho (Eq. 4), u (Eq. 4, half-force), mu (mu0 - kappa lap rho).  Any of the
 * four host arrays may be NULL; `obs` may be NULL.  Synchronous.  Returns
 * LBM_ENONFINITE (after filling the outputs) if the state holds NaN/Inf or a
 * non-positive density. */
lbm_status lbm_observe(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* mu,
                       lbm_observation* obs);

/* For callers that cannot allocate memory or wait on the host (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the scalars of lbm_observe without allocating anything and without
 * synchronizing.  Enqueues, on the context's stream, the observe pass and a
 * fixed-order finish whose result is bit-identical to lbm_observe's scalars,
 * and writes LBM_NOALLOC_DOUBLES doubles to `dev_out`, caller-owned DEVICE
 * memory: max|u|, mass, kinetic energy, non-finite flag (1.0 / 0.0),
 * momentum x, y, z (z = 0), and 0.  Read them after synchronizing the stream;
 * a non-finite state is reported in dev_out[3], not by the return status.
 * The per-tile records live in a file-scope device array of the library
 * (8 MiB, at most 131072 tiles: the context's tiling must fit, else
 * LBM_EINVAL), one copy per GPU, held until the process ends; its device
 * address is looked up once per GPU at the first call, so call with the
 * context's device current.  Calls on one GPU share that array: calls that
 * overlap in time on one GPU (different streams or threads) race.  2-D
 * lattices with the central force stencil only (others: LBM_EINVAL);
 * LBM_ESTATE before lbm_init. */
#define LBM_NOALLOC_DOUBLES 8
lbm_status lbm_observe_noalloc(lbm_ctx* ctx, double* dev_out);

/* 3-D forms of lbm_init and lbm_observe with the third velocity component
 * (3-D lattices; on a 2-D lattice uz must be NULL and they act as
 * lbm_init / lbm_observe).  lbm_init3d takes ux, uy and uz together or none
 * of them; lbm_init on a 3-D lattice accepts only u = 0. */
lbm_status lbm_init3d(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy,
                      const double* uz, lbm_scheme scheme);
lbm_status lbm_observe3d(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz,
                         double* mu, lbm_observation* obs);

/* Copy the populations f_i (unshifted, double) to / from host
 * double[9][ny][nx] (3-D: double[q][nz][ny][nx], velocities in the order
 * rest, +x, -x, +y, -y, +z, -z, then the edges (1,1,0), (-1,-1,0), (1,-1,0),
 * (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1),
 * (0,1,-1), (0,-1,1), and on D3Q27 the corners (1,1,1), (-1,-1,-1),
 * (1,1,-1), (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1)).  Used for checkpoints and tests.  Synchronous.
 * lbm_set_populations makes the context initialised with `scheme` and sets
 * the step counter to `step`. */
lbm_status lbm_get_populations(lbm_ctx* ctx, double* f);
/* The populations of a window of a 2-D lattice, columns x0 .. x0+w-1 and
 * rows y0 .. y0+h-1 (periodic: the window may wrap past the last column or
 * row), as host double[9][h][w] in the convention of lbm_get_populations.
 * For inspecting part of a lattice too large to copy whole.  Requires
 * 0 <= x0 < nx, 0 <= y0 < ny, 1 <= w <= nx and 1 <= h <= ny, else
 * LBM_EINVAL; LBM_ESTATE before lbm_init.  Synchronous. */
lbm_status lbm_get_populations_window(lbm_ctx* ctx, int32_t x0, int32_t y0, int32_t w, int32_t h,
                                      double* f);
lbm_status lbm_set_populations(lbm_ctx* ctx, const double* f, lbm_scheme scheme, int64_t step);

/* Tile shape of the step kernel: block width in threads (64, 128, 192, 256,
 * 320 or 512; the block computes block_width output columns), output rows
 * per block (>= 4) and prefetch depth (rows of populations each thread keeps
 * in flight, 1..3).  3-D lattices (nz > 1): block width 256 or 512 threads
 * (tiles of 32 x 8 or 32 x 16 nodes), rows = z planes each block marches
 * through (>= 1), depth = planes of populations in flight (D3Q19: 1..3 with
 * 256 threads, 1..2 with 512; D3Q27: 256 threads, depth 1..2; 1 is the
 * fastest measured).  Any valid shape gives
 * bit-identical populations.
 * Depth 4 (2-D, central force stencil; block width 128 or 256, else
 * LBM_EINVAL) selects two steps per launch:
 * each launch reads and writes the populations once and advances the state
 * two steps (bit-identical to two one-step launches); blocks write strips
 * of block width - 6 columns by `rows` rows, and an odd step count ends
 * with one step of depth 3.  Graph replays (lbm_set_graph_steps) follow the
 * buffer swaps.
 * 0 keeps the current value.  A new 2-D context starts from a default
 * chosen from the lattice size (64-wide strips with short chunks up to
 * 512 columns, 256-wide strips above).  lbm_get_tile reports the shape in
 * use (any output pointer may be NULL). */
lbm_status lbm_set_tile(lbm_ctx* ctx, int32_t block_width, int32_t rows, int32_t depth);
lbm_status lbm_get_tile(const lbm_ctx* ctx, int32_t* block_width, int32_t* rows, int32_t* depth);

/* Steps per captured HIP graph for lbm_step (0 or 1 = plain launches). */
lbm_status lbm_set_graph_steps(lbm_ctx* ctx, int32_t steps);

lbm_status lbm_destroy(lbm_ctx* ctx);

const char* lbm_status_string(lbm_status s);
const char* lbm_last_error(const lbm_ctx* ctx);

/* Number of kernel launches one lbm_step(ctx, 1, .) performs (for profiling). */
int32_t lbm_kernels_per_step(const lbm_ctx* ctx);
/* Steps one step launch advances: 2 with tile depth 4 (two steps per
 * launch), else 1; 1 for a NULL ctx.  A roofline takes the launch's bytes
 * over this many steps' time. */
int32_t lbm_steps_per_launch(const lbm_ctx* ctx);

/* ------------------------------------------------------------------ batch */
/* Many independent lattices of uneven size advanced together: each step is
 * one launch per group of slots that share precision, scheme, force stencil
 * (the central one of Sec. II or the fourth-order variant discussed after
 * Eq. 23) or 3-D velocity set, block width and prefetch depth, and per lane
 * (even and odd slot index), with one block
 * per tile of those slots, reading a device-resident slot table.  Lane 0
 * runs on the batch's stream, lane 1 on a second stream of the batch that
 * forks from it and joins it again within each lbm_batch_run, so one lane's
 * next step overlaps the end of the other's.  Captured step sequences are
 * re-captured when the groups or their tile counts change.  Each slot is a complete single-instance
 * state (same kernels, same arithmetic), so a lattice gives bit-identical
 * populations alone and in a batch.  The caller owns the device arena; the
 * library places slot workspaces and the tables inside it. */

typedef enum {
  LBM_SLOT_FREE = 0,
  LBM_SLOT_ACTIVE = 1,     /* advanced by lbm_batch_run */
  LBM_SLOT_CONVERGED = 2,  /* retired: max|u| < tol */
  LBM_SLOT_CAPPED = 3,     /* retired: step cap reached */
  LBM_SLOT_DIVERGED = 4    /* retired: NaN/Inf or rho <= 0 */
} lbm_slot_status;

/* Arena bytes a slot with these parameters occupies (its workspace). */
size_t lbm_batch_slot_bytes(const lbm_params* params);

/* Bytes the batch reserves at the start of the arena for tables and
 * reduction partials, for a given arena size and slot count. */
size_t lbm_batch_overhead_bytes(size_t arena_bytes, int32_t max_slots);

/* Create a batch over a caller-owned device arena (256-byte aligned). */
lbm_status lbm_batch_create(void* dev_arena, size_t bytes, int32_t max_slots, void* hip_stream,
                            lbm_batch** out);

/* Admit a lattice (2-D with either force stencil, or 3-D: D3Q19 or D3Q27,
 * rho then double[nz][ny][nx]): allocate its workspace in the arena, set
 * f(0) = feq(rho, 0) (as lbm_init) and mark it active; every scheme of
 * lbm_scheme is accepted, and each slot steps with the scheme it was
 * admitted with.  It retires at the first lbm_batch_poll
 * that finds max|u| < tol (tol <= 0: never) or step >= step_cap (<= 0: no
 * cap), or a non-finite state.  LBM_EBUSY if no slot or arena range is free
 * (nothing changes).  Synchronous. */
lbm_status lbm_batch_admit(lbm_batch* b, const lbm_params* params, const double* rho,
                           lbm_scheme scheme, double tol, int64_t step_cap, int32_t* slot);

/* Advance every active slot by k >= 0 steps of its own scheme
 * (asynchronous).  Steps are replayed from captured HIP graphs in chunks of
 * the graph size (lbm_batch_set_graph_steps). */
lbm_status lbm_batch_run(lbm_batch* b, int32_t k_steps);

/* Observe every active slot (one batched launch per group of 2-D slots with
 * the central stencil; the three-pass observe of lbm_observe per slot for
 * 3-D slots and the fourth-order variant), retire the slots
 * that meet their criterion and write their indices to retired[0..n) (at most
 * cap).  Synchronous. */
lbm_status lbm_batch_poll(lbm_batch* b, int32_t* retired, int32_t cap, int32_t* n_retired);

/* Status and last observation of a slot (from the last poll or fetch). */
lbm_status lbm_batch_slot_info(const lbm_batch* b, int32_t slot, int32_t* status,
                               lbm_observation* obs);

/* Fields of a slot (as lbm_observe; 3-D slots: double[nz][ny][nx], the z
 * velocity through the momentum of obs only); any pointer may be NULL.
 * Synchronous. */
lbm_status lbm_batch_fetch(lbm_batch* b, int32_t slot, double* rho, double* ux, double* uy,
                           double* mu, lbm_observation* obs);

/* Populations of a slot as double[9][ny][nx] (3-D: double[q][nz][ny][nx]),
 * as lbm_get_populations. */
lbm_status lbm_batch_get_populations(lbm_batch* b, int32_t slot, double* f);

/* Tile of a slot's kernels (as lbm_set_tile; block width 64, 128 or 256 and
 * depth 1, 2 or 3 for batches; the fourth-order force stencil's slots run
 * block width 256 only; 3-D slots block 256 (32 x 8 tiles), rows = planes
 * per chunk, depth 1 or 2).  Depth 4 (2-D slots with the central stencil,
 * block 128 or 256): two steps per launch,
 * as for a single lattice; lbm_batch_run(k) then launches such a slot k / 2
 * times with two steps and, for an odd k, once with one step (depth 3), and
 * its populations equal those of one-step launches bit for bit. */
lbm_status lbm_batch_set_tile(lbm_batch* b, int32_t slot, int32_t block_width, int32_t rows,
                              int32_t depth);

/* Steps per captured graph in lbm_batch_run (even, 0 = plain launches). */
lbm_status lbm_batch_set_graph_steps(lbm_batch* b, int32_t steps);

/* Free a slot and its arena range. */
lbm_status lbm_batch_release(lbm_batch* b, int32_t slot);

lbm_status lbm_batch_destroy(lbm_batch* b);
const char* lbm_batch_last_error(const lbm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
