/*
 * mcd.h -- C ABI of the MI355X (gfx950) library for the representative-particle
 * collision step of mcdust (arXiv 2507.21239).
 *
 * The paper (Summary) states the problem this library solves: a static,
 * vertically isothermal power-law gas disk holds N representative particles
 * (Zsom & Dullemond 2008), each standing for a swarm of identical bodies;
 * particles are binned into an adaptive grid whose cells hold equal numbers
 * of representative particles; inside each cell particles collide with the
 * outcomes sticking, fragmentation and erosion; particles are transported
 * radially and vertically.  The Benchmark section's table fixes the disk:
 * Sigma_g(1 AU) = 1000 g/cm^2, T(1 AU) = 280 K, alpha = 1e-3, v_frag = 10 m/s,
 * erosion mass ratio 10, p = 1, q = 0.5.
 *
 * Conventions
 *  - CGS units.  All particle arrays are DEVICE pointers owned by the caller
 *    (allocate them with hipMalloc or as torch tensors); the library keeps
 *    non-owning views and never frees them.  They must outlive the context.
 *  - All device work is enqueued on the caller's HIP stream given to
 *    mcd_init; functions marked "async" return before the work completes.
 *  - Device memory beyond the particles is the caller's too: one workspace
 *    of mcd_workspace_size bytes (e.g. a torch uint8 tensor), given to
 *    mcd_init, holds the grid, the binning buffers, the cell lists of the
 *    batched schedule, the device counters, the tuning backups and the
 *    histogram edges.  mcd_init, mcd_bin, mcd_rates, mcd_row_sums, mcd_step,
 *    mcd_tune, mcd_set_schedule and mcd_sigma_hist allocate no device
 *    memory.  The two optional features whose size only their own call
 *    fixes allocate at that call and free in mcd_free: the gas grid's nodes
 *    (mcd_set_gas_grid) and the snapshot staging (mcd_snapshot, first call
 *    or a larger field set).
 *  - Largest cell: 2048 particles in the mixed form, 1536 in FP64 (a
 *    four-wave team's particle records must fit the 160 KB of LDS); larger
 *    cells are rejected with MCD_EINVAL.
 *  - Every function returns an mcd_status; no C++ exception crosses the ABI.
 *    After an error, mcd_last_error(ctx) describes it.  Kernels that detect
 *    an anomaly (a NaN or infinite rate, a non-positive mass or volume) set a
 *    sticky device flag that the next syncing call reports as MCD_EDEVICE.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef MCD_H
#define MCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCD_OK = 0,
  MCD_EINVAL = -1,   /* invalid argument; nothing was enqueued */
  MCD_ENOMEM = -2,   /* device allocation failed */
  MCD_EHIP = -3,     /* a HIP runtime call failed */
  MCD_ESTATE = -4,   /* call out of order (e.g. mcd_step before mcd_bin) */
  MCD_EDEVICE = -5   /* a kernel set the sticky anomaly flag */
} mcd_status;

/* collision kernels */
#define MCD_K_PHYSICAL 0 /* geometric cross-section x relative velocity */
#define MCD_K_CONSTANT 1 /* K = k0 (Smoluchowski test kernel) */
#define MCD_K_LINEAR 2   /* K = k0 (m_i + m_j) (Smoluchowski test kernel) */

/* flags: relative-velocity sources added in quadrature (bits 0-4),
 * transport processes (bits 8-11), collisions on (bit 12) */
#define MCD_DV_BROWNIAN (1u << 0)
#define MCD_DV_TURB (1u << 1)
#define MCD_DV_RADIAL (1u << 2)
#define MCD_DV_AZIMUTHAL (1u << 3)
#define MCD_DV_SETTLING (1u << 4)
#define MCD_TR_DRIFT (1u << 8)
#define MCD_TR_SETTLE (1u << 9)
#define MCD_TR_MIX_R (1u << 10)
#define MCD_TR_MIX_Z (1u << 11)
#define MCD_COAG (1u << 12)

/* arithmetic of the rate matrix */
#define MCD_FP64 0  /* rates, sums and masses in FP64 */
#define MCD_MIXED 1 /* pair rates in FP32 (per-cell power-of-two scale);
                       masses, prefix sums, row-sum state and time in FP64 */

/* cell schedule of the collision kernel */
#define MCD_SCHED_PLAIN 0   /* one four-wave workgroup per cell, launched per step */
#define MCD_SCHED_BATCHED 1 /* one persistent launch: big cells largest-first on
                               four-wave teams, small cells on single waves;
                               multi-step loops replayed from a HIP graph */

/* fragmentation criterion of a collision at relative velocity dv (outcome
 * variants of the literature the paper cites for its collision physics):
 * SHARP fragments iff dv >= v_frag; RAMP with probability rising linearly
 * from 0 at (1 - w) v_frag to 1 at v_frag; MAXWELL with the probability that
 * a Maxwellian collision speed of mean dv exceeds v_frag,
 * erfc(x) + 2/sqrt(pi) x exp(-x^2), x = 2 v_frag / (sqrt(pi) dv).  RAMP and
 * MAXWELL draw their uniform from Philox counter (event, cell, step, 3). */
#define MCD_FRAG_SHARP 0
#define MCD_FRAG_RAMP 1
#define MCD_FRAG_MAXWELL 2

/* outcome codes (event log and statistics) */
#define MCD_OUT_STICK 0
#define MCD_OUT_ERODE 1        /* i is the larger body and loses mass */
#define MCD_OUT_ERODED_SMALL 2 /* i is the small projectile: fragment draw up to m_i */
#define MCD_OUT_FRAG 3

#define MCD_GAS_FIELDS 6 /* per-cell gas record: V, rho_g, T, alpha, r_c, zeta = z_c/H */
#define MCD_GEOM_FIELDS 5 /* per-cell geometry: r_lo, r_hi, z_lo, z_hi, V */
#define MCD_MAX_COMP 8

typedef struct {
  double sigma_g0;      /* gas surface density at r_ref [g cm^-2] */
  double T0;            /* temperature at r_ref [K] */
  double p, q;          /* Sigma_g ~ r^-p, T ~ r^-q */
  double alpha;         /* turbulence strength (adaptive grid) */
  double v_frag;        /* fragmentation velocity [cm/s] */
  double erosion_ratio; /* mass ratio at and above which a fast collision erodes */
  double a_mono;        /* monomer radius [cm]; smallest mass m0 = 4/3 pi a_mono^3 rho_s */
  double rho_s;         /* material density [g cm^-3] */
  double mu;            /* mean molecular weight */
  double m_star;        /* stellar mass [g] */
  double r_ref;         /* reference radius of the power laws [cm] */
  double dm_max;        /* grouping threshold: r_ij is divided by max(1, dm_max m_i/m_j) and
                           a collision moves that many bodies of swarm j (0 = off) */
  double erosion_chi;   /* eroded mass in units of the (grouped) impactor mass */
  double r_in;          /* inner removal radius [cm] (disk mode) */
  double r_col;         /* column radius [cm] (column mode) */
  double k0;            /* coefficient of the test kernels */
  int32_t kernel;       /* MCD_K_* */
  int32_t n_r, n_z;     /* adaptive grid: radial zones x cells per zone */
  int32_t column;       /* 1 = one column at r_col; swarm masses per unit area */
  uint32_t flags;       /* MCD_DV_* | MCD_TR_* | MCD_COAG */
  int32_t n_comp;       /* composition fractions per particle, 0..MCD_MAX_COMP */
  uint64_t seed;        /* Philox4x32-10 key (low word, high word) */
  int32_t precision;    /* MCD_FP64 | MCD_MIXED */
  int32_t schedule;     /* MCD_SCHED_PLAIN | MCD_SCHED_BATCHED */
  int32_t frag_mode;    /* MCD_FRAG_*: how the relative velocity decides fragmentation */
  int32_t max_cells;    /* most cells of an explicit grid this context will bin
                           (0 = n_r * n_z); sizes the workspace's cell lists */
  double frag_width;    /* MCD_FRAG_RAMP: relative width w of the ramp, 0 < w <= 1 */
} mcd_params;

typedef struct {
  int64_t n;            /* number of particles N; particle id = array index */
  double *r;            /* [N] radius [cm]                      (read/write) */
  double *z;            /* [N] height above the midplane, >= 0  (read/write) */
  double *m;            /* [N] representative-particle mass [g] (read/write) */
  const double *M;      /* [N] swarm mass [g]; never written    (read) */
  uint8_t *active;      /* [N] 1 = in the grid                  (read/write) */
  float *comp;          /* [n_comp][N] composition fractions, component-major, or NULL */
} mcd_particles;

typedef struct {
  int32_t n_cells;
  int32_t max_cell;          /* upper bound on any cell's particle count (<= 2048), or 0:
                                the library measures the sizes (one synchronisation) */
  const int32_t *cell_start; /* [n_cells + 1] device; member ranges into order */
  const int32_t *order;      /* [cell_start[n_cells]] device; particle indices, each cell's
                                members in the order that defines cumulative rates */
  const double *gas;         /* [n_cells][MCD_GAS_FIELDS] device */
} mcd_cells;

typedef struct {
  int64_t events;           /* collisions performed since mcd_init */
  int64_t outcomes[4];      /* by MCD_OUT_* */
  int64_t steps;            /* global steps completed */
  int64_t n_active;         /* active particles after the last binning */
  double t_sim;             /* simulated time [s] */
  uint32_t device_flags;    /* sticky anomaly bits (0 = none) */
  int32_t n_cells;          /* cells of the current grid */
  int32_t max_cell;         /* largest cell of the current grid */
  int32_t pad;
} mcd_stats;

typedef struct mcd_ctx mcd_ctx;

/* Bytes of device workspace a context needs for n particles (the paper,
 * Summary: N representative particles in an adaptive grid of n_r x n_z
 * equal-count cells, or explicit cells up to params->max_cells): the grid,
 * the binning buffers, the batched schedule's cell lists, the device
 * counters, the tuning backups and 2^16 histogram edges.  About 70 bytes per
 * particle plus 12 per cell (more when a radial zone can exceed 8192
 * particles).  MCD_EINVAL on bad params or n outside [1, 2^31). */
mcd_status mcd_workspace_size(const mcd_params *params, int64_t n, size_t *bytes);

/* Create a context for the paper's problem (Summary): the static power-law
 * disk and collision physics of params over the caller's N representative
 * particles.  Validates params (MCD_EINVAL on NaN, non-positive physical
 * constants, n_comp out of range, comp == NULL with n_comp > 0) and the
 * workspace (MCD_EINVAL if NULL or smaller than mcd_workspace_size), records
 * the particle views, the stream (a hipStream_t; NULL = the null stream) and
 * the workspace (device memory owned by the caller, which must outlive the
 * context; the library never frees it), and enqueues the clearing of the
 * device counters.  Allocates no device memory.  *out is set only on MCD_OK. */
mcd_status mcd_init(const mcd_params *params, const mcd_particles *particles, void *hip_stream,
                    void *workspace, size_t ws_bytes, mcd_ctx **out);

/* Bin particles into cells (paper, Summary: adaptive grid of equal-count
 * cells).  explicit_or_null == NULL: adaptive binning of the active
 * particles into n_r radial zones of equal count by rank of (r, index), each
 * split into n_z cells of equal count by rank of (z, index), with the floor
 * rule for uneven counts; members of a cell are listed by ascending (z,
 * index); gas state at the cell centre from the power-law disk.  Async;
 * MCD_EINVAL if n_r * n_z exceeds N or a cell could exceed the largest cell.
 * Otherwise the caller's explicit cells: the library keeps non-owning views
 * of cell_start, order and gas, which must stay valid and unchanged while
 * this grid is in use (until the next mcd_bin or mcd_free), and plans the
 * batched schedule on the device without copying to the host.  With
 * max_cell > 0 the call is async and the grid is validated on the device:
 * a grid whose cell_start starts below 0 or decreases, a cell above
 * max_cell or a member index outside [0, N) is not collided and the next
 * syncing call (mcd_get_stats) returns MCD_EDEVICE.  With max_cell == 0
 * the call synchronises once to measure the cells and returns MCD_EINVAL
 * for such a grid.  MCD_EINVAL also if n_cells exceeds the workspace's
 * cells (params->max_cells) or max_cell exceeds the largest cell. */
mcd_status mcd_bin(mcd_ctx *ctx, const mcd_cells *explicit_or_null);

/* Rate matrix of one cell (test path; the swarm rates of Zsom & Dullemond
 * 2008, which the paper's Summary adopts): r_out[i*ld + j] = r_ij, the rate at
 * which representative particle i collides with a body of swarm j, computed
 * by the same pair code as the collision kernel in the context's precision
 * and returned as FP64 (device pointer, n_c x n_c with leading dimension ld
 * >= n_c); rowsum_out[i] = sum_j r_ij in canonical order j = 0..n_c-1
 * (device, may be NULL).  In FP64 these are the collision kernel's starting
 * row sums; the FP32 form's kernel adds the same terms in another order
 * (each unordered pair once), equal up to FP32 rounding.  Synchronises.
 * MCD_EINVAL if cell is out of range. */
mcd_status mcd_rates(mcd_ctx *ctx, int32_t cell, double *r_out, int64_t ld, double *rowsum_out);

/* Starting row sums r_i = sum_j r_ij of every cell (the Zsom & Dullemond
 * rate of representative particle i, paper Summary), exactly as the
 * collision launch of the context's precision and schedule builds them
 * before its first event -- in the mixed form the FP32 build that adds each
 * unordered pair once -- divided by the cell's rate scale.  out [n of the
 * grid's members] is a device FP64 array indexed like the grid's order
 * (out[cell_start[c] + k] belongs to member k of cell c).  No event runs and
 * no particle changes.  Async; test path.  MCD_ESTATE before mcd_bin. */
mcd_status mcd_row_sums(mcd_ctx *ctx, double *out);

/* Advance n_steps global steps of length dt [s] (the paper, Summary: bin
 * into the adaptive grid, collide inside every cell, transport radially and
 * vertically): (re)bin when the grid is adaptive, collide every cell,
 * transport.  Allocates nothing.  Inside a cell, events run until
 * the next waiting time would pass dt (dt > 0) and/or max_events_per_cell
 * events are done (> 0); at least one limit must be set.  Async.  With the
 * batched schedule and n_steps > 1 one step is captured as a HIP graph
 * (again after mcd_bin with explicit cells, mcd_tune, mcd_set_schedule or a
 * change of dt or max_events) and replayed n_steps times; otherwise each
 * step's kernels are launched directly. */
mcd_status mcd_step(mcd_ctx *ctx, double dt, int64_t max_events_per_cell, int32_t n_steps);

/* Schedule of the batched collision launch (one persistent launch over all
 * cells, largest cells first): which team shape processes a cell and how
 * many workgroups run at once.  Results depend on it only through the
 * rounding order of the FP64 prefix scans, which follows the team layout. */
typedef struct {
  int32_t small_max;   /* cells of up to small_max particles run on one
                          wavefront, larger ones on teams of four (0..512) */
  int32_t grid_per_cu; /* persistent workgroups per compute unit; 0 = as many
                          as the kernel's registers and LDS allow */
  int32_t trials;      /* configurations timed by mcd_tune */
  int32_t pad;
  double ms_best;      /* collision-launch time of the chosen schedule [ms] */
  double ms_default;   /* ... of the schedule in force before tuning [ms] */
} mcd_tune_result;

/* Autotuner of the batched schedule on the current cells: times one
 * collision launch (dt, max_events_per_cell as in mcd_step) for each
 * single-wave threshold in {0, 64, 128, 192, 256, 384, 512} that gives a
 * distinct, fitting plan, then 1 and 2 workgroups per compute unit at the
 * best threshold, and keeps the fastest.  Masses, compositions and counters
 * are restored after every trial (the step counter does not advance; no
 * event log is written).  Synchronises; MCD_EINVAL for the plain schedule,
 * MCD_ESTATE before mcd_bin. */
mcd_status mcd_tune(mcd_ctx *ctx, double dt, int64_t max_events_per_cell, mcd_tune_result *out);

/* Set the batched schedule directly (e.g. a stored tuning result).
 * MCD_EINVAL if out of range or if the plan does not fit the GPU's LDS (the
 * previous schedule is kept). */
mcd_status mcd_set_schedule(mcd_ctx *ctx, int32_t small_max, int32_t grid_per_cu);

/* Gridded gas in place of the power-law disk (post-processing a
 * hydrodynamic state, the paper's Statement of Need).  Host arrays:
 * r_nodes [n_gr] (> 0, increasing), z_nodes [n_gz] (heights above the
 * midplane, >= 0, increasing), rho, T, alpha [n_gr][n_gz] (radius-major,
 * positive), copied before the call returns.  Gas at (r, z): bilinear
 * interpolation in (ln r, z) of ln rho_g, ln T and ln alpha, clamped to the
 * boundary nodes outside; c_s from T, Omega from the star, H = c_s / Omega;
 * eta v_K = c_s^2 s / (2 Omega r) with s = -d ln(rho_g T) / d ln r of the
 * interpolant at (r, z); radial diffusion drifts by D c / r with
 * c = d ln(Sigma_g alpha T) / d ln r + 5/2, Sigma_g(r_k) = 2 (z_0 rho(z_0) +
 * trapezoids over the nodes).  Binning (cell gas), the rate matrix (eta v_K
 * of explicit and adaptive cells) and transport use it from the next call
 * on.  r_nodes == NULL restores the power-law disk.  Synchronises; MCD_EINVAL
 * on bad nodes or values. */
mcd_status mcd_set_gas_grid(mcd_ctx *ctx, const double *r_nodes, int32_t n_gr,
                            const double *z_nodes, int32_t n_gz, const double *rho,
                            const double *T, const double *alpha);

/* sigma_d(m, r): dust surface density per particle-mass bin and radius of
 * the current particles (paper, Benchmark: the run's output is the dust
 * surface density as a function of particle mass and distance from the
 * star).
 * r_edges [n_rb+1], m_edges [n_mb+1]: host arrays, finite and strictly
 * increasing (r_edges[0] >= 0), copied before the call returns.
 * sigma [n_rb*n_mb]: device FP64, radius-major; bin (k, l) holds the swarm
 * masses M of the active particles with r_edges[k] <= r < r_edges[k+1] and
 * m_edges[l] <= m < m_edges[l+1], divided by the annulus area
 * pi (r_edges[k+1]^2 - r_edges[k]^2) (area 1 in column mode, where M is per
 * unit area): g/cm^2 per mass bin.  count [n_rb*n_mb]: device uint32, the
 * representative particles per bin, or NULL.  The edges go to the
 * workspace (at most 2^16 in all); the call synchronises the stream first
 * (no earlier upload still reads the host copy), then runs async.
 * The FP64 sums follow the order of device atomics (results may differ by
 * a relative count * 2^-52 between runs).  MCD_EINVAL on bad edges or
 * n_rb * n_mb outside [1, 2^24]. */
mcd_status mcd_sigma_hist(mcd_ctx *ctx, const double *r_edges, int32_t n_rb, const double *m_edges,
                          int32_t n_mb, double *sigma, uint32_t *count);

/* Particle histories (the paper's Statement of Need: a Lagrangian method
 * follows the histories of its particles and their compositions).  A
 * snapshot is the state of the chosen fields at its place in the context
 * stream: their device copy is queued there (so it sees every step queued
 * before, and no later one), and the copy to host_dst runs on a separate
 * stream while later steps proceed.  host_dst must stay valid until
 * mcd_snapshot_wait returns; pinned host memory (hipHostMalloc) makes the
 * transfer asynchronous.  Layout: the chosen fields in the order r, z, m
 * (FP64 [N] each), active (uint8 [N]), comp (FP32 [n_comp][N]), each padded
 * to a multiple of 16 bytes (mcd_snapshot_bytes gives the total).  Two
 * snapshots can be in flight; a third waits, in stream order, for the
 * oldest transfer.  *ticket (may be NULL) numbers the snapshot for
 * mcd_snapshot_wait. */
#define MCD_SNAP_R 1u
#define MCD_SNAP_Z 2u
#define MCD_SNAP_M 4u
#define MCD_SNAP_ACTIVE 8u
#define MCD_SNAP_COMP 16u
#define MCD_SNAP_ALL 31u
mcd_status mcd_snapshot_bytes(mcd_ctx *ctx, uint32_t fields, size_t *bytes);
mcd_status mcd_snapshot(mcd_ctx *ctx, uint32_t fields, void *host_dst, size_t bytes,
                        int64_t *ticket);
/* Block until the snapshot with this ticket is in host memory. */
mcd_status mcd_snapshot_wait(mcd_ctx *ctx, int64_t ticket);

/* Copy the counters to the host (synchronises): collisions by outcome (the
 * paper, Summary: sticking, erosion and fragmentation), steps, simulated
 * time, active particles, the grid's cells and largest cell; report the
 * sticky device flag as MCD_EDEVICE (mcd_last_error names its cause). */
mcd_status mcd_get_stats(mcd_ctx *ctx, mcd_stats *host_out);

/* Copy the current grid into caller device buffers (any may be NULL):
 * cell_start [n_cells+1] int32, order [n_active] int32, geom
 * [n_cells][MCD_GEOM_FIELDS] double (adaptive grids only), gas
 * [n_cells][MCD_GAS_FIELDS] double.  Synchronises. */
mcd_status mcd_get_cells(mcd_ctx *ctx, int32_t *cell_start, int32_t *order, double *geom,
                         double *gas);

/* Record the first per_cell events of every cell in the following steps:
 * device buffer of n_cells * per_cell records of four int32 (i, j, outcome,
 * 0), cell-local indices.  buf == NULL disables logging. */
mcd_status mcd_set_event_log(mcd_ctx *ctx, int32_t *buf, int64_t per_cell);

/* Philox4x32-10 (Salmon et al., SC'11) on the device, for tests: out[4k..4k+3]
 * = Philox(ctr[4k..4k+3], key).  ctr and out are device arrays of 4n uint32.
 * Async on hip_stream. */
mcd_status mcd_philox(const uint32_t *ctr, uint32_t key_lo, uint32_t key_hi, uint32_t *out,
                      int64_t n, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * collision step over explicit cells without a context or a workspace --
 * what mcd_init, mcd_bin(cells) and mcd_step(dt, max_events, 1) do on a
 * fresh context of the same params whose step counter is `step` (the
 * Philox counter word of the step), with the same kernels and schedule.
 * The device counters, the plan and the batched cell lists live in a
 * library-internal device array of MCD_NOALLOC_SCRATCH_BYTES (about 8 MB),
 * of which every GPU the library runs on holds one copy until the process
 * ends; it is cleared by a kernel at every call.  Calls that overlap on one
 * GPU (other streams, other host threads) race on it: serialise them.
 * cells->max_cell must bound the cells (1..2048; grids are validated on the
 * device as in mcd_bin, and a rejected grid collides nothing);
 * cells->n_cells must be at most 2^20.  m (and comp) change in place.
 * counts (device int64[6], may be NULL) receives the events, the outcome
 * counts by MCD_OUT_* and the device anomaly flags of this call.  Async on
 * hip_stream; allocates nothing and calls no allocating routine.
 * MCD_EINVAL for bad params, particles, cells or limits (reason in
 * mcd_last_error(NULL) on this thread). */
#define MCD_NOALLOC_SCRATCH_BYTES 8406016
mcd_status mcd_collide_noalloc(const mcd_params *params, const mcd_particles *particles,
                               const mcd_cells *cells, double dt, int64_t max_events,
                               uint32_t step, void *hip_stream, int64_t *counts);

/* Human-readable description of the last error of ctx (never NULL); with
 * ctx == NULL, of the last failed mcd_collide_noalloc on this thread, or
 * "null context". */
const char *mcd_last_error(const mcd_ctx *ctx);

/* Release the workspace and the context (synchronises the stream first). */
void mcd_free(mcd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
