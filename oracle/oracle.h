/*
 * oracle.h -- plain FP64 CPU oracle of the representative-particle collision
 * step (mcdust, arXiv 2507.21239, "Summary": Zsom & Dullemond representative
 * particles, equal-count adaptive grid, sticking / fragmentation / erosion,
 * vertical and radial transport, static vertically isothermal power-law disk).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against a slow, obviously correct implementation.  The GPU product never
 * links, loads or calls it, and it shares no code with the GPU library.
 *
 * Conventions: CGS units, FP64 everywhere except the composition fractions
 * (FP32 storage, FP64 arithmetic).  The paper gives no formulas (it defers to
 * Drazkowska et al. 2013); every formula below is a stated reading of the
 * literature the paper cites, listed with its justification in the design
 * notes of the repository.  Functions whose result has no independent pin
 * say "parity unpinned" in oracle.c.
 */
#ifndef MCD_ORACLE_H
#define MCD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* pair kernels */
#define ORC_K_PHYSICAL 0
#define ORC_K_CONSTANT 1
#define ORC_K_LINEAR 2

/* flags: relative-velocity sources (bits 0-4), transport (8-11), collisions (12) */
#define ORC_DV_BROWNIAN (1u << 0)
#define ORC_DV_TURB (1u << 1)
#define ORC_DV_RADIAL (1u << 2)
#define ORC_DV_AZIMUTHAL (1u << 3)
#define ORC_DV_SETTLING (1u << 4)
#define ORC_TR_DRIFT (1u << 8)
#define ORC_TR_SETTLE (1u << 9)
#define ORC_TR_MIX_R (1u << 10)
#define ORC_TR_MIX_Z (1u << 11)
#define ORC_COAG (1u << 12)

/* fragmentation criterion (outcome variants of the cited literature) */
#define ORC_FRAG_SHARP 0     /* fragment iff dv >= v_frag */
#define ORC_FRAG_RAMP 1      /* probability rising linearly over [(1 - w) v_frag, v_frag] */
#define ORC_FRAG_MAXWELL 2   /* collision speeds Maxwellian with mean dv: P(speed >= v_frag) */

/* outcome codes written to the event log */
#define ORC_OUT_STICK 0
#define ORC_OUT_ERODE 1      /* i is the larger body and loses mass */
#define ORC_OUT_ERODED_SMALL 2 /* i is the small projectile: fragment draw up to m_i */
#define ORC_OUT_FRAG 3

/* gridded gas (post-processing of hydrodynamic output, the paper's
 * Statement of Need): node values on n_r radii x n_z heights, stored as
 * logarithms; orc_grid_fill builds it from plain node values */
typedef struct {
  int32_t n_r, n_z;
  const double *lr;    /* [n_r] ln r of the radial nodes (increasing) */
  const double *zn;    /* [n_z] heights of the vertical nodes (>= 0, increasing) */
  const double *lrho;  /* [n_r*n_z] ln rho_g, radius-major */
  const double *lT;    /* [n_r*n_z] ln T */
  const double *lA;    /* [n_r*n_z] ln alpha */
  const double *lS;    /* [n_r] ln Sigma_g: twice the trapezoid integral of rho_g over the
                          nodes' heights plus z_0 rho_g(z_0) below the first node */
} orc_gas_grid;

typedef struct {
  double sigma_g0;      /* gas surface density at r_ref [g cm^-2] */
  double T0;            /* temperature at r_ref [K] */
  double p, q;          /* Sigma_g ~ r^-p, T ~ r^-q */
  double alpha;         /* turbulence strength */
  double v_frag;        /* fragmentation velocity [cm/s] */
  double erosion_ratio; /* mass ratio at and above which a fast collision erodes */
  double a_mono;        /* monomer radius [cm]; m0 = 4/3 pi a_mono^3 rho_s */
  double rho_s;         /* material density [g cm^-3] */
  double mu;            /* mean molecular weight */
  double m_star;        /* stellar mass [g] */
  double r_ref;         /* reference radius of the power laws [cm] */
  double dm_max;        /* grouping threshold (0 = no grouping) */
  double erosion_chi;   /* eroded mass in units of the impactor mass */
  double r_in;          /* inner removal radius [cm] (disk mode) */
  double r_col;         /* column radius [cm] (column mode) */
  double k0;            /* constant / linear test-kernel coefficient */
  int32_t kernel;       /* ORC_K_* */
  int32_t n_r, n_z;     /* adaptive grid */
  int32_t column;       /* 1 = single column at r_col, masses per unit area */
  uint32_t flags;       /* ORC_DV_* | ORC_TR_* | ORC_COAG */
  int32_t n_comp;       /* composition fractions per particle (0..8) */
  uint64_t seed;        /* Philox key */
  int32_t frag_mode;    /* ORC_FRAG_*: how the relative velocity decides fragmentation */
  int32_t pad_;
  double frag_width;    /* ORC_FRAG_RAMP: relative width of the ramp below v_frag */
  const orc_gas_grid *grid; /* gridded gas, or NULL for the power-law disk */
} orc_params;

/* gas at one point: density, temperature, turbulence, sound speed, Kepler
 * frequency, scale height, the pressure slope s = -d ln P / d ln r (so that
 * eta v_K = c_s^2 s / (2 Omega r)), and the radial-diffusion correction
 * factor c, such that the random walk drifts by D c / r (the logarithmic
 * r-derivative of Sigma_g alpha c_s H) */
typedef struct {
  double rho_g, T, alpha, cs, Omega, H, slopeP, corr;
} orc_local_gas;

/* per-cell gas record, six primaries: V, rho_g, T, alpha, r_c, zeta (= z_c/H) */
#define ORC_GAS_FIELDS 6

typedef struct {
  double V, rho_g, T, alpha, r_c, zeta;            /* primaries */
  double cs, Omega, H, z_c, eta_vK, v_th, lambda, nu, Re, St_eta, Vg2; /* derived */
} orc_gas;

typedef struct {
  double m, M;                 /* rp mass, swarm mass */
  double a, t_s, St;           /* radius, stopping time, Stokes number */
  double v_r, v_phi, v_z;      /* drift, azimuthal and settling velocity */
  double n;                    /* swarm number density M/(m V) */
} orc_particle;

typedef struct {
  int32_t i, j, outcome, pad;  /* cell-local indices in canonical order */
} orc_event;

typedef struct {
  int64_t events;
  int64_t outcomes[4];
  double t_end;                /* simulated time used inside the cell */
  double drift;                /* max |r_i(incremental) - r_i(fresh)| / R at the end */
} orc_cell_stats;

/* --- building blocks (exported for pin tests) --- */
void orc_grid_fill(int32_t n_r, int32_t n_z, const double *r_nodes, const double *z_nodes,
                   const double *rho, const double *T, const double *alpha, double *lr, double *zn,
                   double *lrho, double *lT, double *lA, double *lS);
void orc_local_gas_at(const orc_params *P, double r, double z, orc_local_gas *o);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t lo, uint32_t hi);
void orc_gas_derive(const orc_params *P, const double prim[ORC_GAS_FIELDS], orc_gas *g);
void orc_disk_local(const orc_params *P, double r, double z, double *Sigma_g, double *T,
                    double *cs, double *Omega, double *H, double *rho_g);
void orc_particle_props(const orc_params *P, const orc_gas *g, double m, double M,
                        orc_particle *out);
double orc_dv2_turb(const orc_gas *g, double St_a, double St_b);
double orc_rel_velocity(const orc_params *P, const orc_gas *g, const orc_particle *pi,
                        const orc_particle *pj);
double orc_pair_kernel(const orc_params *P, const orc_gas *g, const orc_particle *pi,
                       const orc_particle *pj);
double orc_rate(const orc_params *P, const orc_gas *g, const orc_particle *pi,
                const orc_particle *pj);
double orc_frag_draw(double lo, double hi, double u);
/* probability that a collision at mean relative velocity dv fragments
 * (or erodes), by P->frag_mode */
double orc_frag_probability(const orc_params *P, double dv);
int32_t orc_select(const double *v, int32_t n, double target);
int32_t orc_outcome(const orc_params *P, double dv, double mi, double mj, double u, double uf,
                    double *m_new);

/* --- the method --- */
/* n x n rate matrix of one cell (row = representative particle i) and row sums */
void orc_cell_rates(const orc_params *P, const double prim[ORC_GAS_FIELDS], int32_t n,
                    const int32_t *members, const double *m, const double *M,
                    double *r_out, double *rowsum_out);

/* equal-count binning of the active particles into n_r x n_z cells.
 * outputs: cell_start[n_r*n_z+1], order[n_active], geom[n_cells*5]
 * (r_lo, r_hi, z_lo, z_hi, V), gas[n_cells*ORC_GAS_FIELDS]; returns n_active */
int64_t orc_bin(const orc_params *P, int64_t N, const double *r, const double *z,
                const uint8_t *active, int32_t *cell_start, int32_t *order, double *geom,
                double *gas);

/* collision Monte Carlo inside one cell (members in canonical order).
 * m and comp are global arrays updated in place. */
int64_t orc_collide_cell(const orc_params *P, const double prim[ORC_GAS_FIELDS],
                         int32_t cell_id, uint32_t step, int32_t n, const int32_t *members,
                         double *m, const double *M, float *comp, int64_t N, double dt,
                         int64_t max_events, orc_event *evlog, int64_t log_cap,
                         orc_cell_stats *st);

/* transport of every active particle over dt (disk or column mode) */
void orc_transport(const orc_params *P, int64_t N, double *r, double *z, const double *m,
                   uint8_t *active, uint32_t step, double dt);

/* sigma_d(m, r), the dust surface density per mass bin (paper, Benchmark:
 * the run's output is the dust surface density as a function of particle mass
 * and distance from the star).  Bins are half-open, r_edges[k] <= r <
 * r_edges[k+1] and m_edges[l] <= m < m_edges[l+1], edges strictly
 * increasing.  For every active particle in range, its swarm mass M is added
 * to bin (k, l) in particle order; then each bin is divided by its annulus
 * area pi (r_edges[k+1]^2 - r_edges[k]^2) (area 1 in column mode, where M is
 * already per unit area).  sigma[k*n_mb + l] in g/cm^2 per mass bin, count[]
 * the number of representative particles (count may be NULL).  Returns the
 * number of particles counted. */
int64_t orc_sigma_hist(int64_t N, const double *r, const double *m, const double *M,
                       const uint8_t *active, const double *r_edges, int32_t n_rb,
                       const double *m_edges, int32_t n_mb, int32_t column, double *sigma,
                       uint32_t *count);

/* all cells of one step: collide every cell (threads over cells).
 * log may be NULL; otherwise cell c writes log[c*log_per_cell ...] */
void orc_collide_all(const orc_params *P, int32_t n_cells, const int32_t *cell_start,
                     const int32_t *order, const double *gas, uint32_t step, double *m,
                     const double *M, float *comp, int64_t N, double dt, int64_t max_events,
                     orc_event *evlog, int64_t log_per_cell, orc_cell_stats *stats,
                     int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
