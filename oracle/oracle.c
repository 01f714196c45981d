/*
 * oracle.c -- plain FP64 CPU oracle of the representative-particle collision
 * step.  TEST INFRASTRUCTURE ONLY (see oracle.h): the GPU library never links
 * or calls this file, and the two share no code.
 *
 * What the paper fixes (arXiv 2507.21239, Summary): representative particles
 * after Zsom & Dullemond (2008); particles are binned into an adaptive grid of
 * cells holding equal numbers of representative particles, and collide inside
 * their cell; outcomes are sticking, fragmentation and erosion (a small body
 * chips part of a large one); transport is radial and vertical; the gas disk
 * is a static power law, vertically isothermal.  Benchmark table: Sigma_g(1 AU)
 * = 1000 g/cm^2, T(1 AU) = 280 K, alpha = 1e-3, v_frag = 10 m/s, erosion mass
 * ratio 10, p = 1, q = 0.5.  Everything else (the formulas) is a reading of
 * the literature the paper cites; each reading is named where it is used.
 *
 * Pins (tests/): Philox known-answer vectors; the constant- and linear-kernel
 * Smoluchowski solutions; swarm-mass conservation; closed forms of every
 * relative-velocity source; the midplane Epstein identity; drag-law
 * continuity; whole rate matrices of small cells at 50 digits from the
 * physical definitions in other arrangements; selection frequencies against
 * brute-force probabilities; waiting-time and fragment-mass distributions;
 * the null events left by rounding residue; composition mixing in
 * hand-worked collisions and in whole monomers; binning against a library
 * sort; the settling-mixing equilibrium; the planar diffusion law of the
 * radial walk and radially well-mixed tracers.  Parity unpinned: the
 * physical configurations against mcdust itself (no code or output data
 * exists).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).  Summation is
 * plain left-to-right; no blocking or reordering.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* physical constants, CGS (CODATA 2018 / IAU values) */
static const double KB = 1.380649e-16;      /* erg/K */
static const double MH = 1.6735575e-24;     /* g, hydrogen atom */
static const double GRAV = 6.67430e-8;      /* cm^3 g^-1 s^-2 */
static const double SIGMA_H2 = 2e-15;       /* cm^2, H2 collision cross-section */
static const double PI = 3.14159265358979323846;
static const double YA = 1.6;               /* Ormel & Cuzzi (2007) y*_a */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two     */
/* 32x32->64 multiplies and xors, with the Weyl key schedule.                */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* two 32-bit words -> a double strictly inside (0,1): the top 52 bits of
 * the 64-bit word w = hi:lo, offset by half a step (exact in FP64) */
double orc_u01(uint32_t lo, uint32_t hi) {
  uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

static void orc_uniforms(const orc_params *P, uint32_t c0, uint32_t c1, uint32_t c2,
                         uint32_t c3, double *ua, double *ub) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  *ua = orc_u01(x[0], x[1]);
  *ub = orc_u01(x[2], x[3]);
}

/* ------------------------------------------------------------------------ */
/* Gas: static power-law disk, vertically isothermal (paper, Summary and    */
/* Benchmark table).  Sound speed, Kepler frequency, scale height and the   */
/* Gaussian vertical profile are the standard thin-disk forms.              */
/* ------------------------------------------------------------------------ */
void orc_disk_local(const orc_params *P, double r, double z, double *Sigma_g, double *T,
                    double *cs, double *Omega, double *H, double *rho_g) {
  double x = r / P->r_ref;
  *Sigma_g = P->sigma_g0 * pow(x, -P->p);
  *T = P->T0 * pow(x, -P->q);
  *cs = sqrt(KB * (*T) / (P->mu * MH));
  *Omega = sqrt(GRAV * P->m_star / (r * r * r));
  *H = (*cs) / (*Omega);
  *rho_g = (*Sigma_g) / (sqrt(2.0 * PI) * (*H)) * exp(-(z * z) / (2.0 * (*H) * (*H)));
}

/* ------------------------------------------------------------------------
 * gas at a point: the power-law disk, or the gridded gas
 * ------------------------------------------------------------------------ */
void orc_grid_fill(int32_t n_r, int32_t n_z, const double *r_nodes, const double *z_nodes,
                   const double *rho, const double *T, const double *alpha, double *lr, double *zn,
                   double *lrho, double *lT, double *lA, double *lS) {
  for (int32_t k = 0; k < n_r; ++k) lr[k] = log(r_nodes[k]);
  for (int32_t l = 0; l < n_z; ++l) zn[l] = z_nodes[l];
  for (int32_t k = 0; k < n_r; ++k) {
    double col = z_nodes[0] * rho[(int64_t)k * n_z];  /* below the first node */
    for (int32_t l = 0; l < n_z; ++l) {
      const int64_t i = (int64_t)k * n_z + l;
      lrho[i] = log(rho[i]);
      lT[i] = log(T[i]);
      lA[i] = log(alpha[i]);
      if (l + 1 < n_z) col += (z_nodes[l + 1] - z_nodes[l]) * (rho[i] + rho[i + 1]) / 2.0;
    }
    lS[k] = log(2.0 * col); /* both halves of the disk */
  }
}

/* cell of a node array containing x (clamped to the first / last cell) and
 * the fractional position inside it (0 or 1 outside the nodes) */
static void orc_locate(const double *nodes, int32_t n, double x, int32_t *k, double *w) {
  if (!(x > nodes[0])) { *k = 0; *w = 0.0; return; }
  if (!(x < nodes[n - 1])) { *k = n - 2; *w = 1.0; return; }
  int32_t lo = 0, hi = n - 1; /* nodes[lo] <= x < nodes[hi] */
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (x < nodes[mid]) hi = mid; else lo = mid;
  }
  *k = lo;
  *w = (x - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
}

void orc_local_gas_at(const orc_params *P, double r, double z, orc_local_gas *o) {
  const orc_gas_grid *G = P->grid;
  if (!G) {
    double Sg;
    orc_disk_local(P, r, z, &Sg, &o->T, &o->cs, &o->Omega, &o->H, &o->rho_g);
    o->alpha = P->alpha;
    o->slopeP = P->p + (P->q + 3.0) / 2.0;
    /* d ln(r Sigma_g D) / d ln r with Sigma_g ~ r^-p and D ~ c_s H ~ r^(3/2 - q) */
    o->corr = 2.5 - P->q - P->p;
    return;
  }
  /* bilinear in (ln r, z) of ln rho_g, ln T, ln alpha; r-slopes of the same
   * interpolants at this height */
  int32_t k, l;
  double wx, wz;
  orc_locate(G->lr, G->n_r, log(r), &k, &wx);
  orc_locate(G->zn, G->n_z, z, &l, &wz);
  const int64_t i00 = (int64_t)k * G->n_z + l, i10 = i00 + G->n_z, i01 = i00 + 1, i11 = i10 + 1;
  const double dx = G->lr[k + 1] - G->lr[k];
  const double *f[3] = {G->lrho, G->lT, G->lA};
  double val[3], slope[3];
  for (int q = 0; q < 3; ++q) {
    const double *a = f[q];
    val[q] = (1.0 - wx) * (1.0 - wz) * a[i00] + wx * (1.0 - wz) * a[i10] +
             (1.0 - wx) * wz * a[i01] + wx * wz * a[i11];
    slope[q] = ((1.0 - wz) * (a[i10] - a[i00]) + wz * (a[i11] - a[i01])) / dx;
  }
  o->rho_g = exp(val[0]);
  o->T = exp(val[1]);
  o->alpha = exp(val[2]);
  o->cs = sqrt(KB * o->T / (P->mu * MH));
  o->Omega = sqrt(GRAV * P->m_star / (r * r * r));
  o->H = o->cs / o->Omega;
  o->slopeP = -(slope[0] + slope[1]); /* pressure rho_g c_s^2 ~ rho_g T */
  const double dlnS = (G->lS[k + 1] - G->lS[k]) / dx;
  /* d ln(r Sigma_g D) / d ln r, D ~ alpha c_s H ~ alpha T r^(3/2) */
  o->corr = dlnS + slope[2] + slope[1] + 2.5;
}

/* derived gas state of a cell from its six primaries (V, rho_g, T, alpha,
 * r_c, zeta = z_c/H).  Mean free path of H2, molecular viscosity, Reynolds
 * number and the large-eddy velocity follow Ormel & Cuzzi (2007); the
 * midplane pressure-gradient velocity eta v_K follows from P ~ r^-(p+(q+3)/2). */
void orc_gas_derive(const orc_params *P, const double prim[ORC_GAS_FIELDS], orc_gas *g) {
  g->V = prim[0];
  g->rho_g = prim[1];
  g->T = prim[2];
  g->alpha = prim[3];
  g->r_c = prim[4];
  g->zeta = prim[5];
  g->cs = sqrt(KB * g->T / (P->mu * MH));
  g->Omega = sqrt(GRAV * P->m_star / (g->r_c * g->r_c * g->r_c));
  g->H = g->cs / g->Omega;
  g->z_c = g->zeta * g->H;
  if (P->grid) { /* pressure slope of the gridded gas at the cell centre */
    orc_local_gas lg;
    orc_local_gas_at(P, g->r_c, g->z_c, &lg);
    g->eta_vK = 0.5 * (g->cs * g->cs) / (g->Omega * g->r_c) * lg.slopeP;
  } else {
    g->eta_vK = 0.5 * (g->cs * g->cs) / (g->Omega * g->r_c) * (P->p + (P->q + 3.0) / 2.0);
  }
  g->v_th = sqrt(8.0 / PI) * g->cs;
  g->lambda = P->mu * MH / (g->rho_g * SIGMA_H2);
  g->nu = 0.5 * g->v_th * g->lambda;
  g->Re = g->alpha * g->cs * g->H / g->nu;
  g->St_eta = 1.0 / sqrt(g->Re);
  g->Vg2 = 1.5 * g->alpha * g->cs * g->cs;
}

/* stopping time: Epstein drag below a = 9 lambda / 4, Stokes drag above */
static double orc_stopping_time(const orc_params *P, double a, double rho_g, double v_th,
                                double lambda, double nu) {
  if (a < 2.25 * lambda) return P->rho_s * a / (rho_g * v_th);
  return 2.0 * P->rho_s * a * a / (9.0 * nu * rho_g);
}

/* per-particle state inside a cell.  Radius of a compact sphere; drift and
 * azimuthal velocities of a particle in a gas without radial flow
 * (Nakagawa-type solution); terminal settling speed at the cell height. */
void orc_particle_props(const orc_params *P, const orc_gas *g, double m, double M,
                        orc_particle *o) {
  o->m = m;
  o->M = M;
  o->a = cbrt(3.0 * m / (4.0 * PI * P->rho_s));
  o->t_s = orc_stopping_time(P, o->a, g->rho_g, g->v_th, g->lambda, g->nu);
  o->St = o->t_s * g->Omega;
  o->v_r = -2.0 * g->eta_vK * o->St / (1.0 + o->St * o->St);
  o->v_phi = -g->eta_vK / (1.0 + o->St * o->St);
  o->v_z = -g->z_c * g->Omega * o->St / (1.0 + o->St);
  o->n = M / (m * g->V);
}

/* turbulent relative velocity squared, the three closed-form regimes of
 * Ormel & Cuzzi (2007): tightly coupled (St1 < St_eta), intermediate
 * (St_eta <= St1 < 1) and heavy (St1 >= 1); St1 is the larger Stokes number */
double orc_dv2_turb(const orc_gas *g, double St_a, double St_b) {
  double St1 = St_a > St_b ? St_a : St_b;
  double St2 = St_a > St_b ? St_b : St_a;
  if (St1 < g->St_eta) {
    double h1 = St1 * St1 / (St1 + g->St_eta);
    double h2 = St2 * St2 / (St2 + g->St_eta);
    return g->Vg2 * (St1 - St2) / (St1 + St2) * (h1 - h2);
  }
  if (St1 < 1.0) {
    double eps = St2 / St1;
    double bracket = 2.0 * YA - (1.0 + eps) +
                     2.0 / (1.0 + eps) * (1.0 / (1.0 + YA) + eps * eps * eps / (YA + eps));
    return g->Vg2 * St1 * bracket;
  }
  return g->Vg2 * (1.0 / (1.0 + St1) + 1.0 / (1.0 + St2));
}

/* relative velocity: the five sources added in quadrature */
double orc_rel_velocity(const orc_params *P, const orc_gas *g, const orc_particle *pi,
                        const orc_particle *pj) {
  double dv2 = 0.0;
  if (P->flags & ORC_DV_BROWNIAN) dv2 += 8.0 * KB * g->T / PI * (1.0 / pi->m + 1.0 / pj->m);
  if (P->flags & ORC_DV_TURB) dv2 += orc_dv2_turb(g, pi->St, pj->St);
  if (P->flags & ORC_DV_RADIAL) {
    double d = pi->v_r - pj->v_r;
    dv2 += d * d;
  }
  if (P->flags & ORC_DV_AZIMUTHAL) {
    double d = pi->v_phi - pj->v_phi;
    dv2 += d * d;
  }
  if (P->flags & ORC_DV_SETTLING) {
    double d = pi->v_z - pj->v_z;
    dv2 += d * d;
  }
  return sqrt(dv2);
}

/* collision kernel K_ij: geometric cross-section times relative velocity;
 * or the constant / linear test kernels of the Smoluchowski equation */
double orc_pair_kernel(const orc_params *P, const orc_gas *g, const orc_particle *pi,
                       const orc_particle *pj) {
  if (P->kernel == ORC_K_CONSTANT) return P->k0;
  if (P->kernel == ORC_K_LINEAR) return P->k0 * (pi->m + pj->m);
  double s = pi->a + pj->a;
  return PI * s * s * orc_rel_velocity(P, g, pi, pj);
}

/* rate at which representative particle i collides with swarm j
 * (Zsom & Dullemond 2008): n_j K_ij, divided by the grouping factor
 * g_ij = max(1, dm_max m_i / m_j) when grouping is on */
double orc_rate(const orc_params *P, const orc_gas *g, const orc_particle *pi,
                const orc_particle *pj) {
  double k = orc_pair_kernel(P, g, pi, pj);
  double grp = 1.0;
  if (P->dm_max > 0.0) {
    grp = P->dm_max * pi->m / pj->m;
    if (grp < 1.0) grp = 1.0;
  }
  return pj->n * k / grp;
}

/* fragment mass: inverse-CDF draw from the mass-weighted distribution
 * m^(1-xi) with xi = 11/6 on [lo, hi] */
double orc_frag_draw(double lo, double hi, double u) {
  if (!(hi > lo)) return lo;
  double slo = sqrt(cbrt(lo));
  double shi = sqrt(cbrt(hi));
  double x = slo + u * (shi - slo);
  double x2 = x * x;
  return x2 * x2 * x2;
}

/* first index whose inclusive prefix sum exceeds target; if rounding leaves
 * none, the last index with a nonzero entry */
int32_t orc_select(const double *v, int32_t n, double target) {
  double cum = 0.0;
  int32_t last = -1;
  for (int32_t k = 0; k < n; ++k) {
    cum += v[k];
    if (cum > target) return k;
    if (v[k] > 0.0) last = k;
  }
  return last;
}

static double orc_m0(const orc_params *P) {
  return 4.0 / 3.0 * PI * P->a_mono * P->a_mono * P->a_mono * P->rho_s;
}

/* outcome of a collision of representative particle i (mass mi) with a
 * member of swarm j (mass mj): sticking below v_frag; otherwise erosion when
 * the mass ratio reaches erosion_ratio, else fragmentation.  Only i changes. */
/* Fragmentation criterion.  Sharp: fragment iff dv >= v_frag (the paper's
 * fragmentation velocity).  Ramp: the probability rises linearly from 0 at
 * (1 - w) v_frag to 1 at v_frag.  Maxwell: the collision speed follows the
 * Maxwell speed distribution whose mean is dv (scale a = dv sqrt(pi/8)), and
 * the probability is the tail above v_frag,
 * erfc(x) + 2/sqrt(pi) x exp(-x^2) with x = v_frag / (sqrt(2) a). */
double orc_frag_probability(const orc_params *P, double dv) {
  const double vf = P->v_frag;
  if (P->frag_mode == ORC_FRAG_RAMP) {
    const double lo = (1.0 - P->frag_width) * vf;
    if (dv <= lo) return 0.0;
    if (dv >= vf) return 1.0;
    return (dv - lo) / (vf - lo);
  }
  if (P->frag_mode == ORC_FRAG_MAXWELL) {
    if (!(dv > 0.0)) return 0.0;
    const double x = 2.0 * vf / (sqrt(PI) * dv);
    return erfc(x) + 2.0 / sqrt(PI) * x * exp(-x * x);
  }
  return dv < vf ? 0.0 : 1.0;
}

/* uf: the uniform of the fragmentation decision (used unless sharp) */
int32_t orc_outcome(const orc_params *P, double dv, double mi, double mj, double u, double uf,
                    double *m_new) {
  double grp = 1.0;
  if (P->dm_max > 0.0) {
    grp = P->dm_max * mi / mj;
    if (grp < 1.0) grp = 1.0;
  }
  const int fast = P->frag_mode == ORC_FRAG_SHARP ? !(dv < P->v_frag)
                                                  : uf < orc_frag_probability(P, dv);
  if (P->kernel != ORC_K_PHYSICAL || !fast) {
    *m_new = mi + grp * mj;
    return ORC_OUT_STICK;
  }
  double m0 = orc_m0(P);
  double big = mi > mj ? mi : mj;
  double small = mi > mj ? mj : mi;
  if (big / small >= P->erosion_ratio) {
    if (mi >= mj) {
      double m = mi - P->erosion_chi * grp * mj;
      *m_new = m > m0 ? m : m0;
      return ORC_OUT_ERODE;
    }
    *m_new = orc_frag_draw(m0, mi, u);
    return ORC_OUT_ERODED_SMALL;
  }
  *m_new = orc_frag_draw(m0, big, u);
  return ORC_OUT_FRAG;
}

/* ------------------------------------------------------------------------ */
/* Rate matrix of one cell                                                   */
/* ------------------------------------------------------------------------ */
void orc_cell_rates(const orc_params *P, const double prim[ORC_GAS_FIELDS], int32_t n,
                    const int32_t *members, const double *m, const double *M,
                    double *r_out, double *rowsum_out) {
  orc_gas g;
  orc_gas_derive(P, prim, &g);
  orc_particle *pp = (orc_particle *)malloc(sizeof(orc_particle) * (size_t)(n > 0 ? n : 1));
  for (int32_t k = 0; k < n; ++k) orc_particle_props(P, &g, m[members[k]], M[members[k]], &pp[k]);
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      double rij = orc_rate(P, &g, &pp[i], &pp[j]);
      if (r_out) r_out[(int64_t)i * n + j] = rij;
      s += rij;
    }
    if (rowsum_out) rowsum_out[i] = s;
  }
  free(pp);
}

/* ------------------------------------------------------------------------ */
/* Equal-count adaptive binning (paper, Summary: every cell holds the same   */
/* number of representative particles).  Radial zones by rank of (r, index); */
/* cells inside a zone by rank of (|z|, index); the floor rule splits a      */
/* count that does not divide evenly.  Interior edges sit half-way between   */
/* neighbouring ranks; the grid spans the particles.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  double key;
  int32_t idx;
} orc_key;

static int orc_key_cmp(const void *a, const void *b) {
  const orc_key *x = (const orc_key *)a, *y = (const orc_key *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

int64_t orc_bin(const orc_params *P, int64_t N, const double *r, const double *z,
                const uint8_t *active, int32_t *cell_start, int32_t *order, double *geom,
                double *gas) {
  const int32_t nr = P->n_r, nz = P->n_z, nc = nr * nz;
  int64_t na = 0;
  for (int64_t k = 0; k < N; ++k) na += active[k] ? 1 : 0;
  orc_key *kr = (orc_key *)malloc(sizeof(orc_key) * (size_t)(na > 0 ? na : 1));
  orc_key *kz = (orc_key *)malloc(sizeof(orc_key) * (size_t)(na > 0 ? na : 1));
  int64_t w = 0;
  for (int64_t k = 0; k < N; ++k)
    if (active[k]) { kr[w].key = r[k]; kr[w].idx = (int32_t)k; ++w; }
  qsort(kr, (size_t)na, sizeof(orc_key), orc_key_cmp);

  for (int32_t zr = 0; zr < nr; ++zr) {
    int64_t b0 = (int64_t)zr * na / nr, b1 = (int64_t)(zr + 1) * na / nr;
    int64_t nk = b1 - b0;
    double r_lo, r_hi;
    if (nk > 0) {
      /* edges half-way to the neighbouring ranks; the grid ends at the
       * first and last active particle */
      r_lo = (b0 == 0) ? kr[b0].key : 0.5 * (kr[b0 - 1].key + kr[b0].key);
      r_hi = (b1 == na) ? kr[b1 - 1].key : 0.5 * (kr[b1 - 1].key + kr[b1].key);
    } else {
      r_lo = r_hi = 0.0;
    }
    for (int64_t k = 0; k < nk; ++k) { kz[b0 + k].key = z[kr[b0 + k].idx]; kz[b0 + k].idx = kr[b0 + k].idx; }
    qsort(kz + b0, (size_t)nk, sizeof(orc_key), orc_key_cmp);
    for (int64_t k = 0; k < nk; ++k) order[b0 + k] = kz[b0 + k].idx;
    for (int32_t l = 0; l < nz; ++l) {
      int64_t s0 = b0 + (int64_t)l * nk / nz, s1 = b0 + (int64_t)(l + 1) * nk / nz;
      int32_t c = zr * nz + l;
      cell_start[c] = (int32_t)s0;
      double z_lo = 0.0, z_hi = 0.0;
      if (s1 > s0) {
        /* the lowest occupied cell of a zone starts at the midplane, the
         * highest ends at its topmost particle */
        z_lo = (s0 == b0) ? 0.0 : 0.5 * (kz[s0 - 1].key + kz[s0].key);
        z_hi = (s1 == b1) ? kz[s1 - 1].key : 0.5 * (kz[s1 - 1].key + kz[s1].key);
      }
      double V;
      double r_c = P->column ? P->r_col : 0.5 * (r_lo + r_hi);
      double z_c = 0.5 * (z_lo + z_hi);
      if (P->column)
        V = 2.0 * (z_hi - z_lo);
      else
        V = 2.0 * PI * (r_hi * r_hi - r_lo * r_lo) * (z_hi - z_lo);
      double *gm = geom + (int64_t)c * 5;
      gm[0] = r_lo; gm[1] = r_hi; gm[2] = z_lo; gm[3] = z_hi; gm[4] = V;
      double *gs = gas + (int64_t)c * ORC_GAS_FIELDS;
      if (s1 > s0) {
        orc_local_gas lg;
        orc_local_gas_at(P, r_c, z_c, &lg);
        gs[0] = V; gs[1] = lg.rho_g; gs[2] = lg.T; gs[3] = lg.alpha; gs[4] = r_c; gs[5] = z_c / lg.H;
      } else {
        gs[0] = 0.0; gs[1] = 0.0; gs[2] = 0.0; gs[3] = 0.0; gs[4] = 0.0; gs[5] = 0.0;
      }
    }
  }
  cell_start[nc] = (int32_t)na;
  free(kr);
  free(kz);
  return na;
}

/* ------------------------------------------------------------------------ */
/* Collision Monte Carlo inside one cell (Zsom & Dullemond 2008)             */
/* ------------------------------------------------------------------------ */
int64_t orc_collide_cell(const orc_params *P, const double prim[ORC_GAS_FIELDS],
                         int32_t cell_id, uint32_t step, int32_t n, const int32_t *members,
                         double *m, const double *M, float *comp, int64_t N, double dt,
                         int64_t max_events, orc_event *evlog, int64_t log_cap,
                         orc_cell_stats *st) {
  if (st) memset(st, 0, sizeof(*st));
  if (n <= 0) return 0;
  orc_gas g;
  orc_gas_derive(P, prim, &g);
  orc_particle *pp = (orc_particle *)malloc(sizeof(orc_particle) * (size_t)n);
  double *rr = (double *)malloc(sizeof(double) * (size_t)n);   /* row sums r_i */
  double *row = (double *)malloc(sizeof(double) * (size_t)n);  /* r_ij of the chosen i */
  double *col = (double *)malloc(sizeof(double) * (size_t)n);  /* r_ki before the event */
  for (int32_t k = 0; k < n; ++k) orc_particle_props(P, &g, m[members[k]], M[members[k]], &pp[k]);

  /* row sums, diagonal included (a particle also meets its own swarm) */
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t j = 0; j < n; ++j) s += orc_rate(P, &g, &pp[i], &pp[j]);
    rr[i] = s;
  }

  double t = 0.0;
  int64_t e = 0;
  for (;;) {
    double R = 0.0;
    for (int32_t k = 0; k < n; ++k) R += rr[k];
    if (!(R > 0.0)) break;
    if (max_events > 0 && e >= max_events) break;
    double u1, u2, u3, u4;
    orc_uniforms(P, (uint32_t)e, (uint32_t)cell_id, step, 0u, &u1, &u2);
    orc_uniforms(P, (uint32_t)e, (uint32_t)cell_id, step, 1u, &u3, &u4);
    double tau = -log(u1) / R;           /* exponential waiting time */
    if (dt > 0.0 && t + tau > dt) break; /* memoryless: the next event falls outside */
    t += tau;

    int32_t i = orc_select(rr, n, u2 * R);
    double Ri = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      row[j] = orc_rate(P, &g, &pp[i], &pp[j]);
      Ri += row[j];
    }
    if (!(Ri > 0.0)) {
      /* row i has no partner left (its stored sum was rounding residue):
       * clear it and count a null event */
      rr[i] = 0.0;
      if (evlog && e < log_cap) {
        evlog[e].i = i; evlog[e].j = -1; evlog[e].outcome = -1; evlog[e].pad = 0;
      }
      ++e;
      continue;
    }
    int32_t j = orc_select(row, n, u3 * Ri);
    double dv = (P->kernel == ORC_K_PHYSICAL) ? orc_rel_velocity(P, &g, &pp[i], &pp[j]) : 0.0;
    for (int32_t k = 0; k < n; ++k) col[k] = orc_rate(P, &g, &pp[k], &pp[i]);

    double mi = pp[i].m, mj = pp[j].m, mnew, u5 = 0.0, u6;
    if (P->frag_mode != ORC_FRAG_SHARP)
      orc_uniforms(P, (uint32_t)e, (uint32_t)cell_id, step, 3u, &u5, &u6);
    int32_t oc = orc_outcome(P, dv, mi, mj, u4, u5, &mnew);
    if (comp && P->n_comp > 0 && (oc == ORC_OUT_STICK || oc == ORC_OUT_FRAG)) {
      double grp = 1.0;
      if (P->dm_max > 0.0) {
        grp = P->dm_max * mi / mj;
        if (grp < 1.0) grp = 1.0;
      }
      double wi = mi, wj = grp * mj;
      int64_t pi_ = members[i], pj_ = members[j];
      for (int32_t s = 0; s < P->n_comp; ++s) {
        double ci = (double)comp[(int64_t)s * N + pi_];
        double cj = (double)comp[(int64_t)s * N + pj_];
        comp[(int64_t)s * N + pi_] = (float)((wi * ci + wj * cj) / (wi + wj));
      }
    }
    m[members[i]] = mnew;
    orc_particle_props(P, &g, mnew, pp[i].M, &pp[i]);

    /* incremental update of the other rows, fresh sum of row i */
    for (int32_t k = 0; k < n; ++k) {
      if (k == i) continue;
      double x = (rr[k] - col[k]) + orc_rate(P, &g, &pp[k], &pp[i]);
      rr[k] = x > 0.0 ? x : 0.0;
    }
    double s = 0.0;
    for (int32_t q = 0; q < n; ++q) s += orc_rate(P, &g, &pp[i], &pp[q]);
    rr[i] = s;

    if (evlog && e < log_cap) {
      evlog[e].i = i; evlog[e].j = j; evlog[e].outcome = oc; evlog[e].pad = 0;
    }
    if (st) st->outcomes[oc] += 1;
    ++e;
  }
  if (st) {
    st->events = e;
    st->t_end = t;
    /* diagnostic: distance of the incrementally updated row sums from a
     * fresh evaluation, relative to the total rate */
    double R = 0.0, worst = 0.0;
    for (int32_t k = 0; k < n; ++k) R += rr[k];
    for (int32_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int32_t j = 0; j < n; ++j) s += orc_rate(P, &g, &pp[i], &pp[j]);
      double d = fabs(s - rr[i]);
      if (d > worst) worst = d;
    }
    st->drift = R > 0.0 ? worst / R : 0.0;
  }
  free(pp); free(rr); free(row); free(col);
  return e;
}

void orc_collide_all(const orc_params *P, int32_t n_cells, const int32_t *cell_start,
                     const int32_t *order, const double *gas, uint32_t step, double *m,
                     const double *M, float *comp, int64_t N, double dt, int64_t max_events,
                     orc_event *evlog, int64_t log_per_cell, orc_cell_stats *stats,
                     int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int32_t c = 0; c < n_cells; ++c) {
    int32_t s0 = cell_start[c], n = cell_start[c + 1] - s0;
    orc_collide_cell(P, gas + (int64_t)c * ORC_GAS_FIELDS, c, step, n, order + s0, m, M, comp, N,
                     dt, max_events, evlog ? evlog + (int64_t)c * log_per_cell : NULL,
                     evlog ? log_per_cell : 0, stats ? stats + c : NULL);
  }
}

/* ------------------------------------------------------------------------ */
/* Transport (paper, Summary: radial and vertical).  A random walk with       */
/* uniform kicks of variance 2 D dt (Ciesla 2010 type), D = alpha cs H /     */
/* (1 + St^2); semi-implicit settling toward the midplane with the gas-      */
/* density correction D/H^2; mirror symmetry folds z; r < r_in leaves the    */
/* grid.  Radially the walk drifts by (D/r) d ln(r Sigma_g D)/d ln r on top  */
/* of the gas-drag drift: the probability density of a particle's radius,   */
/* per unit r, is P = 2 pi r Sigma_d, and a tracer's concentration          */
/* Sigma_d/Sigma_g diffuses through rings of circumference 2 pi r, so        */
/* dP/dt = d/dr [D w d(P/w)/dr] with w = r Sigma_g; the Ito walk with kicks  */
/* of variance 2 D dt has this Fokker-Planck equation when its drift is      */
/* D/w dw/dr + dD/dr.  For the power-law disk the factor is 5/2 - p - q.    */
/* The particle's 1/(1 + St^2) is held fixed over the derivative.            */
/* ------------------------------------------------------------------------ */
void orc_transport(const orc_params *P, int64_t N, double *r, double *z, const double *m,
                   uint8_t *active, uint32_t step, double dt) {
  const uint32_t fl = P->flags;
  for (int64_t k = 0; k < N; ++k) {
    if (!active[k]) continue;
    double rk = P->column ? P->r_col : r[k];
    double zk = z[k];
    orc_local_gas lg;
    orc_local_gas_at(P, rk, zk, &lg);
    const double cs = lg.cs, Om = lg.Omega, H = lg.H, rho = lg.rho_g;
    double v_th = sqrt(8.0 / PI) * cs;
    double lambda = P->mu * MH / (rho * SIGMA_H2);
    double nu = 0.5 * v_th * lambda;
    double a = cbrt(3.0 * m[k] / (4.0 * PI * P->rho_s));
    double St = orc_stopping_time(P, a, rho, v_th, lambda, nu) * Om;
    double D = lg.alpha * cs * H / (1.0 + St * St);
    double ur, uz;
    orc_uniforms(P, (uint32_t)k, 0u, step, 2u, &ur, &uz);
    double kick_r = 2.0 * ur - 1.0, kick_z = 2.0 * uz - 1.0;

    double kz = 0.0, dz = 0.0;
    if (fl & ORC_TR_SETTLE) kz += Om * St / (1.0 + St);
    if (fl & ORC_TR_MIX_Z) {
      kz += D / (H * H);
      dz = kick_z * sqrt(6.0 * D * dt);
    }
    z[k] = fabs((zk + dz) / (1.0 + kz * dt));

    if (!P->column) {
      double v = 0.0, dr = 0.0;
      if (fl & ORC_TR_DRIFT) {
        double eta_vK = 0.5 * cs * cs / (Om * rk) * lg.slopeP;
        v += -2.0 * eta_vK * St / (1.0 + St * St);
      }
      if (fl & ORC_TR_MIX_R) {
        v += D * lg.corr / rk;
        dr = kick_r * sqrt(6.0 * D * dt);
      }
      double rn = rk + v * dt + dr;
      r[k] = rn;
      if (rn < P->r_in) active[k] = 0;
    }
  }
}

/* ------------------------------------------------------------------------
 * sigma_d(m, r) (paper, Benchmark: surface density by particle mass and
 * distance from the star)
 * ------------------------------------------------------------------------ */
/* index k with e[k] <= x < e[k+1], or -1 outside [e[0], e[n]) */
static int32_t orc_find_bin(const double *e, int32_t n, double x) {
  if (!(x >= e[0]) || !(x < e[n])) return -1;
  int32_t lo = 0, hi = n; /* e[lo] <= x < e[hi] */
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (x < e[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

int64_t orc_sigma_hist(int64_t N, const double *r, const double *m, const double *M,
                       const uint8_t *active, const double *r_edges, int32_t n_rb,
                       const double *m_edges, int32_t n_mb, int32_t column, double *sigma,
                       uint32_t *count) {
  const int64_t nb = (int64_t)n_rb * n_mb;
  for (int64_t b = 0; b < nb; ++b) {
    sigma[b] = 0.0;
    if (count) count[b] = 0u;
  }
  int64_t counted = 0;
  for (int64_t i = 0; i < N; ++i) {
    if (!active[i]) continue;
    const int32_t k = orc_find_bin(r_edges, n_rb, r[i]);
    const int32_t l = orc_find_bin(m_edges, n_mb, m[i]);
    if (k < 0 || l < 0) continue;
    sigma[(int64_t)k * n_mb + l] += M[i];
    if (count) count[(int64_t)k * n_mb + l] += 1u;
    ++counted;
  }
  for (int32_t k = 0; k < n_rb; ++k) {
    const double area = column ? 1.0
                               : PI * (r_edges[k + 1] * r_edges[k + 1] - r_edges[k] * r_edges[k]);
    for (int32_t l = 0; l < n_mb; ++l) sigma[(int64_t)k * n_mb + l] /= area;
  }
  return counted;
}
