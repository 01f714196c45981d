// physics.hpp -- gas state, particle state and the pair collision rate of
// the representative-particle method, for device (and host) code.
//
// The paper (arXiv 2507.21239, Summary) fixes the model: a static
// power-law disk, vertically isothermal; representative particles after
// Zsom & Dullemond (2008) colliding inside equal-count cells; relative
// velocities from Brownian motion, turbulence, radial and azimuthal drift and
// settling (the formulas are deferred to Drazkowska et al. 2013).  The forms
// used here: thin-disk gas (Gaussian vertical profile), Epstein / Stokes
// drag switching at a = 9 lambda / 4, Nakagawa-type drift velocities,
// turbulent velocities in the three closed-form regimes of Ormel & Cuzzi
// (2007), the five sources added in quadrature, geometric cross-sections,
// and the swarm rate r_ij = n_j K_ij / max(1, dm_max m_i / m_j).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mcd {

// physical constants, CGS
constexpr double kBoltz = 1.380649e-16;
constexpr double kMassH = 1.6735575e-24;
constexpr double kGrav = 6.67430e-8;
constexpr double kSigmaH2 = 2e-15;
constexpr double kPi = 3.14159265358979323846;
constexpr double kYa = 1.6;  // Ormel & Cuzzi (2007) y*_a

enum : uint32_t {
  DV_BROWNIAN = 1u << 0,
  DV_TURB = 1u << 1,
  DV_RADIAL = 1u << 2,
  DV_AZIMUTHAL = 1u << 3,
  DV_SETTLING = 1u << 4,
  TR_DRIFT = 1u << 8,
  TR_SETTLE = 1u << 9,
  TR_MIX_R = 1u << 10,
  TR_MIX_Z = 1u << 11,
  COAG = 1u << 12,
};
enum { K_PHYSICAL = 0, K_CONSTANT = 1, K_LINEAR = 2 };
enum { OUT_STICK = 0, OUT_ERODE = 1, OUT_ERODED_SMALL = 2, OUT_FRAG = 3 };

// model constants copied to the device by value
// gridded gas on the device: node values on nr radii x nz heights, as
// logarithms (nr == 0: the power-law disk)
struct GasGridView {
  const double *lr;    // [nr] ln r of the radial nodes
  const double *zn;    // [nz] heights of the vertical nodes
  const double *lrho;  // [nr][nz] ln rho_g
  const double *lT;    // [nr][nz] ln T
  const double *lA;    // [nr][nz] ln alpha
  const double *lS;    // [nr] ln Sigma_g
  int32_t nr, nz;
};

struct Model {
  double sigma_g0, T0, p, q, alpha, v_frag, erosion_ratio, rho_s, mu, m_star, r_ref;
  double dm_max, erosion_chi, r_in, r_col, k0, m0, frag_width;
  uint32_t flags;
  int32_t kernel, column, n_comp, frag_mode;
  uint32_t key0, key1;
  GasGridView grid;
};

enum : int32_t { FRAG_SHARP = 0, FRAG_RAMP = 1, FRAG_MAXWELL = 2 };

// the model parameters a collision outcome reads, gathered per cell into the
// team's LDS scratch: read there once per event instead of being held (and
// spilled) in scalar registers for the whole persistent launch
struct OutcomeConst {
  double v_frag, erosion_ratio, erosion_chi, m0, dm_max, frag_width;
  int32_t kernel, frag_mode, n_comp, pad;
};

__host__ __device__ inline OutcomeConst make_outcome_const(const Model &P) {
  OutcomeConst o;
  o.v_frag = P.v_frag;
  o.erosion_ratio = P.erosion_ratio;
  o.erosion_chi = P.erosion_chi;
  o.m0 = P.m0;
  o.dm_max = P.dm_max;
  o.frag_width = P.frag_width;
  o.kernel = P.kernel;
  o.frag_mode = P.frag_mode;
  o.n_comp = P.n_comp;
  o.pad = 0;
  return o;
}

struct DiskPoint {
  double Sigma_g, T, cs, Omega, H, rho_g;
};

__host__ __device__ inline DiskPoint disk_at(const Model &P, double r, double z) {
  DiskPoint d;
  const double x = r / P.r_ref;
  d.Sigma_g = P.sigma_g0 * pow(x, -P.p);
  d.T = P.T0 * pow(x, -P.q);
  d.cs = sqrt(kBoltz * d.T / (P.mu * kMassH));
  d.Omega = sqrt(kGrav * P.m_star / (r * r * r));
  d.H = d.cs / d.Omega;
  d.rho_g = d.Sigma_g / (sqrt(2.0 * kPi) * d.H) * exp(-(z * z) / (2.0 * d.H * d.H));
  return d;
}

// gas at one point: density, temperature, turbulence, sound speed, Kepler
// frequency, scale height, pressure slope s = -d ln P / d ln r (eta v_K =
// c_s^2 s / (2 Omega r)) and the radial-diffusion correction factor c (the
// random walk drifts by D c / r: the logarithmic r-derivative of
// r Sigma_g D with D ~ alpha c_s H, the drift under which an axisymmetric
// random walk keeps a tracer distributed like the gas)
struct LocalGas {
  double rho_g, T, alpha, cs, Omega, H, slopeP, corr;
};

// cell of a node array containing x, clamped to the first / last cell, and
// the fractional position in it (0 or 1 outside the nodes)
__host__ __device__ inline void grid_locate(const double *nodes, int n, double x, int &k,
                                            double &w) {
  if (!(x > nodes[0])) {
    k = 0;
    w = 0.0;
    return;
  }
  if (!(x < nodes[n - 1])) {
    k = n - 2;
    w = 1.0;
    return;
  }
  int lo = 0, hi = n - 1;  // nodes[lo] <= x < nodes[hi]
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (x < nodes[mid])
      hi = mid;
    else
      lo = mid;
  }
  k = lo;
  w = (x - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
}

// power-law disk, or the gridded gas: bilinear in (ln r, z) of ln rho_g,
// ln T and ln alpha, with the r-slopes of those interpolants at this height;
// the surface density's slope from its radial nodes
__host__ __device__ inline LocalGas local_gas_at(const Model &P, double r, double z) {
  LocalGas o;
  const GasGridView &G = P.grid;
  if (G.nr == 0) {
    const DiskPoint d = disk_at(P, r, z);
    o.rho_g = d.rho_g;
    o.T = d.T;
    o.cs = d.cs;
    o.Omega = d.Omega;
    o.H = d.H;
    o.alpha = P.alpha;
    o.slopeP = P.p + (P.q + 3.0) / 2.0;
    o.corr = 2.5 - P.q - P.p;  // Sigma_g ~ r^-p, c_s H ~ r^(3/2 - q), times r
    return o;
  }
  int k, l;
  double wx, wz;
  grid_locate(G.lr, G.nr, log(r), k, wx);
  grid_locate(G.zn, G.nz, z, l, wz);
  const int64_t i00 = (int64_t)k * G.nz + l, i10 = i00 + G.nz, i01 = i00 + 1, i11 = i10 + 1;
  const double dx = G.lr[k + 1] - G.lr[k];
  const double *f[3] = {G.lrho, G.lT, G.lA};
  double val[3], slope[3];
  for (int q = 0; q < 3; ++q) {
    const double *a = f[q];
    val[q] = (1.0 - wx) * (1.0 - wz) * a[i00] + wx * (1.0 - wz) * a[i10] +
             (1.0 - wx) * wz * a[i01] + wx * wz * a[i11];
    slope[q] = ((1.0 - wz) * (a[i10] - a[i00]) + wz * (a[i11] - a[i01])) / dx;
  }
  o.rho_g = exp(val[0]);
  o.T = exp(val[1]);
  o.alpha = exp(val[2]);
  o.cs = sqrt(kBoltz * o.T / (P.mu * kMassH));
  o.Omega = sqrt(kGrav * P.m_star / (r * r * r));
  o.H = o.cs / o.Omega;
  o.slopeP = -(slope[0] + slope[1]);  // pressure rho_g c_s^2 ~ rho_g T
  const double dlnS = (G.lS[k + 1] - G.lS[k]) / dx;
  o.corr = dlnS + slope[2] + slope[1] + 2.5;  // alpha T r^(3/2), times r
  return o;
}

// gas state of a cell, from its six primaries (V, rho_g, T, alpha, r_c,
// zeta = z_c / H)
struct Gas {
  double V, rho_g, T, alpha, r_c, zeta;
  double cs, Omega, H, z_c, eta_vK, v_th, lambda, nu, Re, St_eta, Vg2;
};

__host__ __device__ inline void gas_from_primaries(const Model &P, const double *prim, Gas &g) {
  g.V = prim[0];
  g.rho_g = prim[1];
  g.T = prim[2];
  g.alpha = prim[3];
  g.r_c = prim[4];
  g.zeta = prim[5];
  g.cs = sqrt(kBoltz * g.T / (P.mu * kMassH));
  g.Omega = sqrt(kGrav * P.m_star / (g.r_c * g.r_c * g.r_c));
  g.H = g.cs / g.Omega;
  g.z_c = g.zeta * g.H;
  // midplane pressure-gradient velocity: P ~ r^-(p + (q+3)/2)
  g.eta_vK = 0.5 * (g.cs * g.cs) / (g.Omega * g.r_c) *
             (P.grid.nr ? local_gas_at(P, g.r_c, g.z_c).slopeP : (P.p + (P.q + 3.0) / 2.0));
  g.v_th = sqrt(8.0 / kPi) * g.cs;
  g.lambda = P.mu * kMassH / (g.rho_g * kSigmaH2);
  g.nu = 0.5 * g.v_th * g.lambda;
  g.Re = g.alpha * g.cs * g.H / g.nu;
  g.St_eta = 1.0 / sqrt(g.Re);
  g.Vg2 = 1.5 * g.alpha * g.cs * g.cs;
}

// power-law disk at (r, z): Sigma_g, T, c_s, Omega, H, rho_g
__host__ __device__ inline double stopping_time(double rho_s, double a, double rho_g, double v_th,
                                                double lambda, double nu) {
  if (a < 2.25 * lambda) return rho_s * a / (rho_g * v_th);  // Epstein
  return 2.0 * rho_s * a * a / (9.0 * nu * rho_g);           // Stokes
}

// per-particle record used by the pair rate, in the rate precision RT
template <typename RT>
struct Rec {
  RT m;    // mass
  RT im;   // 1/m
  RT a;    // radius
  RT St;   // Stokes number
  RT h;    // St^2 / (St + St_eta)
  RT q1;   // 1 / (1 + St)
  RT vr;   // radial drift velocity
  RT vp;   // azimuthal velocity relative to Keplerian
  RT vz;   // settling velocity at the cell height
  RT nd;   // swarm number density M/(m V), times the cell's rate scale
  RT ist;  // 1 / St
  RT Mn;   // swarm mass M / V times the rate scale (nd = Mn / m)
};

// the FP32 record carries sqrt(pi) a in place of a, so that the collision
// cross-section pi (a_i + a_j)^2 needs no extra product
constexpr double kSqrtPi = 1.7724538509055160273;
template <typename RT>
__host__ __device__ constexpr double radius_factor() {
  return sizeof(RT) == 4 ? kSqrtPi : 1.0;
}

// particle state in FP64 (the precompute is always FP64), rounded to RT
template <typename RT>
__host__ __device__ inline Rec<RT> make_rec(const Model &P, const Gas &g, double m, double M,
                                            double nd_scale) {
  const double a = cbrt(3.0 * m / (4.0 * kPi * P.rho_s));
  const double ts = stopping_time(P.rho_s, a, g.rho_g, g.v_th, g.lambda, g.nu);
  const double St = ts * g.Omega;
  Rec<RT> o;
  o.m = (RT)m;
  o.im = (RT)(1.0 / m);
  o.a = (RT)(a * radius_factor<RT>());
  o.St = (RT)St;
  o.ist = (RT)(1.0 / St);
  o.h = (RT)(St * St / (St + g.St_eta));
  o.q1 = (RT)(1.0 / (1.0 + St));
  o.vr = (RT)(-2.0 * g.eta_vK * St / (1.0 + St * St));
  o.vp = (RT)(-g.eta_vK / (1.0 + St * St));
  o.vz = (RT)(-g.z_c * g.Omega * St / (1.0 + St));
  o.nd = (RT)(M / (m * g.V) * nd_scale);
  o.Mn = (RT)(M * (nd_scale / g.V));
  return o;
}

// per-cell constants of the FP32 particle state (mixed precision): the
// same formulas as make_rec with the cell factors folded in single precision
struct CellF {
  float ca;     // 3 / (4 pi rho_s)
  float a_sw;   // Epstein / Stokes switch radius 9 lambda / 4
  float tE;     // Epstein stopping time per unit radius rho_s / (rho_g v_th)
  float tS;     // Stokes stopping time per unit radius^2 2 rho_s / (9 nu rho_g)
  float Om, Ste, m2eta, meta, mzO;
  float pad;
  double nd_fac;  // rate scale / V
};

__host__ __device__ inline CellF make_cellf(const Model &P, const Gas &g, double scale) {
  CellF c;
  c.ca = (float)(3.0 / (4.0 * kPi * P.rho_s));
  c.a_sw = (float)(2.25 * g.lambda);
  c.tE = (float)(P.rho_s / (g.rho_g * g.v_th));
  c.tS = (float)(2.0 * P.rho_s / (9.0 * g.nu * g.rho_g));
  c.Om = (float)g.Omega;
  c.Ste = (float)g.St_eta;
  c.m2eta = (float)(-2.0 * g.eta_vK);
  c.meta = (float)(-g.eta_vK);
  c.mzO = (float)(-g.z_c * g.Omega);
  c.pad = 0.0f;
  c.nd_fac = scale / g.V;
  return c;
}

// per-cell constants of the pair rate
template <typename RT>
struct PairConst {
  RT cBM;      // 8 k T / pi
  RT Vg2;      // large-eddy velocity squared
  RT St_eta;   // Kolmogorov Stokes number Re^-1/2
  RT dm_max;
  RT inv_dm;   // 1 / dm_max (0 when grouping is off)
  RT k0;
  uint32_t flags;
  int32_t kernel;
};

template <typename RT>
__host__ __device__ inline PairConst<RT> make_pair_const(const Model &P, const Gas &g) {
  PairConst<RT> c;
  c.cBM = (RT)(8.0 * kBoltz * g.T / kPi);
  c.Vg2 = (RT)g.Vg2;
  c.St_eta = (RT)g.St_eta;
  c.dm_max = (RT)P.dm_max;
  c.inv_dm = P.dm_max > 0.0 ? (RT)(1.0 / P.dm_max) : (RT)0;
  c.k0 = (RT)P.k0;
  c.flags = P.flags;
  c.kernel = P.kernel;
  return c;
}

// FP32 particle state of the mixed path (after a collision changed m)
// Mn: the particle's swarm mass times the cell's density factor, as the
// record holds it ((float)(M * nd_fac))
__device__ inline Rec<float> make_rec_f(const CellF &c, double m, float Mn) {
  const float mf = (float)m;
  const float a = cbrtf(mf * c.ca);
  const float ts = a < c.a_sw ? c.tE * a : c.tS * a * a;
  const float St = ts * c.Om;
  const float q1 = __builtin_amdgcn_rcpf(1.0f + St);
  const float w = __builtin_amdgcn_rcpf(1.0f + St * St);
  Rec<float> r;
  r.m = mf;
  r.im = __builtin_amdgcn_rcpf(mf);
  r.a = a * (float)kSqrtPi;
  r.St = St;
  r.ist = __builtin_amdgcn_rcpf(St);
  r.h = St * St * __builtin_amdgcn_rcpf(St + c.Ste);
  r.q1 = q1;
  r.vr = c.m2eta * St * w;
  r.vp = c.meta * w;
  r.vz = c.mzO * St * q1;
  r.nd = Mn * r.im;
  r.Mn = Mn;
  return r;
}

// precision-specific division and square root: FP64 correctly rounded;
// FP32 through the hardware reciprocal and square root (about 1 ulp)
__device__ inline double pdiv(double a, double b) { return a / b; }
__device__ inline float pdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double prcp(double b) { return 1.0 / b; }
__device__ inline float prcp(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ inline double psqrt(double x) { return sqrt(x); }
__device__ inline float psqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// turbulent relative velocity squared (Ormel & Cuzzi 2007 closed forms)
template <typename RT>
__device__ inline RT dv2_turb(const PairConst<RT> &c, const Rec<RT> &x, const Rec<RT> &y) {
  const bool xb = x.St > y.St;
  const RT St1 = xb ? x.St : y.St, St2 = xb ? y.St : x.St;
  if (St1 < c.St_eta) {
    const RT h1 = xb ? x.h : y.h, h2 = xb ? y.h : x.h;
    return pdiv(c.Vg2 * (St1 - St2), St1 + St2) * (h1 - h2);
  }
  if (St1 < (RT)1) {
    const RT eps = pdiv(St2, St1);
    const RT br = (RT)(2.0 * kYa) - ((RT)1 + eps) +
                  pdiv((RT)2, (RT)1 + eps) *
                      ((RT)(1.0 / (1.0 + kYa)) + pdiv(eps * eps * eps, (RT)kYa + eps));
    return c.Vg2 * St1 * br;
  }
  return c.Vg2 * (x.q1 + y.q1);
}

// relative velocity of the pair (five sources in quadrature)
template <typename RT>
__device__ inline RT rel_velocity(const PairConst<RT> &c, const Rec<RT> &x, const Rec<RT> &y) {
  RT dv2 = (RT)0;
  if (c.flags & DV_BROWNIAN) dv2 += c.cBM * (x.im + y.im);
  if (c.flags & DV_TURB) dv2 += dv2_turb(c, x, y);
  if (c.flags & DV_RADIAL) {
    const RT d = x.vr - y.vr;
    dv2 += d * d;
  }
  if (c.flags & DV_AZIMUTHAL) {
    const RT d = x.vp - y.vp;
    dv2 += d * d;
  }
  if (c.flags & DV_SETTLING) {
    const RT d = x.vz - y.vz;
    dv2 += d * d;
  }
  return psqrt(dv2);
}

// symmetric collision kernel K_xy; dv receives the relative velocity
template <typename RT>
__device__ inline RT pair_kernel(const PairConst<RT> &c, const Rec<RT> &x, const Rec<RT> &y,
                                 RT &dv) {
  if (c.kernel == K_CONSTANT) {
    dv = (RT)0;
    return c.k0;
  }
  if (c.kernel == K_LINEAR) {
    dv = (RT)0;
    return c.k0 * (x.m + y.m);
  }
  dv = rel_velocity(c, x, y);
  const RT s = x.a + y.a;
  if (sizeof(RT) == 4) return s * s * dv;  // the FP32 radii carry sqrt(pi)
  return (RT)kPi * s * s * dv;
}

// FP32 rates of a pair for the physical kernel with all five velocity
// sources: r_xy = n_y K_xy / max(1, dm m_x/m_y) and r_yx, and the relative
// velocity.  Same quantities as rel_velocity / pair_kernel / swarm_rate,
// arranged for few instructions: the Ormel & Cuzzi regimes evaluated
// branch-free from eps = St2/St1 with one shared reciprocal of
// (1 + eps)(y_a + eps) -- (St1 - St2)/(St1 + St2) = (1 - eps)/(1 + eps) and
// 2/(1 + eps) (1/(1 + y_a) + eps^3/(y_a + eps)) =
// 2 ((y_a + eps)/(1 + y_a) + eps^3) / ((1 + eps)(y_a + eps)) --, fused
// multiply-adds for the quadrature sum, sqrt(pi) folded into the radii.
__device__ inline void pair_rates_all(const PairConst<float> &c, const Rec<float> &x,
                                      const Rec<float> &y, float &dv, float &rxy, float &ryx) {
  constexpr float ya = (float)kYa;
  constexpr float c1 = (float)(1.0 / (1.0 + kYa));
  constexpr float b0 = (float)(2.0 * kYa - 1.0);
  // h and q1 in registers before the arithmetic: otherwise their loads are
  // deferred into the regime choice, a second wait on LDS per pair
  asm volatile("" ::"v"(x.h), "v"(x.q1), "v"(y.h), "v"(y.q1));
  float dv2 = c.cBM * (x.im + y.im);
  const bool xb = x.St > y.St;
  const float St1 = xb ? x.St : y.St;
  const float ist1 = xb ? x.ist : y.ist;
  // h = St^2 / (St + St_eta) grows with St: the larger-St particle has the larger h
  const float hd = fabsf(x.h - y.h);
  const float eps = (xb ? y.St : x.St) * ist1;
  const float ye = ya + eps;
  const float rd = __builtin_amdgcn_rcpf((1.0f + eps) * ye);
  const float tiny = (1.0f - eps) * (ye * rd) * hd;
  const float inter = St1 * (b0 - eps + 2.0f * rd * fmaf(ye, c1, eps * eps * eps));
  const float heavy = x.q1 + y.q1;
  // the regime is chosen by selects, not branches: the two candidate values
  // pass through an empty asm so that the optimizer cannot sink their
  // arithmetic into per-regime blocks (which serialise a wave's pairs)
  float tn = tiny, it = inter;
  asm("" : "+v"(tn), "+v"(it));
  const float turb = St1 < c.St_eta ? tn : (St1 < 1.0f ? it : heavy);
  dv2 = fmaf(c.Vg2, turb, dv2);
  float d = x.vr - y.vr;
  dv2 = fmaf(d, d, dv2);
  d = x.vp - y.vp;
  dv2 = fmaf(d, d, dv2);
  d = x.vz - y.vz;
  dv2 = fmaf(d, d, dv2);
  dv = __builtin_amdgcn_sqrtf(dv2);
  const float s = x.a + y.a;
  const float K = s * s * dv;
  rxy = y.nd * K;
  ryx = x.nd * K;
  if (c.dm_max > 0.0f) {
    rxy *= fminf(1.0f, y.m * (x.im * c.inv_dm));
    ryx *= fminf(1.0f, x.m * (y.im * c.inv_dm));
  }
}

// rate of representative particle x against swarm y given K_xy:
// n_y K / max(1, dm_max m_x / m_y)
__device__ inline double swarm_rate(const PairConst<double> &c, const Rec<double> &x,
                                    const Rec<double> &y, double K) {
  double r = y.nd * K;
  if (c.dm_max > 0.0) {
    const double grp = c.dm_max * x.m / y.m;
    if (grp > 1.0) r = r / grp;
  }
  return r;
}
// FP32: the same factor as n_y K min(1, m_y / (dm_max m_x)), no reciprocal
__device__ inline float swarm_rate(const PairConst<float> &c, const Rec<float> &x,
                                   const Rec<float> &y, float K) {
  float r = y.nd * K;
  if (c.dm_max > 0.0f) r *= fminf(1.0f, y.m * (x.im * c.inv_dm));
  return r;
}

// fragment mass: inverse-CDF draw from the mass-weighted distribution
// ~ m^(-5/6) (number slope 11/6) on [lo, hi]
__host__ __device__ inline double frag_draw(double lo, double hi, double u) {
  if (!(hi > lo)) return lo;
  const double slo = sqrt(cbrt(lo)), shi = sqrt(cbrt(hi));
  const double x = slo + u * (shi - slo);
  const double x2 = x * x;
  return x2 * x2 * x2;
}

// probability that a collision at mean relative velocity dv fragments (or
// erodes): linear ramp from (1 - w) v_frag to v_frag, or the tail above
// v_frag of the Maxwell speed distribution with mean dv (scale a =
// dv sqrt(pi/8)): erfc(x) + 2/sqrt(pi) x exp(-x^2), x = v_frag / (sqrt(2) a)
// in the precision T of dv (double for the FP64 form, float for the mixed one)
template <typename PP, typename T>
__host__ __device__ inline T frag_probability(const PP &P, T dv) {
  const T vf = (T)P.v_frag;
  if (P.frag_mode == FRAG_RAMP) {
    const T lo = ((T)1 - (T)P.frag_width) * vf;
    if (dv <= lo) return (T)0;
    if (dv >= vf) return (T)1;
    return (dv - lo) / (vf - lo);
  }
  if (P.frag_mode == FRAG_MAXWELL) {
    if (!(dv > (T)0)) return (T)0;
    const T x = (T)2 * vf / (sqrt((T)kPi) * dv);
    return erfc(x) + (T)2 / sqrt((T)kPi) * x * exp(-x * x);
  }
  return dv < vf ? (T)0 : (T)1;
}

// grouping factor max(1, dm_max m_i / m_j)
__host__ __device__ inline double group_factor(double dm_max, double mi, double mj) {
  if (!(dm_max > 0.0)) return 1.0;
  const double g = dm_max * mi / mj;
  return g < 1.0 ? 1.0 : g;
}

// collision outcome for representative particle i (mass mi) hitting a body
// of swarm j (mass mj) at relative velocity dv; returns the outcome code.
// EXACT: the grouped mass grp * mj and the mass-ratio test as written (the
// FP64 path); otherwise their division-free equivalents max(mj, dm_max mi)
// and big >= ratio * small, equal up to one rounding (the mixed path)
template <bool EXACT = true, typename PP>
__host__ __device__ inline int outcome(const PP &P, bool fast, double mi, double mj, double u,
                                       double &m_new) {
  // grouped mass grp * mj; the eroded mass chi grp mj
  double gm, em;
  if (EXACT) {
    const double grp = group_factor(P.dm_max, mi, mj);
    gm = grp * mj;
    em = P.erosion_chi * grp * mj;
  } else {
    const double d = P.dm_max * mi;
    gm = (P.dm_max > 0.0 && d > mj) ? d : mj;
    em = P.erosion_chi * gm;
  }
  if (P.kernel != K_PHYSICAL || !fast) {
    m_new = mi + gm;
    return OUT_STICK;
  }
  const double big = mi > mj ? mi : mj;
  const double small = mi > mj ? mj : mi;
  if (EXACT ? big / small >= P.erosion_ratio : big >= P.erosion_ratio * small) {
    if (mi >= mj) {
      const double m = mi - em;
      m_new = m > P.m0 ? m : P.m0;
      return OUT_ERODE;
    }
    m_new = frag_draw(P.m0, mi, u);
    return OUT_ERODED_SMALL;
  }
  m_new = frag_draw(P.m0, big, u);
  return OUT_FRAG;
}

}  // namespace mcd
