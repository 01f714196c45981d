// capi.hip -- the C ABI declared in include/mcd.h: argument validation, the
// caller's workspace, cell schedules, the step loop and its HIP-graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "mcd.h"

using namespace mcd;

namespace {

constexpr int kSmallLimit = 512;      // largest single-wave cell a schedule may choose
constexpr size_t kAlign = 256;        // alignment of every workspace array
constexpr int64_t kMaxEdges = 1 << 16;  // histogram edges held in the workspace
constexpr uint32_t kKnownFlags = DV_BROWNIAN | DV_TURB | DV_RADIAL | DV_AZIMUTHAL | DV_SETTLING |
                                 TR_DRIFT | TR_SETTLE | TR_MIX_R | TR_MIX_Z | COAG;

// byte offsets of the workspace arrays (mcd_workspace_size, mcd_init)
struct Layout {
  size_t state, sbak, plan;                   // DevState, its tuning backup, Plan
  size_t cs, order, gas, geom;                // the adaptive grid
  size_t big, small, hist, cursor;            // cell lists and their planning
  size_t mbak, cbak;                          // tuning backups of m and comp
  size_t edges;                               // histogram edges
  size_t k32[2], vals[2], flag, bs, part, by_r, hist_r, digit, k64[2], zone;  // binning
  size_t total;
  int64_t cells_adaptive, cells_cap;
  int tiles;
  bool global_z;
};

Layout layout_for(const mcd_params &p, int64_t N) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
    return o;
  };
  const int64_t na = (int64_t)p.n_r * p.n_z;
  L.cells_adaptive = na;
  L.cells_cap = std::max<int64_t>(std::max<int64_t>(na, p.max_cells), 1);
  const size_t n = (size_t)N;
  L.state = take(sizeof(DevState));
  L.sbak = take(sizeof(DevState));
  L.plan = take(sizeof(Plan));
  L.cs = take(((size_t)na + 1) * sizeof(int32_t));
  L.order = take(n * sizeof(int32_t));
  L.gas = take((size_t)na * MCD_GAS_FIELDS * sizeof(double));
  L.geom = take((size_t)na * MCD_GEOM_FIELDS * sizeof(double));
  L.big = take((size_t)L.cells_cap * sizeof(int32_t));
  L.small = take((size_t)L.cells_cap * sizeof(int32_t));
  L.hist = take(kPlanBuckets * sizeof(uint32_t));
  L.cursor = take(kPlanBuckets * sizeof(uint32_t));
  L.mbak = take(n * sizeof(double));
  L.cbak = take((size_t)p.n_comp * n * sizeof(float));
  L.edges = take((size_t)kMaxEdges * sizeof(double));
  L.tiles = radix_tiles(N);
  for (int k = 0; k < 2; ++k) {
    L.k32[k] = take(n * sizeof(uint32_t));
    L.vals[k] = take(n * sizeof(int32_t));
  }
  L.flag = take(n);
  L.bs = take(sizeof(BinState));
  L.part = take((size_t)3 * kMinmaxParts * sizeof(uint64_t));
  L.by_r = take(n * sizeof(int32_t));
  L.hist_r = take((size_t)256 * L.tiles * sizeof(uint32_t));
  L.digit = take(256 * sizeof(uint32_t));
  // zones above the LDS zone sort take the global radix path by z
  L.global_z = p.n_r >= 1 && (N + p.n_r - 1) / p.n_r > kZoneSortMax;
  if (L.global_z) {
    L.k64[0] = take(n * sizeof(uint64_t));
    L.k64[1] = take(n * sizeof(uint64_t));
    L.zone = take(n * sizeof(int32_t));
  }
  L.total = off + kAlign;  // room to align the caller's base address
  return L;
}

}  // namespace

struct mcd_ctx {
  mcd_params prm{};
  Model model{};
  mcd_particles part{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  Layout L{};
  char *ws = nullptr;           // the caller's workspace, aligned
  bool adaptive = false, have_cells = false;
  int32_t n_cells = 0;
  // the grid in use: the library's adaptive grid or the caller's explicit one
  const int32_t *cell_start = nullptr, *order = nullptr;
  const double *gas = nullptr;
  int32_t *g_cell_start = nullptr, *g_order = nullptr;  // adaptive grid (workspace)
  double *g_gas = nullptr, *g_geom = nullptr;
  // largest cell: the bound the caps follow (adaptive: the floor rule's;
  // explicit: the caller's, or measured when the caller gave none)
  int32_t bound = 0;
  bool exact = false;           // explicit grid without a bound: caps from measured sizes
  int32_t max_big = 0, max_small = 0, max_cell = 0;
  int big_cap = 0, small_cap = 0;
  PlanBuffers pb{};
  BinBuffers bb{};
  DevState *d_state = nullptr;
  int32_t *evlog = nullptr;
  int64_t log_per_cell = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool g_valid = false;
  double g_dt = 0.0;
  int64_t g_max = 0;
  // schedule of the batched launch (set by mcd_tune): cells up to small_max
  // particles run on one wave, larger ones on four-wave teams; grid_per_cu
  // persistent workgroups per compute unit (0: as many as fit)
  int small_max = 256;
  int grid_per_cu = 0;
  int cus = 0;
  // snapshots: two device staging buffers filled in stream order, each
  // copied to the caller's host memory on copy_stream
  hipStream_t copy_stream = nullptr;
  char *d_stage[2] = {nullptr, nullptr};
  size_t stage_cap = 0;
  hipEvent_t ev_staged[2] = {nullptr, nullptr}, ev_landed[2] = {nullptr, nullptr};
  bool slot_used[2] = {false, false};
  int64_t snap_count = 0;
  double *d_grid = nullptr;     // gridded gas: lr, zn, lrho, lT, lA, lS back to back
  std::vector<double> h_grid;
  std::vector<double> h_edges;  // histogram bin edges (host copy, read by the async upload)
  double *d_edges = nullptr;    // workspace
  double *d_mbak = nullptr;     // tuning backups of m, comp and the device state (workspace)
  float *d_cbak = nullptr;
  DevState *d_sbak = nullptr;
  std::string err;
};

namespace {

mcd_status fail(mcd_ctx *c, mcd_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

mcd_status hip_fail(mcd_ctx *c, hipError_t e, const char *what) {
  return fail(c, MCD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define MCD_HIP(c, expr)                                \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(c, _e, #expr); \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T));
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

bool pos_finite(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

namespace mcd {

std::string check_params(const mcd_params &p) {
  const struct {
    const char *name;
    double v;
  } positive[] = {{"sigma_g0", p.sigma_g0}, {"T0", p.T0}, {"a_mono", p.a_mono},
                  {"rho_s", p.rho_s},       {"mu", p.mu}, {"m_star", p.m_star},
                  {"r_ref", p.r_ref},       {"v_frag", p.v_frag}};
  for (const auto &f : positive)
    if (!pos_finite(f.v)) return std::string(f.name) + " must be finite and > 0";
  if (!std::isfinite(p.p) || !std::isfinite(p.q)) return "p and q must be finite";
  if (!(std::isfinite(p.alpha) && p.alpha >= 0.0)) return "alpha must be finite and >= 0";
  if (!(std::isfinite(p.erosion_ratio) && p.erosion_ratio >= 1.0)) return "erosion_ratio must be >= 1";
  if (!(std::isfinite(p.dm_max) && p.dm_max >= 0.0 && p.dm_max < 1.0)) return "dm_max must be in [0, 1)";
  if (!(std::isfinite(p.erosion_chi) && p.erosion_chi >= 0.0)) return "erosion_chi must be >= 0";
  if (!(std::isfinite(p.r_in) && p.r_in >= 0.0)) return "r_in must be >= 0";
  if (!(std::isfinite(p.k0) && p.k0 >= 0.0)) return "k0 must be >= 0";
  if (p.column && !pos_finite(p.r_col)) return "r_col must be > 0 in column mode";
  if (p.kernel < MCD_K_PHYSICAL || p.kernel > MCD_K_LINEAR) return "unknown kernel";
  if (p.n_r < 1 || p.n_z < 1) return "n_r and n_z must be >= 1";
  if ((int64_t)p.n_r * p.n_z > (1 << 24)) return "too many cells";
  if (p.max_cells < 0 || p.max_cells > (1 << 24)) return "max_cells must be in [0, 2^24]";
  if (p.flags & ~kKnownFlags) return "unknown flag bits";
  if (p.n_comp < 0 || p.n_comp > MCD_MAX_COMP) return "n_comp must be in [0, 8]";
  if (p.precision != MCD_FP64 && p.precision != MCD_MIXED) return "unknown precision";
  if (p.schedule != MCD_SCHED_PLAIN && p.schedule != MCD_SCHED_BATCHED) return "unknown schedule";
  if (p.frag_mode != MCD_FRAG_SHARP && p.frag_mode != MCD_FRAG_RAMP && p.frag_mode != MCD_FRAG_MAXWELL)
    return "unknown frag_mode";
  if (p.frag_mode == MCD_FRAG_RAMP && !(p.frag_width > 0.0 && p.frag_width <= 1.0))
    return "frag_width must be in (0, 1] for the ramp";
  return "";
}

Model make_model(const mcd_params &p) {
  Model m{};
  m.sigma_g0 = p.sigma_g0;
  m.T0 = p.T0;
  m.p = p.p;
  m.q = p.q;
  m.alpha = p.alpha;
  m.v_frag = p.v_frag;
  m.erosion_ratio = p.erosion_ratio;
  m.rho_s = p.rho_s;
  m.mu = p.mu;
  m.m_star = p.m_star;
  m.r_ref = p.r_ref;
  m.dm_max = p.dm_max;
  m.erosion_chi = p.erosion_chi;
  m.r_in = p.r_in;
  m.r_col = p.r_col;
  m.k0 = p.k0;
  m.m0 = 4.0 / 3.0 * kPi * p.a_mono * p.a_mono * p.a_mono * p.rho_s;  // monomer mass
  m.flags = p.flags;
  m.kernel = p.kernel;
  m.column = p.column;
  m.n_comp = p.n_comp;
  m.frag_mode = p.frag_mode;
  m.frag_width = p.frag_width;
  m.key0 = (uint32_t)p.seed;
  m.key1 = (uint32_t)(p.seed >> 32);
  return m;
}

}  // namespace mcd

namespace {

void drop_graph(mcd_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->g_valid = false;
}

// carve the arrays of the layout out of the (aligned) workspace
void carve(mcd_ctx *c) {
  const Layout &L = c->L;
  char *w = c->ws;
  c->d_state = (DevState *)(w + L.state);
  c->d_sbak = (DevState *)(w + L.sbak);
  c->pb.plan = (Plan *)(w + L.plan);
  c->g_cell_start = (int32_t *)(w + L.cs);
  c->g_order = (int32_t *)(w + L.order);
  c->g_gas = (double *)(w + L.gas);
  c->g_geom = (double *)(w + L.geom);
  c->pb.big = (int32_t *)(w + L.big);
  c->pb.small = (int32_t *)(w + L.small);
  c->pb.hist = (uint32_t *)(w + L.hist);
  c->pb.cursor = (uint32_t *)(w + L.cursor);
  c->d_mbak = (double *)(w + L.mbak);
  c->d_cbak = c->prm.n_comp > 0 ? (float *)(w + L.cbak) : nullptr;
  c->d_edges = (double *)(w + L.edges);
  BinBuffers &b = c->bb;
  for (int k = 0; k < 2; ++k) {
    b.k32[k] = (uint32_t *)(w + L.k32[k]);
    b.vals[k] = (int32_t *)(w + L.vals[k]);
    b.keys[k] = L.global_z ? (uint64_t *)(w + L.k64[k]) : nullptr;
  }
  b.flag = (uint8_t *)(w + L.flag);
  b.bs = (BinState *)(w + L.bs);
  b.part = (uint64_t *)(w + L.part);
  b.by_r = (int32_t *)(w + L.by_r);
  b.zone = L.global_z ? (int32_t *)(w + L.zone) : nullptr;
  b.hist = (uint32_t *)(w + L.hist_r);
  b.digit_tot = (uint32_t *)(w + L.digit);
  b.cap = c->part.n;
  b.tiles = L.tiles;
}

// LDS region capacities of the batched (or plain) launch from the largest
// cell of each list; EINVAL if a region does not fit the LDS
mcd_status set_caps(mcd_ctx *c, int32_t max_big, int32_t max_small, int32_t max_cell) {
  c->max_big = max_big;
  c->max_small = max_small;
  c->max_cell = max_cell;
  const bool f64 = c->prm.precision == MCD_FP64;
  if (!lds_caps(c->prm.precision, c->prm.schedule, max_big, max_small, max_cell, c->big_cap,
                c->small_cap))
    return fail(c, MCD_EINVAL,
                std::string("largest cell does not fit the 160 KB LDS in this precision (") +
                    std::to_string(max_cell) + " particles; at most " +
                    std::to_string(f64 ? kMaxCellFp64 : kMaxCell) + ")");
  return MCD_OK;
}

// plan the batched lists for the current grid and schedule on the device
// (in stream order: work already queued still sees the old lists); the caps
// follow the bound, or the measured sizes (one synchronisation) when the
// caller of an explicit grid gave no bound
mcd_status plan_lists(mcd_ctx *c) {
  hipError_t e;
  if (c->adaptive) {
    e = launch_plan_uniform(c->n_cells, c->bound, c->small_max, c->pb, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "planning the cell lists");
    const bool big = c->bound > c->small_max;
    return set_caps(c, big ? c->bound : 0, big ? 0 : c->bound, c->bound);
  }
  e = launch_plan_explicit(c->cell_start, c->order, c->n_cells, c->part.n,
                           c->exact ? kMaxCell : c->bound, c->small_max, c->pb, c->d_state,
                           c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "planning the cell lists");
  if (!c->exact) {
    const bool big = c->bound > c->small_max;
    return set_caps(c, big ? c->bound : 0, std::min(c->bound, c->small_max), c->bound);
  }
  Plan pl{};
  MCD_HIP(c, hipMemcpyAsync(&pl, c->pb.plan, sizeof(Plan), hipMemcpyDeviceToHost, c->stream));
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  if (pl.bad)
    return fail(c, MCD_EINVAL,
                "explicit cells rejected: cell_start must start >= 0 and not decrease, no cell "
                "may exceed 2048 particles and every member index must be in [0, N)");
  return set_caps(c, pl.max_big, pl.max_small, pl.max_cell);
}

CollideArgs collide_args(mcd_ctx *c, double dt, int64_t max_events) {
  CollideArgs a{};
  a.P = c->model;
  a.cell_start = c->cell_start;
  a.order = c->order;
  a.gas = c->gas;
  a.big_list = c->pb.big;
  a.small_list = c->pb.small;
  a.plan = c->pb.plan;
  a.big_cap = c->big_cap;
  a.small_cap = c->small_cap;
  a.m = c->part.m;
  a.M = c->part.M;
  a.comp = c->part.comp;
  a.N = c->part.n;
  a.dt = dt;
  a.max_events = max_events;
  a.state = c->d_state;
  a.evlog = c->evlog;
  a.log_per_cell = c->log_per_cell;
  a.rowsum_dump = nullptr;
  return a;
}

bool transport_on(const mcd_ctx *c) {
  return (c->prm.flags & (TR_DRIFT | TR_SETTLE | TR_MIX_R | TR_MIX_Z)) != 0;
}

mcd_status enqueue_bin(mcd_ctx *c, hipStream_t s) {
  hipError_t e = launch_binning(c->model, c->prm.n_r, c->prm.n_z, c->part.r, c->part.z,
                                c->part.active, c->part.n, c->bb, c->g_cell_start, c->g_order,
                                c->g_geom, c->g_gas, c->d_state, s);
  if (e != hipSuccess) return hip_fail(c, e, "binning");
  return MCD_OK;
}

mcd_status enqueue_step(mcd_ctx *c, double dt, int64_t max_events, hipStream_t s) {
  mcd_status st;
  if (c->adaptive && (st = enqueue_bin(c, s)) != MCD_OK) return st;
  if (c->prm.flags & COAG) {
    hipError_t e = launch_collide(collide_args(c, dt, max_events), c->prm.precision,
                                  c->prm.schedule, c->n_cells, c->max_cell,
                                  c->grid_per_cu * c->cus, s);
    if (e != hipSuccess) return hip_fail(c, e, "collide");
  }
  if (c->adaptive && transport_on(c)) {
    hipError_t e = launch_transport(c->model, c->part.r, c->part.z, c->part.m, c->part.active,
                                    c->part.n, dt, c->d_state, s);
    if (e != hipSuccess) return hip_fail(c, e, "transport");
  }
  hipError_t e = launch_finish_step(c->d_state, dt, s);
  if (e != hipSuccess) return hip_fail(c, e, "finish_step");
  return MCD_OK;
}

std::string why_params(const mcd_params *params, const mcd_particles *particles) {
  if (!params || !particles) return "params and particles must not be NULL";
  std::string why = check_params(*params);
  const mcd_particles &p = *particles;
  if (why.empty()) {
    if (p.n <= 0 || p.n >= (int64_t)1 << 31) why = "particle count must be in [1, 2^31)";
    else if (!p.r || !p.z || !p.m || !p.M || !p.active) why = "particle arrays must not be NULL";
    else if (params->n_comp > 0 && !p.comp) why = "comp must be given when n_comp > 0";
  }
  return why;
}

}  // namespace

extern "C" {

mcd_status mcd_workspace_size(const mcd_params *params, int64_t n, size_t *bytes) {
  if (!params || !bytes || n <= 0 || n >= (int64_t)1 << 31) return MCD_EINVAL;
  if (!check_params(*params).empty()) return MCD_EINVAL;
  *bytes = layout_for(*params, n).total;
  return MCD_OK;
}

mcd_status mcd_init(const mcd_params *params, const mcd_particles *particles, void *hip_stream,
                    void *workspace, size_t ws_bytes, mcd_ctx **out) {
  if (!out) return MCD_EINVAL;
  if (!why_params(params, particles).empty()) return MCD_EINVAL;
  const Layout L = layout_for(*params, particles->n);
  if (!workspace || ws_bytes < L.total) return MCD_EINVAL;
  mcd_ctx *c = new (std::nothrow) mcd_ctx();
  if (!c) return MCD_ENOMEM;
  c->prm = *params;
  c->model = make_model(*params);
  c->part = *particles;
  if (params->n_comp == 0) c->part.comp = nullptr;
  c->stream = (hipStream_t)hip_stream;
  c->L = L;
  c->ws = (char *)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign);
  carve(c);
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = launch_clear_state(c->d_state, c->pb.plan, 0u, c->stream);
  int dev = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    mcd_free(c);
    return MCD_EHIP;
  }
  *out = c;
  return MCD_OK;
}

mcd_status mcd_bin(mcd_ctx *c, const mcd_cells *cells) {
  if (!c) return MCD_EINVAL;
  if (!cells && c->adaptive && c->have_cells) {
    // re-binning on the same grid: the cell lists, buffers and any captured
    // step graph stay valid; only the binning kernels are enqueued
    return enqueue_bin(c, c->stream);
  }
  drop_graph(c);
  if (!cells) {
    const int64_t N = c->part.n;
    const int nr = c->prm.n_r, nz = c->prm.n_z;
    if ((int64_t)nr * nz > N) return fail(c, MCD_EINVAL, "n_r * n_z exceeds the particle count");
    const int64_t zone_max = (N + nr - 1) / nr;
    const int32_t cell_max = (int32_t)((zone_max + nz - 1) / nz);
    if (cell_max > kMaxCell)
      return fail(c, MCD_EINVAL, "cells would exceed " + std::to_string(kMaxCell) +
                                     " particles; use more cells");
    c->adaptive = true;
    c->have_cells = false;
    c->n_cells = nr * nz;
    c->cell_start = c->g_cell_start;
    c->order = c->g_order;
    c->gas = c->g_gas;
    // equal-count cells differ by at most one particle: one class, bounded
    // by the floor rule's largest cell
    c->bound = cell_max;
    c->exact = false;
    mcd_status st;
    if ((st = plan_lists(c)) != MCD_OK) return st;
    if ((st = enqueue_bin(c, c->stream)) != MCD_OK) return st;
    c->have_cells = true;
    return MCD_OK;
  }
  // explicit cells: non-owning views, validated and planned on the device
  const int32_t nc = cells->n_cells;
  if (nc < 1 || !cells->cell_start || !cells->order || !cells->gas)
    return fail(c, MCD_EINVAL, "explicit cells need n_cells >= 1 and device arrays");
  if ((int64_t)nc > c->L.cells_cap)
    return fail(c, MCD_EINVAL, "n_cells exceeds the workspace's cells (" +
                                   std::to_string(c->L.cells_cap) + "; set max_cells)");
  if (cells->max_cell < 0 || cells->max_cell > kMaxCell)
    return fail(c, MCD_EINVAL, "max_cell must be in [0, " + std::to_string(kMaxCell) + "]");
  c->adaptive = false;
  c->have_cells = false;
  c->n_cells = nc;
  c->cell_start = cells->cell_start;
  c->order = cells->order;
  c->gas = cells->gas;
  c->bound = cells->max_cell;
  c->exact = cells->max_cell == 0;
  mcd_status st = plan_lists(c);
  if (st != MCD_OK) return st;
  c->have_cells = true;
  return MCD_OK;
}

mcd_status mcd_rates(mcd_ctx *c, int32_t cell, double *r_out, int64_t ld, double *rowsum_out) {
  if (!c) return MCD_EINVAL;
  if (!c->have_cells) return fail(c, MCD_ESTATE, "mcd_rates before mcd_bin");
  if (cell < 0 || cell >= c->n_cells || !r_out) return fail(c, MCD_EINVAL, "bad cell or r_out");
  int32_t se[2];
  Plan pl{};
  MCD_HIP(c, hipMemcpyAsync(se, c->cell_start + cell, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                            c->stream));
  MCD_HIP(c, hipMemcpyAsync(&pl, c->pb.plan, sizeof(Plan), hipMemcpyDeviceToHost, c->stream));
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  if (pl.bad) return fail(c, MCD_EINVAL, "the explicit grid failed validation");
  if (ld < se[1] - se[0]) return fail(c, MCD_EINVAL, "ld smaller than the cell size");
  hipError_t e = launch_rates_cell(collide_args(c, 0.0, 0), c->prm.precision, cell, r_out, ld,
                                   rowsum_out, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "rates");
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  return MCD_OK;
}

mcd_status mcd_row_sums(mcd_ctx *c, double *out) {
  if (!c || !out) return MCD_EINVAL;
  if (!c->have_cells) return fail(c, MCD_ESTATE, "mcd_row_sums before mcd_bin");
  CollideArgs a = collide_args(c, 0.0, 1);
  a.evlog = nullptr;
  a.rowsum_dump = out;
  hipError_t e = launch_collide(a, c->prm.precision, c->prm.schedule, c->n_cells, c->max_cell,
                                c->grid_per_cu * c->cus, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "row sums");
  return MCD_OK;
}

mcd_status mcd_step(mcd_ctx *c, double dt, int64_t max_events, int32_t n_steps) {
  if (!c) return MCD_EINVAL;
  if (!c->have_cells) return fail(c, MCD_ESTATE, "mcd_step before mcd_bin");
  if (!(std::isfinite(dt) && dt >= 0.0) || max_events < 0 || n_steps < 0)
    return fail(c, MCD_EINVAL, "dt, max_events and n_steps must be >= 0");
  if (!(dt > 0.0) && max_events == 0)
    return fail(c, MCD_EINVAL, "set a time limit dt > 0 or max_events > 0");
  if (max_events >= ((int64_t)1 << 32)) return fail(c, MCD_EINVAL, "max_events must be < 2^32");
  if (c->adaptive && transport_on(c) && !(dt > 0.0))
    return fail(c, MCD_EINVAL, "transport needs dt > 0");
  if (n_steps == 0) return MCD_OK;
  const bool use_graph = c->prm.schedule == MCD_SCHED_BATCHED && n_steps > 1;
  if (!use_graph) {
    for (int32_t k = 0; k < n_steps; ++k) {
      mcd_status st = enqueue_step(c, dt, max_events, c->stream);
      if (st != MCD_OK) return st;
    }
    return MCD_OK;
  }
  if (!c->g_valid || c->g_dt != dt || c->g_max != max_events) {
    drop_graph(c);
    MCD_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    mcd_status st = enqueue_step(c, dt, max_events, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != MCD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    c->graph = g;
    MCD_HIP(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->g_valid = true;
    c->g_dt = dt;
    c->g_max = max_events;
  }
  for (int32_t k = 0; k < n_steps; ++k) MCD_HIP(c, hipGraphLaunch(c->gexec, c->stream));
  return MCD_OK;
}

mcd_status mcd_set_schedule(mcd_ctx *c, int32_t small_max, int32_t grid_per_cu) {
  if (!c) return MCD_EINVAL;
  if (small_max < 0 || small_max > kSmallLimit || grid_per_cu < 0 || grid_per_cu > 64)
    return fail(c, MCD_EINVAL, "small_max must be in [0, 512], grid_per_cu in [0, 64]");
  const int sm0 = c->small_max, g0 = c->grid_per_cu;
  c->small_max = small_max;
  c->grid_per_cu = grid_per_cu;
  if (c->have_cells) {
    mcd_status st = plan_lists(c);
    if (st != MCD_OK) {
      const std::string why = c->err;
      c->small_max = sm0;
      c->grid_per_cu = g0;
      (void)plan_lists(c);
      c->err = why;
      return st;
    }
  }
  drop_graph(c);
  return MCD_OK;
}

mcd_status mcd_tune(mcd_ctx *c, double dt, int64_t max_events, mcd_tune_result *out) {
  if (!c || !out) return MCD_EINVAL;
  if (!c->have_cells) return fail(c, MCD_ESTATE, "mcd_tune before mcd_bin");
  if (c->prm.schedule != MCD_SCHED_BATCHED)
    return fail(c, MCD_EINVAL, "mcd_tune applies to the batched schedule");
  if (!(std::isfinite(dt) && dt >= 0.0) || max_events < 0 || max_events >= ((int64_t)1 << 32))
    return fail(c, MCD_EINVAL, "dt and max_events must be >= 0, max_events < 2^32");
  if (!(dt > 0.0) && max_events == 0)
    return fail(c, MCD_EINVAL, "set a time limit dt > 0 or max_events > 0");
  std::memset(out, 0, sizeof(*out));
  out->small_max = c->small_max;
  out->grid_per_cu = c->grid_per_cu;
  if (!(c->prm.flags & COAG)) return MCD_OK;
  const int64_t N = c->part.n;
  const size_t ncomp = c->part.comp ? (size_t)c->prm.n_comp * (size_t)N : 0;
  hipStream_t s = c->stream;
  MCD_HIP(c, hipMemcpyAsync(c->d_mbak, c->part.m, (size_t)N * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
  if (ncomp)
    MCD_HIP(c, hipMemcpyAsync(c->d_cbak, c->part.comp, ncomp * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
  MCD_HIP(c, hipMemcpyAsync(c->d_sbak, c->d_state, sizeof(DevState), hipMemcpyDeviceToDevice, s));
  auto restore = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(c->part.m, c->d_mbak, (size_t)N * sizeof(double),
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && ncomp)
      e = hipMemcpyAsync(c->part.comp, c->d_cbak, ncomp * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->d_state, c->d_sbak, sizeof(DevState), hipMemcpyDeviceToDevice, s);
    return e;
  };
  int32_t *const evlog = c->evlog;
  c->evlog = nullptr;  // trial runs leave no event log
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  hipError_t herr = hipEventCreate(&ev_a);
  if (herr == hipSuccess) herr = hipEventCreate(&ev_b);
  // the lists of the schedule in force, read back (the tuner synchronises)
  auto plan_key = [&](std::array<int, 4> &key) -> bool {
    Plan pl{};
    if (hipMemcpyAsync(&pl, c->pb.plan, sizeof(Plan), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return false;
    key = {pl.n_big, pl.n_small, c->big_cap, c->small_cap};
    return true;
  };
  // time one collision launch per configuration, state restored before each
  auto trial = [&](int sm, int gpc, double &ms) -> bool {
    c->small_max = sm;
    c->grid_per_cu = gpc;
    if (plan_lists(c) != MCD_OK) return false;  // does not fit this GPU
    for (int rep = 0; rep < 2 && herr == hipSuccess; ++rep) {
      herr = restore();
      if (herr == hipSuccess && rep == 1) herr = hipEventRecord(ev_a, s);
      if (herr == hipSuccess)
        herr = launch_collide(collide_args(c, dt, max_events), c->prm.precision, c->prm.schedule,
                              c->n_cells, c->max_cell, gpc * c->cus, s);
      if (herr == hipSuccess && rep == 1) herr = hipEventRecord(ev_b, s);
    }
    float f = 0.0f;
    if (herr == hipSuccess) herr = hipEventSynchronize(ev_b);
    if (herr == hipSuccess) herr = hipEventElapsedTime(&f, ev_a, ev_b);
    ms = f;
    ++out->trials;
    return herr == hipSuccess;
  };
  const int sm0 = c->small_max, g0 = c->grid_per_cu;
  double best = 0.0, t = 0.0;
  int best_sm = sm0, best_g = g0;
  // single-wave threshold at the full grid, then the grid at that threshold;
  // thresholds giving the same lists as one already timed are skipped
  std::vector<std::array<int, 4>> seen;
  if (trial(sm0, g0, t)) {
    best = t;
    out->ms_default = t;
    std::array<int, 4> key{};
    if (g0 == 0 && plan_key(key)) seen.push_back(key);
  }
  const int sms[] = {0, 64, 128, 192, 256, 384, 512};
  for (int sm : sms) {
    if (herr != hipSuccess) break;
    c->small_max = sm;
    if (plan_lists(c) != MCD_OK) continue;
    std::array<int, 4> key{};
    if (!plan_key(key)) break;
    if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
    seen.push_back(key);
    if (trial(sm, 0, t) && (best == 0.0 || t < best)) {
      best = t;
      best_sm = sm;
      best_g = 0;
    }
  }
  for (int gpc : {1, 2}) {
    if (herr != hipSuccess) break;
    if (trial(best_sm, gpc, t) && (best == 0.0 || t < best)) {
      best = t;
      best_g = gpc;
    }
  }
  if (ev_a) (void)hipEventDestroy(ev_a);
  if (ev_b) (void)hipEventDestroy(ev_b);
  c->evlog = evlog;
  c->small_max = best_sm;
  c->grid_per_cu = best_g;
  mcd_status st = plan_lists(c);
  if (herr == hipSuccess) herr = restore();
  if (herr == hipSuccess) herr = hipStreamSynchronize(s);
  drop_graph(c);
  if (herr != hipSuccess) return hip_fail(c, herr, "mcd_tune");
  if (st != MCD_OK) return st;
  out->small_max = best_sm;
  out->grid_per_cu = best_g;
  out->ms_best = best;
  return MCD_OK;
}

mcd_status mcd_set_gas_grid(mcd_ctx *c, const double *r_nodes, int32_t n_gr, const double *z_nodes,
                            int32_t n_gz, const double *rho, const double *T, const double *alpha) {
  if (!c) return MCD_EINVAL;
  if (!r_nodes) {  // back to the power-law disk
    MCD_HIP(c, hipStreamSynchronize(c->stream));
    dfree(c->d_grid);
    c->d_grid = nullptr;
    c->model.grid = GasGridView{};
    drop_graph(c);
    return MCD_OK;
  }
  if (n_gr < 2 || n_gz < 2 || (int64_t)n_gr * n_gz > ((int64_t)1 << 24) || !z_nodes || !rho || !T ||
      !alpha)
    return fail(c, MCD_EINVAL, "the gas grid needs n_gr, n_gz >= 2 and all node arrays");
  for (int32_t k = 0; k < n_gr; ++k)
    if (!(std::isfinite(r_nodes[k]) && r_nodes[k] > 0.0) || (k && !(r_nodes[k] > r_nodes[k - 1])))
      return fail(c, MCD_EINVAL, "r_nodes must be positive, finite and strictly increasing");
  for (int32_t l = 0; l < n_gz; ++l)
    if (!(std::isfinite(z_nodes[l]) && z_nodes[l] >= 0.0) || (l && !(z_nodes[l] > z_nodes[l - 1])))
      return fail(c, MCD_EINVAL, "z_nodes must be >= 0, finite and strictly increasing");
  const size_t nn = (size_t)n_gr * n_gz;
  for (size_t i = 0; i < nn; ++i)
    if (!(std::isfinite(rho[i]) && rho[i] > 0.0 && std::isfinite(T[i]) && T[i] > 0.0 &&
          std::isfinite(alpha[i]) && alpha[i] > 0.0))
      return fail(c, MCD_EINVAL, "rho, T and alpha must be positive and finite at every node");
  // logarithms at the nodes and the surface density of every radial node:
  // twice (z_0 rho(z_0) + trapezoids over the nodes' heights)
  const size_t total = (size_t)n_gr + n_gz + 3 * nn + n_gr;
  std::vector<double> h(total);
  double *lr = h.data(), *zn = lr + n_gr, *lrho = zn + n_gz, *lT = lrho + nn, *lA = lT + nn,
         *lS = lA + nn;
  for (int32_t k = 0; k < n_gr; ++k) lr[k] = std::log(r_nodes[k]);
  for (int32_t l = 0; l < n_gz; ++l) zn[l] = z_nodes[l];
  for (int32_t k = 0; k < n_gr; ++k) {
    double col = z_nodes[0] * rho[(size_t)k * n_gz];
    for (int32_t l = 0; l < n_gz; ++l) {
      const size_t i = (size_t)k * n_gz + l;
      lrho[i] = std::log(rho[i]);
      lT[i] = std::log(T[i]);
      lA[i] = std::log(alpha[i]);
      if (l + 1 < n_gz) col += (z_nodes[l + 1] - z_nodes[l]) * (rho[i] + rho[i + 1]) / 2.0;
    }
    lS[k] = std::log(2.0 * col);
  }
  MCD_HIP(c, hipStreamSynchronize(c->stream));  // no queued kernel reads the old grid
  dfree(c->d_grid);
  c->d_grid = nullptr;
  c->model.grid = GasGridView{};
  if (dalloc(&c->d_grid, total) != hipSuccess)
    return fail(c, MCD_ENOMEM, "device allocation of the gas grid failed");
  c->h_grid.swap(h);
  MCD_HIP(c, hipMemcpyAsync(c->d_grid, c->h_grid.data(), total * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
  GasGridView g;
  g.lr = c->d_grid;
  g.zn = g.lr + n_gr;
  g.lrho = g.zn + n_gz;
  g.lT = g.lrho + nn;
  g.lA = g.lT + nn;
  g.lS = g.lA + nn;
  g.nr = n_gr;
  g.nz = n_gz;
  c->model.grid = g;
  drop_graph(c);
  return MCD_OK;
}

mcd_status mcd_sigma_hist(mcd_ctx *c, const double *r_edges, int32_t n_rb, const double *m_edges,
                          int32_t n_mb, double *sigma, uint32_t *count) {
  if (!c) return MCD_EINVAL;
  if (!r_edges || !m_edges || !sigma || n_rb < 1 || n_mb < 1 ||
      (int64_t)n_rb * n_mb > ((int64_t)1 << 24))
    return fail(c, MCD_EINVAL, "sigma_hist needs edges, an output and 1 <= n_rb * n_mb <= 2^24");
  auto increasing = [](const double *e, int32_t n) {
    for (int32_t k = 0; k <= n; ++k) {
      if (!std::isfinite(e[k])) return false;
      if (k > 0 && !(e[k] > e[k - 1])) return false;
    }
    return true;
  };
  if (!increasing(r_edges, n_rb) || !increasing(m_edges, n_mb) || r_edges[0] < 0.0)
    return fail(c, MCD_EINVAL, "bin edges must be finite and strictly increasing, r_edges[0] >= 0");
  const size_t ne = (size_t)n_rb + 1 + (size_t)n_mb + 1;
  if ((int64_t)ne > kMaxEdges)
    return fail(c, MCD_EINVAL, "at most " + std::to_string(kMaxEdges) + " bin edges in all");
  // the previous histogram's upload must be done before its host copy is replaced
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  c->h_edges.assign(r_edges, r_edges + n_rb + 1);
  c->h_edges.insert(c->h_edges.end(), m_edges, m_edges + n_mb + 1);
  MCD_HIP(c, hipMemcpyAsync(c->d_edges, c->h_edges.data(), ne * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
  const double *re = c->d_edges, *me = c->d_edges + n_rb + 1;
  hipError_t e = launch_sigma_hist(c->part.r, c->part.m, c->part.M, c->part.active, c->part.n, re,
                                   n_rb, me, n_mb, c->prm.column ? 1 : 0, sigma, count, c->cus,
                                   c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sigma_hist");
  return MCD_OK;
}

// bytes of a snapshot of the given fields, each field padded to 16 bytes:
// r, z, m (8 N each), active (N), comp (4 n_comp N), in that order
static size_t snapshot_layout(const mcd_ctx *c, uint32_t fields, size_t off[5]) {
  const size_t N = (size_t)c->part.n;
  const size_t sz[5] = {8 * N, 8 * N, 8 * N, N,
                        c->part.comp ? 4 * (size_t)c->prm.n_comp * N : 0};
  size_t total = 0;
  for (int f = 0; f < 5; ++f) {
    off[f] = total;
    if (fields & (1u << f)) total += (sz[f] + 15) / 16 * 16;
  }
  return total;
}

mcd_status mcd_snapshot_bytes(mcd_ctx *c, uint32_t fields, size_t *bytes) {
  if (!c || !bytes) return MCD_EINVAL;
  if (fields == 0 || (fields & ~(uint32_t)MCD_SNAP_ALL))
    return fail(c, MCD_EINVAL, "snapshot fields must be a nonzero set of MCD_SNAP_* bits");
  size_t off[5];
  *bytes = snapshot_layout(c, fields, off);
  return MCD_OK;
}

mcd_status mcd_snapshot(mcd_ctx *c, uint32_t fields, void *host_dst, size_t bytes,
                        int64_t *ticket) {
  if (!c) return MCD_EINVAL;
  if (!host_dst || fields == 0 || (fields & ~(uint32_t)MCD_SNAP_ALL))
    return fail(c, MCD_EINVAL, "snapshot needs a destination and a nonzero set of MCD_SNAP_* bits");
  if ((fields & MCD_SNAP_COMP) && !c->part.comp)
    return fail(c, MCD_EINVAL, "no composition fractions to snapshot");
  size_t off[5];
  const size_t total = snapshot_layout(c, fields, off);
  if (bytes < total) return fail(c, MCD_EINVAL, "snapshot buffer too small");
  if (!c->copy_stream) {
    MCD_HIP(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
      MCD_HIP(c, hipEventCreateWithFlags(&c->ev_staged[k], hipEventDisableTiming));
      MCD_HIP(c, hipEventCreateWithFlags(&c->ev_landed[k], hipEventDisableTiming));
    }
  }
  if (total > c->stage_cap) {
    // wait until no transfer reads the old buffers, then grow them
    MCD_HIP(c, hipStreamSynchronize(c->copy_stream));
    for (int k = 0; k < 2; ++k) {
      dfree(c->d_stage[k]);
      c->d_stage[k] = nullptr;
    }
    c->stage_cap = 0;
    for (int k = 0; k < 2; ++k)
      if (dalloc(&c->d_stage[k], total) != hipSuccess)
        return fail(c, MCD_ENOMEM, "device allocation of the snapshot staging failed");
    c->stage_cap = total;
    c->slot_used[0] = c->slot_used[1] = false;
  }
  const int k = (int)(c->snap_count & 1);
  // the staging buffer of this slot must have been copied out before reuse
  if (c->slot_used[k]) MCD_HIP(c, hipStreamWaitEvent(c->stream, c->ev_landed[k], 0));
  const size_t N = (size_t)c->part.n;
  const void *src[5] = {c->part.r, c->part.z, c->part.m, c->part.active, c->part.comp};
  const size_t sz[5] = {8 * N, 8 * N, 8 * N, N,
                        c->part.comp ? 4 * (size_t)c->prm.n_comp * N : 0};
  for (int f = 0; f < 5; ++f)
    if ((fields & (1u << f)) && sz[f])
      MCD_HIP(c, hipMemcpyAsync(c->d_stage[k] + off[f], src[f], sz[f], hipMemcpyDeviceToDevice,
                                c->stream));
  MCD_HIP(c, hipEventRecord(c->ev_staged[k], c->stream));
  MCD_HIP(c, hipStreamWaitEvent(c->copy_stream, c->ev_staged[k], 0));
  MCD_HIP(c, hipMemcpyAsync(host_dst, c->d_stage[k], total, hipMemcpyDeviceToHost, c->copy_stream));
  MCD_HIP(c, hipEventRecord(c->ev_landed[k], c->copy_stream));
  c->slot_used[k] = true;
  if (ticket) *ticket = c->snap_count;
  ++c->snap_count;
  return MCD_OK;
}

mcd_status mcd_snapshot_wait(mcd_ctx *c, int64_t ticket) {
  if (!c) return MCD_EINVAL;
  if (ticket < 0 || ticket >= c->snap_count)
    return fail(c, MCD_EINVAL, "unknown snapshot ticket");
  // transfers land in order on one stream; the slot's event belongs to this
  // snapshot or to a later one, either way this snapshot has landed after it
  MCD_HIP(c, hipEventSynchronize(c->ev_landed[ticket & 1]));
  return MCD_OK;
}

mcd_status mcd_get_stats(mcd_ctx *c, mcd_stats *o) {
  if (!c || !o) return MCD_EINVAL;
  DevState s{};
  MCD_HIP(c, hipMemcpyAsync(&s, c->d_state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  std::memset(o, 0, sizeof(*o));
  o->events = (int64_t)s.events;
  for (int k = 0; k < 4; ++k) o->outcomes[k] = (int64_t)s.outcomes[k];
  o->steps = s.step;
  o->n_active = c->have_cells ? s.n_active : 0;
  o->t_sim = s.t_sim;
  o->device_flags = s.flags;
  o->n_cells = c->n_cells;
  o->max_cell = c->max_cell;
  if (s.flags) {
    char hex[16];
    std::snprintf(hex, sizeof(hex), "%x", s.flags);
    c->err = std::string("device anomaly flags 0x") + hex;
    if (s.flags & FLAG_BAD_GRID)
      c->err += ": explicit cells rejected on the device (cell_start must start >= 0 and not "
                "decrease, no cell above max_cell, member indices in [0, N)); nothing collided";
    if (s.flags & FLAG_CAPACITY) c->err += ": a cell exceeded its launch's capacity and was skipped";
    return MCD_EDEVICE;
  }
  return MCD_OK;
}

mcd_status mcd_get_cells(mcd_ctx *c, int32_t *cell_start, int32_t *order, double *geom,
                         double *gas) {
  if (!c) return MCD_EINVAL;
  if (!c->have_cells) return fail(c, MCD_ESTATE, "no grid yet");
  int32_t n_order = 0;
  MCD_HIP(c, hipMemcpyAsync(&n_order, c->cell_start + c->n_cells, sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  const size_t nc = (size_t)c->n_cells;
  if (cell_start)
    MCD_HIP(c, hipMemcpyAsync(cell_start, c->cell_start, (nc + 1) * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, c->stream));
  if (order && n_order > 0)
    MCD_HIP(c, hipMemcpyAsync(order, c->order, (size_t)n_order * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, c->stream));
  if (geom && c->adaptive)
    MCD_HIP(c, hipMemcpyAsync(geom, c->g_geom, nc * MCD_GEOM_FIELDS * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
  if (gas)
    MCD_HIP(c, hipMemcpyAsync(gas, c->gas, nc * MCD_GAS_FIELDS * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
  MCD_HIP(c, hipStreamSynchronize(c->stream));
  return MCD_OK;
}

mcd_status mcd_set_event_log(mcd_ctx *c, int32_t *buf, int64_t per_cell) {
  if (!c) return MCD_EINVAL;
  if (buf && per_cell <= 0) return fail(c, MCD_EINVAL, "per_cell must be > 0");
  c->evlog = buf;
  c->log_per_cell = buf ? per_cell : 0;
  drop_graph(c);
  return MCD_OK;
}

mcd_status mcd_philox(const uint32_t *ctr, uint32_t key_lo, uint32_t key_hi, uint32_t *out,
                      int64_t n, void *hip_stream) {
  if (n < 0 || (n > 0 && (!ctr || !out))) return MCD_EINVAL;
  hipError_t e = launch_philox(ctr, key_lo, key_hi, out, n, (hipStream_t)hip_stream);
  return e == hipSuccess ? MCD_OK : MCD_EHIP;
}

const char *mcd_last_error(const mcd_ctx *c) {
  if (!c) return mcd::contextless_error();
  return c->err.c_str();
}

void mcd_free(mcd_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  dfree(c->d_grid);
  if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
  for (int k = 0; k < 2; ++k) {
    dfree(c->d_stage[k]);
    if (c->ev_staged[k]) (void)hipEventDestroy(c->ev_staged[k]);
    if (c->ev_landed[k]) (void)hipEventDestroy(c->ev_landed[k]);
  }
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

}  // extern "C"
