// noalloc.hip -- one collision step over explicit cells without a context
// or a workspace, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops).  The device counters, the plan and
// the batched cell lists that a context keeps in its workspace live here in
// one file-scope device array, `scratch`, of fixed size; every call on a GPU
// reuses that GPU's copy.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "mcd.h"

using namespace mcd;

namespace {

constexpr int kNoallocMaxCells = 1 << 20;   // cells of one call
constexpr int kNoallocSmallMax = 256;       // single-wave threshold of a fresh context
constexpr size_t kA = 256;

constexpr size_t up(size_t x) { return (x + kA - 1) / kA * kA; }

// offsets of the arrays in the scratch array
constexpr size_t kOffState = 0;
constexpr size_t kOffPlan = kOffState + up(sizeof(DevState));
constexpr size_t kOffHist = kOffPlan + up(sizeof(Plan));
constexpr size_t kOffCursor = kOffHist + up(kPlanBuckets * sizeof(uint32_t));
constexpr size_t kOffBig = kOffCursor + up(kPlanBuckets * sizeof(uint32_t));
constexpr size_t kOffSmall = kOffBig + up((size_t)kNoallocMaxCells * sizeof(int32_t));
constexpr size_t kScratchBytes = kOffSmall + up((size_t)kNoallocMaxCells * sizeof(int32_t));
static_assert(kScratchBytes == MCD_NOALLOC_SCRATCH_BYTES, "the header states the scratch size");

constexpr int kMaxDevices = 64;

}  // namespace

// the fixed scratch memory: each GPU the library runs on holds one copy
// until the process ends.  Host code reaches it only through the device
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};
thread_local std::string g_err;

mcd_status fail(mcd_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

// the current device's copy of the scratch array, looked up once per device
mcd_status scratch_address(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(MCD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(MCD_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MCD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = (char *)g_scratch[dev];
  return MCD_OK;
}

__global__ void k_counts_out(const DevState *st, int64_t *out) {
  out[0] = (int64_t)st->events;
  for (int k = 0; k < 4; ++k) out[1 + k] = (int64_t)st->outcomes[k];
  out[5] = (int64_t)st->flags;
}

}  // namespace

namespace mcd {
const char *contextless_error() { return g_err.empty() ? "null context" : g_err.c_str(); }
}  // namespace mcd

extern "C" mcd_status mcd_collide_noalloc(const mcd_params *params, const mcd_particles *particles,
                                          const mcd_cells *cells, double dt, int64_t max_events,
                                          uint32_t step, void *hip_stream, int64_t *counts) {
  g_err.clear();
  if (!params || !particles || !cells) return fail(MCD_EINVAL, "params, particles and cells are needed");
  const std::string why = check_params(*params);
  if (!why.empty()) return fail(MCD_EINVAL, why);
  const mcd_particles &p = *particles;
  if (p.n <= 0 || p.n >= (int64_t)1 << 31 || !p.m || !p.M)
    return fail(MCD_EINVAL, "particles need 1 <= n < 2^31, m and M");
  if (params->n_comp > 0 && !p.comp) return fail(MCD_EINVAL, "comp must be given when n_comp > 0");
  if (cells->n_cells < 1 || cells->n_cells > kNoallocMaxCells)
    return fail(MCD_EINVAL, "n_cells must be in [1, " + std::to_string(kNoallocMaxCells) +
                                "]: the fixed scratch holds the lists of that many cells");
  if (!cells->cell_start || !cells->order || !cells->gas)
    return fail(MCD_EINVAL, "cell_start, order and gas are needed");
  if (cells->max_cell < 1 || cells->max_cell > kMaxCell)
    return fail(MCD_EINVAL, "max_cell must be in [1, " + std::to_string(kMaxCell) + "]");
  if (!(std::isfinite(dt) && dt >= 0.0) || max_events < 0 || max_events >= ((int64_t)1 << 32))
    return fail(MCD_EINVAL, "dt >= 0 and 0 <= max_events < 2^32");
  if (!(dt > 0.0) && max_events == 0) return fail(MCD_EINVAL, "set a time limit dt > 0 or max_events > 0");
  const int precision = params->precision, schedule = params->schedule;
  const int bound = cells->max_cell;
  const bool big = bound > kNoallocSmallMax;
  int big_cap = 0, small_cap = 0;
  if (!lds_caps(precision, schedule, big ? bound : 0, big ? kNoallocSmallMax : bound, bound,
                big_cap, small_cap))
    return fail(MCD_EINVAL, "cells of max_cell particles do not fit the 160 KB LDS in this precision"
                            " (at most " + std::to_string(precision == MCD_FP64 ? kMaxCellFp64 : kMaxCell) + ")");
  char *sc = nullptr;
  mcd_status st = scratch_address(&sc);
  if (st != MCD_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  DevState *state = (DevState *)(sc + kOffState);
  PlanBuffers pb;
  pb.plan = (Plan *)(sc + kOffPlan);
  pb.hist = (uint32_t *)(sc + kOffHist);
  pb.cursor = (uint32_t *)(sc + kOffCursor);
  pb.big = (int32_t *)(sc + kOffBig);
  pb.small = (int32_t *)(sc + kOffSmall);
  // the previous call's counters and plan are cleared by a kernel (no memset
  // node, so that the call can be captured in a graph)
  hipError_t e = launch_clear_state(state, pb.plan, step, s);
  if (e == hipSuccess)
    e = launch_plan_explicit(cells->cell_start, cells->order, cells->n_cells, p.n, bound,
                             kNoallocSmallMax, pb, state, s);
  if (e == hipSuccess && (params->flags & COAG)) {
    CollideArgs a{};
    a.P = make_model(*params);
    a.cell_start = cells->cell_start;
    a.order = cells->order;
    a.gas = cells->gas;
    a.big_list = pb.big;
    a.small_list = pb.small;
    a.plan = pb.plan;
    a.big_cap = big_cap;
    a.small_cap = small_cap;
    a.m = p.m;
    a.M = p.M;
    a.comp = params->n_comp > 0 ? p.comp : nullptr;
    a.N = p.n;
    a.dt = dt;
    a.max_events = max_events;
    a.state = state;
    a.evlog = nullptr;
    a.log_per_cell = 0;
    a.rowsum_dump = nullptr;
    e = launch_collide(a, precision, schedule, cells->n_cells, bound, 0, s);
  }
  if (e == hipSuccess && counts) {
    k_counts_out<<<1, 1, 0, s>>>(state, counts);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(MCD_EHIP, std::string("mcd_collide_noalloc: ") + hipGetErrorString(e));
  return MCD_OK;
}
