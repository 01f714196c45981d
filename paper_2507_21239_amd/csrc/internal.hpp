// internal.hpp -- launch arguments and device state shared by the kernels
// and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.hpp"

namespace mcd {

// device-resident state: everything a replayed graph must see change
struct DevState {
  uint32_t step;          // global step index (Philox counter word 2)
  uint32_t flags;         // sticky anomaly bits
  int32_t n_active;       // active particles after binning
  int32_t big_head;       // persistent work queues
  int32_t small_head;
  int32_t pad0;
  double t_sim;           // simulated time
  unsigned long long events;
  unsigned long long outcomes[4];
};

enum : uint32_t {
  FLAG_BAD_RATE = 1u << 0,   // NaN / inf rate sum
  FLAG_BAD_MASS = 1u << 1,   // non-positive or non-finite mass produced
  FLAG_BAD_VOLUME = 1u << 2, // non-positive cell volume with members
  FLAG_CAPACITY = 1u << 3,   // cell larger than the launch's capacity
  FLAG_BAD_GRID = 1u << 4,   // explicit grid failed validation (nothing collides)
};

// largest cell any schedule takes, and the buckets of the size histogram
constexpr int kMaxCell = 2048;
constexpr int kPlanBuckets = kMaxCell + 1;

// the cell lists of the batched launch, written by the planning kernels
struct Plan {
  int32_t n_big, n_small;      // list lengths
  int32_t max_big, max_small;  // largest cell of each list
  int32_t max_cell;            // largest cell of the grid
  int32_t n_members;           // members of the grid
  int32_t bad;                 // nonzero: the grid failed validation (empty lists)
  int32_t pad;
};

struct PlanBuffers {
  Plan *plan;
  int32_t *big, *small;        // [cells] each
  uint32_t *hist, *cursor;     // [kPlanBuckets] each
};

struct CollideArgs {
  Model P;
  const int32_t *cell_start;
  const int32_t *order;
  const double *gas;        // [n_cells][6]
  const int32_t *big_list;  // cells processed by four-wave teams, largest first
  const int32_t *small_list;// cells processed by single waves, largest first
  const Plan *plan;         // list lengths (device), grid validation result
  int32_t big_cap, small_cap;   // particle capacity of a team's LDS region
  double *m;
  const double *M;
  float *comp;
  int64_t N;
  double dt;
  int64_t max_events;
  DevState *state;
  int32_t *evlog;
  int64_t log_per_cell;
  double *rowsum_dump;  // test path: starting row sums written here, no events
};

// a selection result: payloads of the chosen slot, its slot and team lane
struct Cand {
  double p0, p1;
  int q, lane, hit, gi;
};

// team scratch after a region's particle records: wave totals, selection
// candidates (double-buffered), the cell's gas state and the outcome
// parameters
struct TeamScratch {
  double tot[2][8];
  Cand cand[2][4];
  Gas gas;
  CellF cf;
  OutcomeConst oc;
};

// LDS bytes of one particle record in rate precision RT
template <typename RT>
constexpr size_t rec_bytes() {
  return 12 * sizeof(RT);
}

// partner-sum exchange of a four-wave FP32 team's row-sum build:
// [wave][lane] pairs of floats (two slots per round), after the team scratch.
// 2 KB keeps a 1024-particle team region within the LDS of four 256-particle
// one-wave regions, so the exchange costs no occupancy
constexpr size_t kXbufBytes = 4 * 64 * 2 * sizeof(float);

// byte offset of the exchange buffer in a team region holding `cap` particles
template <typename RT>
constexpr size_t xbuf_offset(int cap) {
  return ((size_t)cap * rec_bytes<RT>() + sizeof(TeamScratch) + 15) / 16 * 16;
}

// LDS bytes of one team region holding `cap` particles (16-byte multiple);
// four-wave FP32 teams add the exchange buffer
template <typename RT>
constexpr size_t region_bytes(int cap, int waves) {
  return xbuf_offset<RT>(cap) + (sizeof(RT) == 4 && waves == 4 ? kXbufBytes : 0);
}

// largest FP64 cell: a four-wave team's region of 96-byte records and its
// scratch must fit the 160 KB of LDS (the FP32 form's 48-byte records fit
// kMaxCell)
constexpr int kMaxCellFp64 = 1536;
static_assert(region_bytes<double>(kMaxCellFp64, 4) <= 160 * 1024, "FP64 cells of kMaxCellFp64 fit");
static_assert(region_bytes<double>(kMaxCellFp64 + 256, 4) > 160 * 1024, "and no larger ones");
static_assert(region_bytes<float>(kMaxCell, 4) <= 160 * 1024, "FP32 cells of kMaxCell fit");

// zero the device state and the plan (a new context, or a context-free
// step), with the Philox step index `step`
hipError_t launch_clear_state(DevState *state, Plan *plan, uint32_t step, hipStream_t s);

// LDS capacities of the collision launch from the largest cell of each list
// (particles): false if a team's region does not fit the 160 KB of LDS
inline bool lds_caps(int precision, int schedule, int max_big, int max_small, int max_cell,
                     int &big_cap, int &small_cap) {
  big_cap = max_big > 0 ? (max_big + 255) / 256 * 256 : 0;
  small_cap = (max_small + 63) / 64 * 64;
  if (small_cap < 64) small_cap = 64;
  const int plain_cap = (max_cell + 255) / 256 * 256;
  if (schedule == 0) big_cap = plain_cap > 256 ? plain_cap : 256;  // one team per cell
  const bool f64 = precision == 0;
  const size_t lds_big = f64 ? region_bytes<double>(big_cap, 4) : region_bytes<float>(big_cap, 4);
  const size_t lds_small =
      4 * (f64 ? region_bytes<double>(small_cap, 1) : region_bytes<float>(small_cap, 1));
  const size_t lds = schedule == 0 ? lds_big : (lds_big > lds_small ? lds_big : lds_small);
  return lds <= 160 * 1024;
}

}  // namespace mcd

#include <string>

#include "mcd.h"

namespace mcd {

// parameter checks ("" if valid) and the device model of a parameter set
// (capi.hip), shared by the context and the context-free entry point
std::string check_params(const mcd_params &p);
Model make_model(const mcd_params &p);
// message of the last failed context-free call on this thread
// (noalloc.hip), or "null context"
const char *contextless_error();

// planning of the batched lists (plan.hip): an explicit grid is validated
// (member ranges, cells of at most `bound` particles, member indices below
// N) and its cells sorted by size; a uniform grid takes every cell in order
hipError_t launch_plan_explicit(const int32_t *cell_start, const int32_t *order, int32_t nc,
                                int64_t N, int32_t bound, int32_t small_max, PlanBuffers pb,
                                DevState *state, hipStream_t s);
hipError_t launch_plan_uniform(int32_t nc, int32_t size, int32_t small_max, PlanBuffers pb,
                               hipStream_t s);

// launchers (collide.hip)
hipError_t launch_collide(const CollideArgs &a, int precision, int schedule, int n_cells,
                          int max_cell, int grid_override, hipStream_t s);
hipError_t launch_rates_cell(const CollideArgs &a, int precision, int cell, double *r_out,
                             int64_t ld, double *rowsum_out, hipStream_t s);
// transport (transport.hip)
hipError_t launch_transport(const Model &P, double *r, double *z, const double *m,
                            uint8_t *active, int64_t N, double dt, DevState *state,
                            hipStream_t s);
hipError_t launch_finish_step(DevState *state, double dt, hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n,
                         hipStream_t s);

// binning (binning.hip)
// active count and range of the IEEE bit patterns of r
struct BinState {
  uint64_t min_bits, max_bits;
  uint32_t count, pad;
};

// zones up to this many members are ordered by z in one workgroup (bitonic
// network of 1024 threads x 8 elements, 96 KB of LDS); larger zones take the
// global radix path
constexpr int kZoneSortMax = 8192;
// workgroups of the first reduction over r (partials of 3 words each)
constexpr int kMinmaxParts = 1024;

struct BinBuffers {
  uint64_t *keys[2];   // 64-bit keys of the global z path
  uint32_t *k32[2];    // 32-bit keys of the r sort
  int32_t *vals[2];
  uint8_t *flag;       // neighbours with equal r keys but different r
  BinState *bs;
  uint64_t *part;      // [3 kMinmaxParts] partial {min, max, count}
  int32_t *by_r;       // active particle indices by ascending (r, index)
  int32_t *zone;       // zone of every particle (n_r for inactive)
  uint32_t *hist;      // radix histogram [256][tiles]
  uint32_t *digit_tot; // [256]
  int64_t cap;         // particles
  int32_t tiles;
};
// sigma_d(m, r) histogram of the particles (diagnostics.hip)
hipError_t launch_sigma_hist(const double *r, const double *m, const double *M,
                             const uint8_t *active, int64_t N, const double *re, int n_rb,
                             const double *me, int n_mb, int column, double *sigma,
                             uint32_t *count, int cus, hipStream_t s);

hipError_t launch_binning(const Model &P, int n_r, int n_z, const double *r, const double *z,
                          const uint8_t *active, int64_t N, BinBuffers &b, int32_t *cell_start,
                          int32_t *order, double *geom, double *gas, DevState *state,
                          hipStream_t s);
int radix_tiles(int64_t n);

}  // namespace mcd
