// collide.hip -- launches of the collision kernels (collide_device.hpp):
// the batched persistent launch, one workgroup per cell, and the test path
// that writes one cell's full rate matrix.
//
// The batched kernel of the mixed form without the composition mix and the
// event log (the form of runs that track neither) is instantiated in
// collide_ilp.hip, compiled with the scheduling strategy that maximises
// instruction-level parallelism: its four-wave teams and lone cells wait
// less on dependencies.  It comes in two instantiations, one for either
// event budget and one for fixed event counts only (no waiting times); the
// FP64 form's kernel without them is instantiated there for fixed counts
// too.  The variant with the composition mix keeps the default schedule,
// under which it spills less.
#include <algorithm>

#include "collide_device.hpp"

namespace mcd {

// defined in collide_ilp.hip
extern template __global__ void collide_batched<float, 4, true, false, false>(CollideArgs A);
extern template __global__ void collide_batched<float, 4, true, false, false, kFixedCount>(
    CollideArgs A);
extern template __global__ void collide_batched<double, 4, false, false, false, kFixedCount>(
    CollideArgs A);

__global__ void reset_queues(DevState *st) {
  st->big_head = 0;
  st->small_head = 0;
}

// ---------------------------------------------------------------------------
// test path: the full rate matrix of one cell, from the same records and
// pair code as the collision kernel
// ---------------------------------------------------------------------------
template <typename RT, bool FAST>
__global__ __launch_bounds__(256) void rates_cell(CollideArgs A, int cell, double *r_out,
                                                  int64_t ld, double *rowsum) {
  if (A.plan->bad) return;
  const int s0 = A.cell_start[cell];
  const int n = A.cell_start[cell + 1] - s0;
  Gas g;
  gas_from_primaries(A.P, A.gas + (size_t)cell * 6, g);
  const PairConst<RT> pc = make_pair_const<RT>(A.P, g);
  double scale = 1.0;
  if (sizeof(RT) == 4) {
    double ndmax = 0.0;
    for (int k = 0; k < n; ++k) {
      const int p = A.order[s0 + k];
      ndmax = fmax(ndmax, A.M[p] / (A.m[p] * g.V));
    }
    int e2 = 0;
    frexp(ndmax, &e2);
    scale = ldexp(1.0, -e2);
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int pi = A.order[s0 + i];
    const Rec<RT> ri = make_rec<RT>(A.P, g, A.m[pi], A.M[pi], scale);
    RT acc = (RT)0;
    for (int k = 0; k < n; ++k) {
      const int pk = A.order[s0 + k];
      const Rec<RT> rk = make_rec<RT>(A.P, g, A.m[pk], A.M[pk], scale);
      RT dv, x, y;
      PairEval<RT, FAST>::run(pc, ri, rk, dv, x, y);
      acc += x;
      r_out[(int64_t)i * ld + k] = (double)x / scale;
    }
    if (rowsum) rowsum[i] = (double)acc / scale;
  }
}

// ---------------------------------------------------------------------------
template <typename Kern>
static hipError_t prepare(Kern kern, size_t lds) {
  if (lds > 64 * 1024)
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
  return hipSuccess;
}

template <typename RT, int KMAX, bool FAST, bool PROB>
static hipError_t run_batched(const CollideArgs &a, int grid_override, hipStream_t s) {
  const size_t lds = std::max(region_bytes<RT>(a.big_cap, 4), 4 * region_bytes<RT>(a.small_cap, 1));
  // the composition mix and the event log only where they are used
  const bool aux = (a.comp != nullptr && a.P.n_comp > 0) || a.evlog != nullptr;
  auto kern = aux ? collide_batched<RT, KMAX, FAST, PROB, true>
                  : collide_batched<RT, KMAX, FAST, PROB, false>;
  // the kernels without them of the mixed form's fast path and of the FP64
  // form (up to 4 slots per lane) also come without waiting times, for fixed
  // event counts
  if constexpr (KMAX == 4 && !PROB && (sizeof(RT) == 8 || FAST))
    if (!aux && !(a.dt > 0.0)) kern = collide_batched<RT, KMAX, FAST, PROB, false, kFixedCount>;
  hipError_t e = prepare(kern, lds);
  int dev = 0, cus = 0, per_cu = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  // persistent workgroups: as many as fit (the list lengths are on the
  // device; workgroups beyond the work exit at their first queue pop)
  int grid = per_cu * cus;
  if (grid_override > 0) grid = grid_override;
  reset_queues<<<1, 1, 0, s>>>(a.state);
  kern<<<grid, 256, lds, s>>>(a);
  return hipGetLastError();
}

template <typename RT, int KMAX, bool FAST, bool PROB>
static hipError_t run_plain(const CollideArgs &a, int n_cells, hipStream_t s) {
  const size_t lds = region_bytes<RT>(a.big_cap, 4);
  auto kern = collide_plain<RT, KMAX, FAST, PROB>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  if (n_cells > 0) kern<<<n_cells, 256, lds, s>>>(a);
  return hipGetLastError();
}

// the FP32 fast pair path applies to the physical kernel with all five
// velocity sources (the benchmark disk); everything else takes the generic one
static bool fast_path(const CollideArgs &a, int precision) {
  const uint32_t all = DV_BROWNIAN | DV_TURB | DV_RADIAL | DV_AZIMUTHAL | DV_SETTLING;
  return precision != 0 && a.P.kernel == K_PHYSICAL && (a.P.flags & all) == all;
}

template <bool PROB>
static hipError_t launch_collide_t(const CollideArgs &a, int precision, int schedule, int n_cells,
                                   bool wide, int grid_override, hipStream_t s) {
  const bool fast = fast_path(a, precision);
  if (schedule == 0) {
    if (precision == 0)
      return wide ? run_plain<double, 8, false, PROB>(a, n_cells, s)
                  : run_plain<double, 4, false, PROB>(a, n_cells, s);
    if (fast)
      return wide ? run_plain<float, 8, true, PROB>(a, n_cells, s)
                  : run_plain<float, 4, true, PROB>(a, n_cells, s);
    return wide ? run_plain<float, 8, false, PROB>(a, n_cells, s)
                : run_plain<float, 4, false, PROB>(a, n_cells, s);
  }
  if (precision == 0)
    return wide ? run_batched<double, 8, false, PROB>(a, grid_override, s)
                : run_batched<double, 4, false, PROB>(a, grid_override, s);
  if (fast)
    return wide ? run_batched<float, 8, true, PROB>(a, grid_override, s)
                : run_batched<float, 4, true, PROB>(a, grid_override, s);
  return wide ? run_batched<float, 8, false, PROB>(a, grid_override, s)
              : run_batched<float, 4, false, PROB>(a, grid_override, s);
}

hipError_t launch_collide(const CollideArgs &a, int precision, int schedule, int n_cells,
                          int max_cell, int grid_override, hipStream_t s) {
  // slots per lane: four-wave teams hold big_cap particles, single waves
  // small_cap; kernels exist for up to 4 and up to 8
  const int k_big = (a.big_cap + 255) / 256, k_small = (a.small_cap + 63) / 64;
  const int kneed = schedule == 0 ? std::max(k_big, (max_cell + 255) / 256) : std::max(k_big, k_small);
  if (kneed > 8) return hipErrorInvalidValue;
  const bool wide = kneed > 4;
  // the probabilistic fragmentation criteria apply only to the physical kernel
  const bool prob = a.P.frag_mode != FRAG_SHARP && a.P.kernel == K_PHYSICAL;
  return prob ? launch_collide_t<true>(a, precision, schedule, n_cells, wide, grid_override, s)
              : launch_collide_t<false>(a, precision, schedule, n_cells, wide, grid_override, s);
}

hipError_t launch_rates_cell(const CollideArgs &a, int precision, int cell, double *r_out,
                             int64_t ld, double *rowsum_out, hipStream_t s) {
  if (precision == 0)
    rates_cell<double, false><<<1, 256, 0, s>>>(a, cell, r_out, ld, rowsum_out);
  else if (fast_path(a, precision))
    rates_cell<float, true><<<1, 256, 0, s>>>(a, cell, r_out, ld, rowsum_out);
  else
    rates_cell<float, false><<<1, 256, 0, s>>>(a, cell, r_out, ld, rowsum_out);
  return hipGetLastError();
}

}  // namespace mcd
