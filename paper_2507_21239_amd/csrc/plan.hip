// plan.hip -- the cell lists of the batched collision launch, planned on the
// device from the grid's member ranges: validation of an explicit grid, then
// a counting sort of the cells by particle count (largest first) into the
// list of four-wave teams (cells above small_max particles) and the list of
// single waves (1..small_max particles).  Equal-sized cells may come in any
// order: cells are independent and their results do not depend on their
// place in a list, only on their team shape.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace mcd {

constexpr int kPlanThreads = 256;

__global__ void k_plan_clear(Plan *plan, uint32_t *hist, DevState *st) {
  for (int b = threadIdx.x; b < kPlanBuckets; b += blockDim.x) hist[b] = 0u;
  if (threadIdx.x == 0) {
    *plan = Plan{};
    st->flags &= ~(uint32_t)FLAG_BAD_GRID;  // a new grid replaces the old one's validation result
  }
}

// per cell: size check (cell_start non-decreasing from >= 0, no cell above
// `bound`) and its count in the size histogram; per member: index in
// [0, N).  Block-private histograms in LDS, flushed with global atomics.
__global__ __launch_bounds__(kPlanThreads) void k_plan_count(const int32_t *__restrict__ cs,
                                                             const int32_t *__restrict__ order,
                                                             int32_t nc, int64_t N, int32_t bound,
                                                             uint32_t *hist, Plan *plan,
                                                             DevState *st) {
  __shared__ uint32_t h[kPlanBuckets];
  __shared__ int s_bad, s_max;
  for (int b = threadIdx.x; b < kPlanBuckets; b += blockDim.x) h[b] = 0u;
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_max = 0;
  }
  __syncthreads();
  const int32_t c0 = cs[0];
  const int32_t cn = cs[nc];
  int bad = (c0 < 0 || cn < c0) ? 1 : 0;
  int mx = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
    const int32_t sz = cs[c + 1] - cs[c];
    if (sz < 0 || sz > bound) {
      bad = 1;
      continue;
    }
    mx = sz > mx ? sz : mx;
    atomicAdd(&h[sz], 1u);
  }
  if (!bad && c0 >= 0) {
    for (int64_t k = (int64_t)c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cn; k += stride) {
      const int32_t p = order[k];
      if (p < 0 || (int64_t)p >= N) bad = 1;
    }
  }
  if (bad) atomicOr(&s_bad, 1);
  atomicMax(&s_max, mx);
  __syncthreads();
  for (int b = threadIdx.x; b < kPlanBuckets; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
  if (threadIdx.x == 0) {
    atomicMax(&plan->max_cell, s_max);
    if (s_bad) {
      atomicOr(&plan->bad, 1);
      atomicOr(&st->flags, FLAG_BAD_GRID);
    }
    if (blockIdx.x == 0) {
      plan->n_members = (c0 >= 0 && cn >= c0) ? cn - c0 : 0;
      st->n_active = plan->n_members;
    }
  }
}

// exclusive offsets of the size classes, largest size first: the big list
// takes sizes above small_max, the small list 1..small_max (positions in
// the small list start at n_big, the scatter subtracts it); size 0 is left
// out.  One workgroup of 1024 threads, a scan over the 2049 buckets in LDS.
__global__ __launch_bounds__(1024) void k_plan_offsets(const uint32_t *__restrict__ hist,
                                                       int32_t small_max, uint32_t *cursor,
                                                       Plan *plan) {
  constexpr int kPer = (kPlanBuckets + 1023) / 1024;  // buckets per thread
  __shared__ uint32_t tot[1024];
  __shared__ uint32_t s_big;
  const int t = threadIdx.x;
  if (t == 0) s_big = 0u;
  // thread t takes descending-size positions d = t*kPer .. t*kPer+kPer-1,
  // size = kMaxCell - d; size 0 (d = kMaxCell) counts nowhere
  uint32_t v[kPer];
  uint32_t sum = 0, nbig = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int d = t * kPer + e;
    const int size = kMaxCell - d;
    v[e] = (d < kMaxCell) ? hist[size] : 0u;
    sum += v[e];
    nbig += size > small_max ? v[e] : 0u;
  }
  tot[t] = sum;
  __syncthreads();
  if (nbig) atomicAdd(&s_big, nbig);
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
    const uint32_t x = t >= off ? tot[t - off] : 0u;
    __syncthreads();
    tot[t] += x;
    __syncthreads();
  }
  uint32_t run = tot[t] - sum;  // exclusive prefix of this thread's buckets
  int my_big = 0, my_small = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int d = t * kPer + e;
    const int size = kMaxCell - d;
    if (d < kMaxCell) {
      cursor[size] = run;
      if (v[e]) {
        if (size > small_max)
          my_big = size > my_big ? size : my_big;
        else
          my_small = size > my_small ? size : my_small;
      }
    }
    run += v[e];
  }
  if (my_big) atomicMax(&plan->max_big, my_big);
  if (my_small) atomicMax(&plan->max_small, my_small);
  if (t == 0) {
    const uint32_t total = tot[1023];
    const bool bad = plan->bad != 0;
    plan->n_big = bad ? 0 : (int32_t)s_big;
    plan->n_small = bad ? 0 : (int32_t)(total - s_big);
  }
}

// every occupied cell to its list position: a block reserves a range per
// size bucket with one global atomic, its cells take consecutive places
__global__ __launch_bounds__(kPlanThreads) void k_plan_scatter(const int32_t *__restrict__ cs,
                                                               int32_t nc, int32_t small_max,
                                                               uint32_t *cursor, const Plan *plan,
                                                               int32_t *big, int32_t *small) {
  __shared__ uint32_t h[kPlanBuckets];
  if (plan->bad) return;
  for (int b = threadIdx.x; b < kPlanBuckets; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const int64_t chunk = (int64_t)blockDim.x * 4;
  const int n_big = plan->n_big;
  for (int64_t c00 = (int64_t)blockIdx.x * chunk; c00 < nc; c00 += (int64_t)gridDim.x * chunk) {
    int32_t cell[4], sz[4];
    uint32_t rank[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t c = c00 + e * blockDim.x + threadIdx.x;
      cell[e] = c < nc ? (int32_t)c : -1;
      sz[e] = c < nc ? cs[c + 1] - cs[c] : 0;
      rank[e] = sz[e] > 0 ? atomicAdd(&h[sz[e]], 1u) : 0u;
    }
    __syncthreads();
    // one reservation per bucket with members in this chunk
    for (int b = threadIdx.x; b < kPlanBuckets; b += blockDim.x)
      if (h[b]) h[b] = atomicAdd(&cursor[b], h[b]);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (sz[e] <= 0) continue;
      const uint32_t pos = h[sz[e]] + rank[e];
      if (sz[e] > small_max)
        big[pos] = cell[e];
      else
        small[pos - n_big] = cell[e];
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kPlanBuckets; b += blockDim.x) h[b] = 0u;
    __syncthreads();
  }
}

// a grid whose cells all have (at most) the same size: every cell in index
// order into one list
__global__ __launch_bounds__(kPlanThreads) void k_plan_uniform(int32_t nc, int32_t size,
                                                               int32_t small_max, Plan *plan,
                                                               int32_t *big, int32_t *small) {
  const bool to_big = size > small_max;
  int32_t *dst = to_big ? big : small;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x)
    dst[c] = (int32_t)c;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Plan p{};
    p.n_big = to_big ? nc : 0;
    p.n_small = to_big ? 0 : nc;
    p.max_big = to_big ? size : 0;
    p.max_small = to_big ? 0 : size;
    p.max_cell = size;
    *plan = p;
  }
}

__global__ void k_clear_state(DevState *st, Plan *plan, uint32_t step) {
  DevState z{};
  z.step = step;
  *st = z;
  *plan = Plan{};
}

hipError_t launch_clear_state(DevState *state, Plan *plan, uint32_t step, hipStream_t s) {
  k_clear_state<<<1, 1, 0, s>>>(state, plan, step);
  return hipGetLastError();
}

hipError_t launch_plan_explicit(const int32_t *cell_start, const int32_t *order, int32_t nc,
                                int64_t N, int32_t bound, int32_t small_max, PlanBuffers pb,
                                DevState *state, hipStream_t s) {
  if (nc < 1 || bound < 0 || bound > kMaxCell) return hipErrorInvalidValue;
  const unsigned g = (unsigned)std::min<int64_t>(1024, ((int64_t)nc + kPlanThreads - 1) / kPlanThreads);
  k_plan_clear<<<1, 256, 0, s>>>(pb.plan, pb.hist, state);
  k_plan_count<<<std::max(g, 64u), kPlanThreads, 0, s>>>(cell_start, order, nc, N, bound, pb.hist,
                                                         pb.plan, state);
  k_plan_offsets<<<1, 1024, 0, s>>>(pb.hist, small_max, pb.cursor, pb.plan);
  const unsigned gs = (unsigned)std::min<int64_t>(1024, ((int64_t)nc + 4 * kPlanThreads - 1) / (4 * kPlanThreads));
  k_plan_scatter<<<gs, kPlanThreads, 0, s>>>(cell_start, nc, small_max, pb.cursor, pb.plan, pb.big,
                                             pb.small);
  return hipGetLastError();
}

hipError_t launch_plan_uniform(int32_t nc, int32_t size, int32_t small_max, PlanBuffers pb,
                               hipStream_t s) {
  if (nc < 1) return hipErrorInvalidValue;
  const unsigned g = (unsigned)std::min<int64_t>(1024, ((int64_t)nc + kPlanThreads - 1) / kPlanThreads);
  k_plan_uniform<<<g, kPlanThreads, 0, s>>>(nc, size, small_max, pb.plan, pb.big, pb.small);
  return hipGetLastError();
}

}  // namespace mcd
