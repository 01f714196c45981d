// diagnostics.hip -- sigma_d(m, r), the dust surface density per particle
// mass bin and radius (paper, Benchmark: the run's output is the dust surface
// density as a function of particle mass and distance from the star).
//
// Bins are half-open, r_edges[k] <= r < r_edges[k+1] and m_edges[l] <= m <
// m_edges[l+1], found by binary search on the edges (comparisons only, so a
// particle's bin does not depend on rounding).  Each active particle in range
// adds its swarm mass M to bin (k, l); each bin is then divided by its
// annulus area pi (r_edges[k+1]^2 - r_edges[k]^2) (1 in column mode, where M
// is per unit area).  Up to 4096 bins a workgroup accumulates its
// contiguous range of particles in LDS and flushes its nonzero bins with
// global atomics; beyond that every particle adds to global memory directly.  The FP64 sums therefore follow the order
// of the atomics.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace mcd {

constexpr int kHistLdsBins = 4096;
constexpr int kHistLdsEdges = 1024;

__device__ inline int find_bin(const double *e, int n, double x) {
  if (!(x >= e[0]) || !(x < e[n])) return -1;
  int lo = 0, hi = n;  // e[lo] <= x < e[hi]
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (x < e[mid])
      hi = mid;
    else
      lo = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_hist_clear(double *sigma, uint32_t *count, int64_t nb) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    sigma[b] = 0.0;
    if (count) count[b] = 0u;
  }
}

// Workgroup b takes the contiguous particle range [b chunk, (b+1) chunk):
// particles stored roughly by radius then touch few bins per workgroup, which
// keeps the flush short.  Edges are staged in LDS when they fit.
template <bool LDS>
__global__ __launch_bounds__(256) void k_hist(const double *__restrict__ r,
                                              const double *__restrict__ m,
                                              const double *__restrict__ M,
                                              const uint8_t *__restrict__ active, int64_t N,
                                              int64_t chunk, const double *re, int n_rb,
                                              const double *me, int n_mb, double *sigma,
                                              uint32_t *count) {
  __shared__ double ls[LDS ? kHistLdsBins : 1];
  __shared__ uint32_t lc[LDS ? kHistLdsBins : 1];
  __shared__ double le[kHistLdsEdges];
  const int nb = n_rb * n_mb;
  const bool edges_lds = n_rb + n_mb + 2 <= kHistLdsEdges;
  if (edges_lds) {
    for (int k = threadIdx.x; k <= n_rb; k += blockDim.x) le[k] = re[k];
    for (int k = threadIdx.x; k <= n_mb; k += blockDim.x) le[n_rb + 1 + k] = me[k];
  }
  if (LDS) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      ls[b] = 0.0;
      lc[b] = 0u;
    }
  }
  __syncthreads();
  const double *er = edges_lds ? le : re;
  const double *em = edges_lds ? le + n_rb + 1 : me;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < N ? i0 + chunk : N;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    if (!active[i]) continue;
    const int k = find_bin(er, n_rb, r[i]);
    const int l = find_bin(em, n_mb, m[i]);
    if (k < 0 || l < 0) continue;
    const int b = k * n_mb + l;
    if (LDS) {
      unsafeAtomicAdd(&ls[b], M[i]);
      atomicAdd(&lc[b], 1u);
    } else {
      unsafeAtomicAdd(&sigma[b], M[i]);
      if (count) atomicAdd(&count[b], 1u);
    }
  }
  if (LDS) {
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      if (lc[b]) {
        unsafeAtomicAdd(&sigma[b], ls[b]);
        if (count) atomicAdd(&count[b], lc[b]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_hist_area(double *sigma, const double *re, int n_rb,
                                                   int n_mb, int column) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (int64_t)n_rb * n_mb) return;
  const int k = (int)(b / n_mb);
  const double area = column ? 1.0 : kPi * (re[k + 1] * re[k + 1] - re[k] * re[k]);
  sigma[b] /= area;
}

hipError_t launch_sigma_hist(const double *r, const double *m, const double *M,
                             const uint8_t *active, int64_t N, const double *re, int n_rb,
                             const double *me, int n_mb, int column, double *sigma,
                             uint32_t *count, int cus, hipStream_t s) {
  const int64_t nb = (int64_t)n_rb * n_mb;
  const unsigned gb = (unsigned)std::min<int64_t>((nb + 255) / 256, 4096);
  k_hist_clear<<<gb, 256, 0, s>>>(sigma, count, nb);
  const int64_t gp = std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, 4 * (int64_t)cus));
  const int64_t chunk = (N + gp - 1) / gp;
  if (nb <= kHistLdsBins)
    k_hist<true><<<(unsigned)gp, 256, 0, s>>>(r, m, M, active, N, chunk, re, n_rb, me, n_mb, sigma,
                                              count);
  else
    k_hist<false><<<(unsigned)gp, 256, 0, s>>>(r, m, M, active, N, chunk, re, n_rb, me, n_mb,
                                               sigma, count);
  k_hist_area<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(sigma, re, n_rb, n_mb, column);
  return hipGetLastError();
}

}  // namespace mcd
