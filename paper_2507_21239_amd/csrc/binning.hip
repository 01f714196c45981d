// binning.hip -- equal-count adaptive grid (paper, Summary: every cell holds
// the same number of representative particles).
//
// Radial zones: active particles ranked by (r, index), zone k holds ranks
// [floor(k Na / n_r), floor((k+1) Na / n_r)).  Cells: inside a zone, ranked
// by (z, index) and split the same way into n_z cells.  The ranking is a
// stable least-significant-digit radix sort written for wave64: 8-bit
// digits, a tile of 2048 keys per 256-thread workgroup, per-tile digit
// histograms, a scan over tiles per digit, and a stable scatter in which a
// lane finds the earlier lanes of its wave holding the same digit with eight
// ballots.  Keys are the IEEE bit patterns of the non-negative coordinates
// (order-preserving); inactive particles carry the largest key and sort
// last.  Three sorts per binning: r (8 passes), z (8 passes), then the zone
// index (1-2 passes), each stable, so ties fall back to the particle index.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace mcd {

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixThreads * kRadixItems;

int radix_tiles(int64_t n) {
  return (int)std::max<int64_t>(1, (n + kRadixTile - 1) / kRadixTile);
}

__device__ inline uint64_t key_bits(double x) {
  return (uint64_t)__double_as_longlong(x + 0.0);  // -0 -> +0
}

__global__ __launch_bounds__(256) void k_keys_from_double(const double *__restrict__ x,
                                                          const uint8_t *__restrict__ active,
                                                          int64_t N, uint64_t *keys, int32_t *vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  keys[i] = active[i] ? key_bits(x[i]) : ~0ull;
  vals[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t N,
                                                    int shift, uint32_t *hist, int tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    const int64_t i = base + it * kRadixThreads + threadIdx.x;
    if (i < N) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

__device__ inline uint32_t block_incl_scan_u32(uint32_t v, uint32_t *s) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t y = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += y;
    __syncthreads();
  }
  return s[t];
}

// exclusive scan of one digit's row of tile counts; row total -> digit_tot
__global__ __launch_bounds__(256) void k_radix_scan_rows(uint32_t *hist, int tiles,
                                                         uint32_t *digit_tot) {
  __shared__ uint32_t s[256];
  uint32_t *row = hist + (size_t)blockIdx.x * tiles;
  const int per = (tiles + 255) / 256;
  const int start = threadIdx.x * per;
  uint32_t loc = 0;
  for (int k = 0; k < per; ++k) {
    const int x = start + k;
    if (x < tiles) loc += row[x];
  }
  const uint32_t inc = block_incl_scan_u32(loc, s);
  uint32_t run = inc - loc;
  for (int k = 0; k < per; ++k) {
    const int x = start + k;
    if (x < tiles) {
      const uint32_t c = row[x];
      row[x] = run;
      run += c;
    }
  }
  if (threadIdx.x == 255) digit_tot[blockIdx.x] = inc;
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint64_t *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t N,
                                                       int shift, const uint32_t *hist,
                                                       const uint32_t *digit_tot, int tiles) {
  __shared__ uint32_t base_d[256];
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t s[256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  {
    const uint32_t v = digit_tot[tid];
    const uint32_t inc = block_incl_scan_u32(v, s);
    base_d[tid] = (inc - v) + hist[(size_t)tid * tiles + blockIdx.x];
  }
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * kRadixTile;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int it = 0; it < kRadixItems; ++it) {
    const int64_t i = tbase + it * kRadixThreads + tid;
    const bool valid = i < N;
    const uint64_t key = valid ? kin[i] : 0ull;
    const int32_t val = valid ? vin[i] : 0;
    const uint32_t digit = (uint32_t)(key >> shift) & 255u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      same &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    if (valid && rank == 0) wcnt[wave][digit] = (uint32_t)__popcll(same);
    __syncthreads();
    {
      uint32_t run = base_d[tid];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = run;
        run += c;
      }
      base_d[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wcnt[wave][digit] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_count_active(const uint64_t *__restrict__ keys, int64_t N,
                                                      DevState *st) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const bool act = keys[p] != ~0ull;
  if (act && (p + 1 == N || keys[p + 1] == ~0ull)) st->n_active = (int32_t)(p + 1);
  if (p == 0 && !act) st->n_active = 0;
}

__global__ __launch_bounds__(256) void k_copy_i32(const int32_t *__restrict__ a,
                                                  int32_t *__restrict__ b, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) b[i] = a[i];
}

// zone of the particle of rank p: the largest k with floor(k Na / n_r) <= p
__global__ __launch_bounds__(256) void k_zone(const int32_t *__restrict__ by_r, int64_t N, int n_r,
                                              const DevState *st, int32_t *zone) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int64_t na = st->n_active;
  zone[by_r[p]] = p < na ? (int32_t)(((p + 1) * (int64_t)n_r - 1) / na) : n_r;
}

__global__ __launch_bounds__(256) void k_keys_zone(const int32_t *__restrict__ vals,
                                                   const int32_t *__restrict__ zone, int64_t N,
                                                   uint64_t *keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) keys[i] = (uint64_t)(uint32_t)zone[vals[i]];
}

// member ranges, edges, volumes and gas primaries of every cell
__global__ __launch_bounds__(256) void k_cells(Model P, int n_r, int n_z,
                                               const double *__restrict__ r,
                                               const double *__restrict__ z,
                                               const int32_t *__restrict__ by_r,
                                               const int32_t *__restrict__ order,
                                               const DevState *st, int32_t *cell_start,
                                               double *geom, double *gas) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int nc = n_r * n_z;
  if (c >= nc) return;
  const int64_t na = st->n_active;
  const int k = c / n_z, l = c % n_z;
  const int64_t b0 = (int64_t)k * na / n_r, b1 = (int64_t)(k + 1) * na / n_r;
  const int64_t nk = b1 - b0;
  const int64_t s0 = b0 + (int64_t)l * nk / n_z, s1 = b0 + (int64_t)(l + 1) * nk / n_z;
  cell_start[c] = (int32_t)s0;
  if (c == nc - 1) cell_start[nc] = (int32_t)na;
  double r_lo = 0.0, r_hi = 0.0, z_lo = 0.0, z_hi = 0.0;
  if (nk > 0) {
    r_lo = b0 == 0 ? r[by_r[b0]] : 0.5 * (r[by_r[b0 - 1]] + r[by_r[b0]]);
    r_hi = b1 == na ? r[by_r[b1 - 1]] : 0.5 * (r[by_r[b1 - 1]] + r[by_r[b1]]);
  }
  if (s1 > s0) {
    z_lo = s0 == b0 ? 0.0 : 0.5 * (z[order[s0 - 1]] + z[order[s0]]);
    z_hi = s1 == b1 ? z[order[s1 - 1]] : 0.5 * (z[order[s1 - 1]] + z[order[s1]]);
  }
  const double r_c = P.column ? P.r_col : 0.5 * (r_lo + r_hi);
  const double z_c = 0.5 * (z_lo + z_hi);
  const double V = P.column ? 2.0 * (z_hi - z_lo)
                            : 2.0 * kPi * (r_hi * r_hi - r_lo * r_lo) * (z_hi - z_lo);
  double *gm = geom + (size_t)c * 5;
  gm[0] = r_lo;
  gm[1] = r_hi;
  gm[2] = z_lo;
  gm[3] = z_hi;
  gm[4] = V;
  double *gs = gas + (size_t)c * 6;
  if (s1 > s0) {
    const DiskPoint d = disk_at(P, r_c, z_c);
    gs[0] = V;
    gs[1] = d.rho_g;
    gs[2] = d.T;
    gs[3] = P.alpha;
    gs[4] = r_c;
    gs[5] = z_c / d.H;
  } else {
    for (int f = 0; f < 6; ++f) gs[f] = 0.0;
  }
}

static hipError_t radix_pass(BinBuffers &b, int &cur, int64_t N, int shift, hipStream_t s) {
  const int tiles = radix_tiles(N);
  k_radix_hist<<<tiles, kRadixThreads, 0, s>>>(b.keys[cur], N, shift, b.hist, tiles);
  k_radix_scan_rows<<<256, 256, 0, s>>>(b.hist, tiles, b.digit_tot);
  k_radix_scatter<<<tiles, kRadixThreads, 0, s>>>(b.keys[cur], b.vals[cur], b.keys[cur ^ 1],
                                                  b.vals[cur ^ 1], N, shift, b.hist, b.digit_tot,
                                                  tiles);
  cur ^= 1;
  return hipGetLastError();
}

hipError_t launch_binning(const Model &P, int n_r, int n_z, const double *r, const double *z,
                          const uint8_t *active, int64_t N, BinBuffers &b, int32_t *cell_start,
                          int32_t *order, double *geom, double *gas, DevState *state,
                          hipStream_t s) {
  if (N <= 0 || N > b.cap) return hipErrorInvalidValue;
  const unsigned g1 = (unsigned)((N + 255) / 256);
  hipError_t e;
  int cur = 0;
  // 1. rank by (r, index)
  k_keys_from_double<<<g1, 256, 0, s>>>(r, active, N, b.keys[0], b.vals[0]);
  for (int sh = 0; sh < 64; sh += 8)
    if ((e = radix_pass(b, cur, N, sh, s)) != hipSuccess) return e;
  k_count_active<<<g1, 256, 0, s>>>(b.keys[cur], N, state);
  k_copy_i32<<<g1, 256, 0, s>>>(b.vals[cur], b.by_r, N);
  k_zone<<<g1, 256, 0, s>>>(b.by_r, N, n_r, state, b.zone);
  // 2. rank by (zone, z, index): z first, then a stable pass over the zone
  cur = 0;
  k_keys_from_double<<<g1, 256, 0, s>>>(z, active, N, b.keys[0], b.vals[0]);
  for (int sh = 0; sh < 64; sh += 8)
    if ((e = radix_pass(b, cur, N, sh, s)) != hipSuccess) return e;
  if (n_r > 1) {
    k_keys_zone<<<g1, 256, 0, s>>>(b.vals[cur], b.zone, N, b.keys[cur]);
    for (int sh = 0; sh < 16 && (n_r >> sh) > 0; sh += 8)
      if ((e = radix_pass(b, cur, N, sh, s)) != hipSuccess) return e;
  }
  k_copy_i32<<<g1, 256, 0, s>>>(b.vals[cur], order, N);
  // 3. cells
  const int nc = n_r * n_z;
  k_cells<<<(nc + 255) / 256, 256, 0, s>>>(P, n_r, n_z, r, z, b.by_r, order, state, cell_start,
                                           geom, gas);
  return hipGetLastError();
}

}  // namespace mcd
