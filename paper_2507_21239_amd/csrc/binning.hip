// binning.hip -- equal-count adaptive grid (paper, Summary: every cell holds
// the same number of representative particles).
//
// Radial zones: active particles ranked by (r, index), zone k holds ranks
// [floor(k Na / n_r), floor((k+1) Na / n_r)).  Cells: inside a zone, ranked
// by (z, index) and split the same way into n_z cells.
//
// Rank by r: one reduction gives the active count and the range of the IEEE
// bit patterns of r (non-negative doubles order like their bits); a 32-bit
// key (bits - min) >> shift, with shift chosen so keys keep 31 bits, is
// sorted by a stable least-significant-digit radix sort (8-bit digits, tiles
// of 2048 keys per 256-thread workgroup, per-tile digit histograms, a scan
// over tiles per digit, and a scatter that first orders the tile by digit in
// LDS and then writes each digit's run contiguously).  Stability keeps equal
// keys in index order; a fix-up pass then orders each run of equal keys by
// the full 64-bit pattern and index, so the result is the exact (r, index)
// order.  Rank by z: each zone is a contiguous range of the r order; one
// workgroup loads its members' (z bits, index) pairs and sorts them with a
// bitonic network held in registers.  Zones larger than that sort takes
// (8192) go the global path: 64-bit radix sort by z, then a stable radix pass
// by zone.
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

// ---------------------------------------------------------------------------
// active count and range of the r bit patterns
// ---------------------------------------------------------------------------
// per-workgroup partials {min, max, count}, then one workgroup combines them
// (no atomics: a few thousand 64-bit atomics on one address serialise)
__device__ inline void minmax_wave(uint64_t &lo, uint64_t &hi, uint64_t &cnt) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, off, 64), h2 = __shfl_xor(hi, off, 64);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
    cnt += __shfl_xor(cnt, off, 64);
  }
}

__device__ inline void minmax_block(uint64_t &lo, uint64_t &hi, uint64_t &cnt) {
  __shared__ uint64_t s[3][16];
  minmax_wave(lo, hi, cnt);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s[0][w] = lo;
    s[1][w] = hi;
    s[2][w] = cnt;
  }
  __syncthreads();
  lo = ~0ull;
  hi = 0ull;
  cnt = 0ull;
  for (int k = 0; k < nw; ++k) {
    lo = s[0][k] < lo ? s[0][k] : lo;
    hi = s[1][k] > hi ? s[1][k] : hi;
    cnt += s[2][k];
  }
}

__global__ __launch_bounds__(256) void k_minmax_part(const double *__restrict__ r,
                                                     const uint8_t *__restrict__ active,
                                                     int64_t N, uint64_t *part) {
  uint64_t lo = ~0ull, hi = 0ull, cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (active[i]) {
      const uint64_t b = key_bits(r[i]);
      lo = b < lo ? b : lo;
      hi = b > hi ? b : hi;
      ++cnt;
    }
  }
  minmax_block(lo, hi, cnt);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = lo;
    part[3 * blockIdx.x + 1] = hi;
    part[3 * blockIdx.x + 2] = cnt;
  }
}

__global__ __launch_bounds__(1024) void k_minmax_final(const uint64_t *part, int n_part,
                                                       BinState *bs, DevState *st) {
  uint64_t lo = ~0ull, hi = 0ull, cnt = 0;
  for (int k = threadIdx.x; k < n_part; k += blockDim.x) {
    lo = part[3 * k] < lo ? part[3 * k] : lo;
    hi = part[3 * k + 1] > hi ? part[3 * k + 1] : hi;
    cnt += part[3 * k + 2];
  }
  minmax_block(lo, hi, cnt);
  if (threadIdx.x == 0) {
    bs->min_bits = lo;
    bs->max_bits = hi;
    bs->count = (uint32_t)cnt;
    st->n_active = (int32_t)cnt;
  }
}

__device__ inline int key_shift(const BinState *bs) {
  const uint64_t span = bs->max_bits - bs->min_bits;
  const int bits = span ? 64 - __builtin_clzll(span) : 0;
  return bits > 31 ? bits - 31 : 0;
}

// 32-bit keys of one radix tile, and the tile's histogram of the first
// digit (the first pass needs no histogram kernel of its own); elements in
// the tile order of the radix kernels
__global__ __launch_bounds__(256) void k_keys_r32_hist(const double *__restrict__ r,
                                                       const uint8_t *__restrict__ active, int64_t N,
                                                       const BinState *bs, uint32_t *keys,
                                                       int32_t *vals, uint32_t *hist, int tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int sh = key_shift(bs);
  const uint64_t lo = bs->min_bits;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    const int64_t i = base + it * kRadixThreads + threadIdx.x;
    if (i < N) {
      const uint32_t k = active[i] ? (uint32_t)((key_bits(r[i]) - lo) >> sh) : 0xFFFFFFFFu;
      keys[i] = k;
      vals[i] = (int32_t)i;
      atomicAdd(&h[k & 255u], 1u);
    }
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_keys_from_double(const double *__restrict__ x,
                                                          const uint8_t *__restrict__ active,
                                                          int64_t N, uint64_t *keys, int32_t *vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  keys[i] = active[i] ? key_bits(x[i]) : ~0ull;
  vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// stable LSD radix pass, 8-bit digits
// ---------------------------------------------------------------------------
template <typename KeyT>
__global__ __launch_bounds__(256) void k_radix_hist(const KeyT *__restrict__ keys, int64_t N,
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

// Stable scatter of one tile.  Element order within the tile is (item, wave,
// lane); a lane finds the earlier lanes of its wave with the same digit by
// eight ballots, waves and items are chained through per-digit counters.
// The tile is first written to LDS in digit order, then each digit's run is
// copied to its global range, so consecutive lanes write consecutive words.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_radix_scatter(const KeyT *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       KeyT *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t N,
                                                       int shift, const uint32_t *hist,
                                                       const uint32_t *digit_tot, int tiles) {
  __shared__ KeyT sk[kRadixTile];
  __shared__ int32_t sv[kRadixTile];
  __shared__ uint32_t gbase[256];   // global position of the tile's first element of digit d
  __shared__ uint32_t lstart[256];  // position of digit d in the tile's digit order
  __shared__ uint32_t run_d[256];
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t s[256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t tbase = (int64_t)blockIdx.x * kRadixTile;
  const int tile_n = (int)std::min<int64_t>(kRadixTile, N - tbase);

  KeyT key[kRadixItems];
  int32_t val[kRadixItems];
  run_d[tid] = 0u;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    const int li = it * kRadixThreads + tid;
    key[it] = li < tile_n ? kin[tbase + li] : (KeyT)0;
    val[it] = li < tile_n ? vin[tbase + li] : 0;
    if (li < tile_n) atomicAdd(&run_d[(uint32_t)(key[it] >> shift) & 255u], 1u);
  }
  __syncthreads();
  {
    const uint32_t cnt = run_d[tid];
    const uint32_t inc = block_incl_scan_u32(cnt, s);
    lstart[tid] = inc - cnt;
    const uint32_t v = digit_tot[tid];
    const uint32_t ginc = block_incl_scan_u32(v, s);
    gbase[tid] = (ginc - v) + hist[(size_t)tid * tiles + blockIdx.x];
    run_d[tid] = inc - cnt;  // running local position of digit d
  }
  __syncthreads();
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int it = 0; it < kRadixItems; ++it) {
    const int li = it * kRadixThreads + tid;
    const bool valid = li < tile_n;
    const uint32_t digit = (uint32_t)(key[it] >> shift) & 255u;
    uint64_t same = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t bb = ballot(bit);
      same &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    if (valid && rank == 0) wcnt[wave][digit] = (uint32_t)__popcll(same);
    __syncthreads();
    {
      uint32_t run = run_d[tid];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = run;
        run += c;
      }
      run_d[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wcnt[wave][digit] + rank;
      sk[pos] = key[it];
      sv[pos] = val[it];
    }
    __syncthreads();
  }
  for (int p = tid; p < tile_n; p += kRadixThreads) {
    const KeyT k = sk[p];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint32_t g = gbase[d] + (uint32_t)p - lstart[d];
    kout[g] = k;
    vout[g] = sv[p];
  }
}

// have_hist: the tile histograms of this pass are already in hist
template <typename KeyT>
static hipError_t radix_pass(KeyT *const keys[2], int32_t *const vals[2], uint32_t *hist,
                             uint32_t *digit_tot, int &cur, int64_t N, int shift, hipStream_t s,
                             bool have_hist = false) {
  const int tiles = radix_tiles(N);
  if (!have_hist) k_radix_hist<KeyT><<<tiles, kRadixThreads, 0, s>>>(keys[cur], N, shift, hist, tiles);
  k_radix_scan_rows<<<256, 256, 0, s>>>(hist, tiles, digit_tot);
  k_radix_scatter<KeyT><<<tiles, kRadixThreads, 0, s>>>(keys[cur], vals[cur], keys[cur ^ 1],
                                                        vals[cur ^ 1], N, shift, hist, digit_tot,
                                                        tiles);
  cur ^= 1;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exact order inside runs of equal 32-bit keys: by full r bits, then index.
// Stability leaves every run in index order, so a run needs work only if two
// neighbours in it differ in r.  The first kernel copies the order out and
// flags such neighbours; the second lets the first flagged position of each
// run (flags and keys are read-only there) insertion-sort the run by
// (bits of r, index).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ties_copy(const uint32_t *__restrict__ keys,
                                                   const int32_t *__restrict__ vals,
                                                   const double *__restrict__ r, int64_t N,
                                                   const DevState *st, int32_t *__restrict__ by_r,
                                                   uint8_t *__restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int32_t v = vals[p];
  by_r[p] = v;
  uint8_t f = 0;
  if (p + 1 < (int64_t)st->n_active && keys[p + 1] == keys[p])
    f = key_bits(r[v]) != key_bits(r[vals[p + 1]]) ? 1 : 0;
  flag[p] = f;
}

__global__ __launch_bounds__(256) void k_fix_ties(const uint32_t *__restrict__ keys,
                                                  const uint8_t *__restrict__ flag,
                                                  const double *__restrict__ r, int64_t N,
                                                  const DevState *st, int32_t *by_r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N || !flag[p]) return;
  const int64_t na = st->n_active;
  const uint32_t k = keys[p];
  int64_t s = p;
  while (s > 0 && keys[s - 1] == k) {
    if (flag[s - 1]) return;  // an earlier position of this run does the work
    --s;
  }
  int64_t e = p + 2;
  while (e < na && keys[e] == k) ++e;
  for (int64_t a = s + 1; a < e; ++a) {
    const int32_t v = by_r[a];
    const uint64_t bv = key_bits(r[v]);
    int64_t b = a - 1;
    while (b >= s) {
      const int32_t u = by_r[b];
      const uint64_t bu = key_bits(r[u]);
      if (bu < bv || (bu == bv && u < v)) break;
      by_r[b + 1] = u;
      --b;
    }
    by_r[b + 1] = v;
  }
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

// ---------------------------------------------------------------------------
// order of each zone by (z, index): one workgroup per zone runs a bitonic
// network over the zone padded to P = 8 x threads (a power of two, >= 512).
// The key of an element packs its z bit pattern, range-reduced to 32 bits
// over the zone ((bits - min) >> shift), above its 32-bit particle index, so
// that one 64-bit comparison orders (reduced z, index).  Thread t keeps
// positions 8t .. 8t+7 in registers: strides below 8 compare inside a
// thread, strides 8 .. 256 pair lanes of one wave (DPP and permutes, no
// barrier), strides of 512 and up exchange through LDS between barriers.
// When shift > 0 distinct z can share a reduced key; each run of equal
// reduced keys is then re-sorted by (full bits, index), so the result is the
// exact (z, index) order.
// ---------------------------------------------------------------------------
constexpr int kZoneItems = 8;

// the element at position p takes the smaller of (own, partner) if it is the
// lower position of an ascending pair or the upper one of a descending pair
__device__ inline void keep_one(uint64_t &k, uint64_t k2, int p, int stride, int size) {
  const bool want_min = ((p & stride) == 0) == ((p & size) == 0);
  const bool take = want_min ? k > k2 : k2 > k;
  k = take ? k2 : k;
}

// value of lane (lane ^ LM) of the wave.  Lane xors below 16 are DPP moves
// (VALU): quad permutes give xor 1 and xor 2; a half-row mirror (xor 7)
// followed by a quad reverse (xor 3) gives xor 4; a row mirror (xor 15)
// followed by a half-row mirror gives xor 8.  Xors 16 and 32 use the LDS
// permute network.
template <int LM>
__device__ inline uint32_t lane_xor(uint32_t v) {
  const int x = (int)v;
  if constexpr (LM == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xf, 0xf, true);
  } else if constexpr (LM == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xf, 0xf, true);
  } else if constexpr (LM == 4) {
    const int y = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, true);
    return (uint32_t)__builtin_amdgcn_update_dpp(0, y, 0x1B, 0xf, 0xf, true);
  } else if constexpr (LM == 8) {
    const int y = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xf, 0xf, true);
    return (uint32_t)__builtin_amdgcn_update_dpp(0, y, 0x141, 0xf, 0xf, true);
  } else {
    return (uint32_t)__shfl_xor(x, LM, 64);
  }
}

// one exchange phase between lanes (strides 8 .. 256): for these strides the
// bits tested by the pair direction lie above the thread's own 8 positions
template <int LM>
__device__ inline void zone_lane_phase(uint64_t (&key)[kZoneItems], int base, int stride,
                                       int size) {
  const bool want_min = ((base & stride) == 0) == ((base & size) == 0);
#pragma unroll
  for (int e = 0; e < kZoneItems; ++e) {
    const uint32_t lo = lane_xor<LM>((uint32_t)key[e]);
    const uint32_t hi = lane_xor<LM>((uint32_t)(key[e] >> 32));
    const uint64_t k2 = ((uint64_t)hi << 32) | lo;
    const bool take = want_min ? key[e] > k2 : k2 > key[e];
    key[e] = take ? k2 : key[e];
  }
}

template <int S>
__device__ inline void zone_reg_phase(uint64_t (&key)[kZoneItems], int base, int size) {
#pragma unroll
  for (int e = 0; e < kZoneItems; ++e) {
    if (e & S) continue;
    const bool up = ((base + e) & size) == 0;
    if ((key[e] > key[e + S]) == up) {
      const uint64_t t = key[e];
      key[e] = key[e + S];
      key[e + S] = t;
    }
  }
}

__global__ __launch_bounds__(1024) void k_zone_sort(const int32_t *__restrict__ by_r,
                                                    const double *__restrict__ z, int n_r,
                                                    const DevState *st, int32_t *order) {
  extern __shared__ __align__(16) char smem[];
  __shared__ unsigned long long s_lo, s_hi;
  const int64_t na = st->n_active;
  const int zk = blockIdx.x;
  const int64_t b0 = (int64_t)zk * na / n_r, b1 = (int64_t)(zk + 1) * na / n_r;
  const int nk = (int)(b1 - b0);
  if (nk <= 0) return;
  const int P = blockDim.x * kZoneItems;
  const int tid = threadIdx.x;
  const int base = tid * kZoneItems;
  uint64_t bits[kZoneItems];
  int32_t idx[kZoneItems];
  unsigned long long lo = ~0ull, hi = 0ull;
#pragma unroll
  for (int e = 0; e < kZoneItems; ++e) {
    const int p = base + e;
    idx[e] = 0x7FFFFFFF;
    bits[e] = 0;
    if (p < nk) {
      idx[e] = by_r[b0 + p];
      bits[e] = key_bits(z[idx[e]]);
      lo = bits[e] < lo ? bits[e] : lo;
      hi = bits[e] > hi ? bits[e] : hi;
    }
  }
  // range of the zone's bit patterns: 32 significant bits after the shift
  if (tid == 0) {
    s_lo = ~0ull;
    s_hi = 0ull;
  }
  __syncthreads();
  atomicMin(&s_lo, lo);
  atomicMax(&s_hi, hi);
  __syncthreads();
  const uint64_t zmin = s_lo, range = s_hi - s_lo;
  const int shift = (range >> 32) ? 32 - __clzll((long long)range) : 0;
  uint64_t key[kZoneItems];
#pragma unroll
  for (int e = 0; e < kZoneItems; ++e)
    key[e] = base + e < nk ? (((bits[e] - zmin) >> shift) << 32) | (uint32_t)idx[e] : ~0ull;
  uint64_t *lk = (uint64_t *)smem;
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64 * kZoneItems) {
#pragma unroll
        for (int e = 0; e < kZoneItems; ++e) lk[base + e] = key[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kZoneItems; ++e) keep_one(key[e], lk[(base + e) ^ stride], base + e, stride, size);
        __syncthreads();
      } else if (stride >= kZoneItems) {
        switch (stride / kZoneItems) {
          case 1: zone_lane_phase<1>(key, base, stride, size); break;
          case 2: zone_lane_phase<2>(key, base, stride, size); break;
          case 4: zone_lane_phase<4>(key, base, stride, size); break;
          case 8: zone_lane_phase<8>(key, base, stride, size); break;
          case 16: zone_lane_phase<16>(key, base, stride, size); break;
          default: zone_lane_phase<32>(key, base, stride, size); break;
        }
      } else if (stride == 4) {
        zone_reg_phase<4>(key, base, size);
      } else if (stride == 2) {
        zone_reg_phase<2>(key, base, size);
      } else {
        zone_reg_phase<1>(key, base, size);
      }
    }
  }
  if (shift > 0) {
    // runs of equal reduced keys, re-sorted by (full bits, index) by the
    // thread that holds the run's first position.  Only members of such runs
    // need their full bits (read again from z): a reduced key keeps 32
    // significant bits of the zone's range, so runs are rare
    uint64_t *lz = lk + P;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kZoneItems; ++e) lk[base + e] = key[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kZoneItems; ++e) {
      const int p = base + e;
      if (p >= nk) continue;
      const uint32_t h = (uint32_t)(lk[p] >> 32);
      const bool tied = (p + 1 < nk && (uint32_t)(lk[p + 1] >> 32) == h) ||
                        (p > 0 && (uint32_t)(lk[p - 1] >> 32) == h);
      if (tied) lz[p] = key_bits(z[(int32_t)(uint32_t)key[e]]);
    }
    __syncthreads();
    for (int e = 0; e < kZoneItems; ++e) {
      const int p = base + e;
      const uint32_t h = (uint32_t)(lk[p] >> 32);
      if (p + 1 >= nk || (uint32_t)(lk[p + 1] >> 32) != h) continue;
      if (p > 0 && (uint32_t)(lk[p - 1] >> 32) == h) continue;
      int end = p + 2;
      while (end < nk && (uint32_t)(lk[end] >> 32) == h) ++end;
      for (int a = p + 1; a < end; ++a) {  // insertion sort of [p, end)
        const uint64_t kv = lk[a], zv = lz[a];
        const uint32_t iv = (uint32_t)kv;
        int b = a - 1;
        while (b >= p && (lz[b] > zv || (lz[b] == zv && (uint32_t)lk[b] > iv))) {
          lk[b + 1] = lk[b];
          lz[b + 1] = lz[b];
          --b;
        }
        lk[b + 1] = kv;
        lz[b + 1] = zv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kZoneItems; ++e) key[e] = lk[base + e];
  }
#pragma unroll
  for (int e = 0; e < kZoneItems; ++e)
    if (base + e < nk) order[b0 + base + e] = (int32_t)(uint32_t)key[e];
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
    const LocalGas d = local_gas_at(P, r_c, z_c);
    gs[0] = V;
    gs[1] = d.rho_g;
    gs[2] = d.T;
    gs[3] = d.alpha;
    gs[4] = r_c;
    gs[5] = z_c / d.H;
  } else {
    for (int f = 0; f < 6; ++f) gs[f] = 0.0;
  }
}

// padded size of the zone sort: a power of two, at least 512 (one full wave)
int zone_sort_size(int64_t zone_max) {
  int P = 64 * kZoneItems;
  while (P < zone_max) P <<= 1;
  return P;
}

hipError_t launch_binning(const Model &P, int n_r, int n_z, const double *r, const double *z,
                          const uint8_t *active, int64_t N, BinBuffers &b, int32_t *cell_start,
                          int32_t *order, double *geom, double *gas, DevState *state,
                          hipStream_t s) {
  if (N <= 0 || N > b.cap) return hipErrorInvalidValue;
  const unsigned g1 = (unsigned)((N + 255) / 256);
  hipError_t e;
  // 1. rank by (r, index)
  const unsigned n_part = std::min<unsigned>(g1, kMinmaxParts);
  k_minmax_part<<<n_part, 256, 0, s>>>(r, active, N, b.part);
  k_minmax_final<<<1, 1024, 0, s>>>(b.part, (int)n_part, b.bs, state);
  const int tiles = radix_tiles(N);
  k_keys_r32_hist<<<tiles, kRadixThreads, 0, s>>>(r, active, N, b.bs, b.k32[0], b.vals[0], b.hist,
                                                  tiles);
  int cur = 0;
  for (int sh = 0; sh < 32; sh += 8)
    if ((e = radix_pass<uint32_t>(b.k32, b.vals, b.hist, b.digit_tot, cur, N, sh, s, sh == 0)) !=
        hipSuccess)
      return e;
  k_ties_copy<<<g1, 256, 0, s>>>(b.k32[cur], b.vals[cur], r, N, state, b.by_r, b.flag);
  k_fix_ties<<<g1, 256, 0, s>>>(b.k32[cur], b.flag, r, N, state, b.by_r);
  // 2. rank by (z, index) inside each zone
  const int64_t zone_max = (N + n_r - 1) / n_r;  // no zone holds more
  if (zone_max > kZoneSortMax && (b.keys[0] == nullptr || b.zone == nullptr))
    return hipErrorInvalidValue;  // the workspace holds no buffers of the global path
  if (zone_max <= kZoneSortMax) {
    const int Pz = zone_sort_size(zone_max);
    const size_t lds = (size_t)Pz * 2 * sizeof(uint64_t);  // keys, then full bits for the runs
    if (lds > 64 * 1024) {
      e = hipFuncSetAttribute((const void *)k_zone_sort, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
      if (e != hipSuccess) return e;
    }
    k_zone_sort<<<n_r, Pz / kZoneItems, lds, s>>>(b.by_r, z, n_r, state, order);
  } else {
    k_zone<<<g1, 256, 0, s>>>(b.by_r, N, n_r, state, b.zone);
    cur = 0;
    k_keys_from_double<<<g1, 256, 0, s>>>(z, active, N, b.keys[0], b.vals[0]);
    for (int sh = 0; sh < 64; sh += 8)
      if ((e = radix_pass<uint64_t>(b.keys, b.vals, b.hist, b.digit_tot, cur, N, sh, s)) != hipSuccess)
        return e;
    if (n_r > 1) {
      k_keys_zone<<<g1, 256, 0, s>>>(b.vals[cur], b.zone, N, b.keys[cur]);
      for (int sh = 0; sh < 16 && (n_r >> sh) > 0; sh += 8)
        if ((e = radix_pass<uint64_t>(b.keys, b.vals, b.hist, b.digit_tot, cur, N, sh, s)) != hipSuccess)
          return e;
    }
    k_copy_i32<<<g1, 256, 0, s>>>(b.vals[cur], order, N);
  }
  // 3. cells
  const int nc = n_r * n_z;
  k_cells<<<(nc + 255) / 256, 256, 0, s>>>(P, n_r, n_z, r, z, b.by_r, order, state, cell_start,
                                           geom, gas);
  return hipGetLastError();
}

}  // namespace mcd
