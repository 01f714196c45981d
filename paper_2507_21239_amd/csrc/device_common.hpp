// device_common.hpp -- counter-based random numbers and wavefront / team
// primitives for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcd {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds, each with
// two 32x32 -> 64-bit products, xors with the other two words and the round
// key, and a Weyl increment of the key.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint32_t a = 0xD2511F53u, b = 0xCD9E8D57u;
    const uint64_t pa = (uint64_t)a * c.x;
    const uint64_t pb = (uint64_t)b * c.z;
    U4 n;
    n.x = (uint32_t)(pb >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)pb;
    n.z = (uint32_t)(pa >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)pa;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// uniform in (0,1): top 52 bits of the 64-bit word hi:lo plus half a step
__host__ __device__ inline double u01(uint32_t lo, uint32_t hi) {
  const uint64_t w = ((uint64_t)hi << 32) | lo;
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// wavefront primitives (64 lanes)
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ inline double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

__device__ inline double wave_incl_scan(double x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// ---------------------------------------------------------------------------
// A team is T consecutive waves of one workgroup working on one cell.
// T == 1 needs no barrier (a wave runs in lockstep); T > 1 synchronises the
// whole workgroup, so every wave of the workgroup must belong to the team.
// scratch: LDS area of at least 8*T doubles + 4*T ints.
// ---------------------------------------------------------------------------
template <int T>
struct Team {
  int wave;       // wave index inside the team
  int lane;       // lane inside the wave
  int tl;         // team lane = wave*64 + lane
  double *red;    // 2 x 2T doubles (double-buffered)
  int *ired;      // 2 x 2T ints
  int phase;

  __device__ Team(int wave_, int lane_, void *scratch)
      : wave(wave_), lane(lane_), tl(wave_ * 64 + lane_), red((double *)scratch),
        ired((int *)((double *)scratch + 4 * T)), phase(0) {}

  __device__ void sync() {
    if (T > 1)
      __syncthreads();
    else
      wave_sync();
  }

  __device__ double sum(double x) {
    x = wave_sum(x);
    if (T == 1) return x;
    phase ^= 1;
    double *buf = red + phase * 2 * T;
    if (lane == 0) buf[wave] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < T; ++w) s += buf[w];
    return s;
  }

  __device__ double max(double x) {
    x = wave_max(x);
    if (T == 1) return x;
    phase ^= 1;
    double *buf = red + phase * 2 * T;
    if (lane == 0) buf[wave] = x;
    __syncthreads();
    double s = buf[0];
#pragma unroll
    for (int w = 1; w < T; ++w) s = fmax(s, buf[w]);
    return s;
  }

  // inclusive scan over team lanes; also returns the exclusive prefix and
  // the total (identical on every lane)
  __device__ double incl_scan(double x, double &excl, double &total) {
    double inc = wave_incl_scan(x);
    double prev = __shfl_up(inc, 1, 64);
    if (lane == 0) prev = 0.0;
    if (T == 1) {
      total = __shfl(inc, 63, 64);
      excl = prev;
      return inc;
    }
    phase ^= 1;
    double *buf = red + phase * 2 * T;
    if (lane == 63) buf[wave] = inc;
    __syncthreads();
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int w = 0; w < T; ++w) {
      if (w < wave) off += buf[w];
      tot += buf[w];
    }
    total = tot;
    excl = off + prev;
    return off + inc;
  }

  // first team lane with pred set (or -1); on a miss, the last team lane
  // with fallback set (or -1) goes into *fb
  __device__ int first_lane(bool pred, bool fallback, int *fb) {
    const uint64_t b = __ballot(pred);
    const uint64_t f = __ballot(fallback);
    if (T == 1) {
      *fb = f ? 63 - __clzll(f) : -1;
      return b ? __ffsll((unsigned long long)b) - 1 : -1;
    }
    phase ^= 1;
    int *buf = ired + phase * 2 * T;
    if (lane == 0) {
      buf[wave] = b ? __ffsll((unsigned long long)b) - 1 : -1;
      buf[T + wave] = f ? 63 - __clzll(f) : -1;
    }
    __syncthreads();
    int first = -1, last = -1;
#pragma unroll
    for (int w = T - 1; w >= 0; --w) {
      if (buf[w] >= 0) first = w * 64 + buf[w];
    }
#pragma unroll
    for (int w = 0; w < T; ++w) {
      if (buf[T + w] >= 0) last = w * 64 + buf[T + w];
    }
    *fb = last;
    return first;
  }

  // broadcast an int and a double from team lane `src`
  __device__ void bcast(int src, int &iv, double &dv) {
    if (T == 1) {
      iv = __shfl(iv, src, 64);
      dv = __shfl(dv, src, 64);
      return;
    }
    phase ^= 1;
    int *ib = ired + phase * 2 * T;
    double *db = red + phase * 2 * T;
    if (tl == src) {
      ib[0] = iv;
      db[0] = dv;
    }
    __syncthreads();
    iv = ib[0];
    dv = db[0];
  }
};

}  // namespace mcd
