// device_common.hpp -- counter-based random numbers and wavefront primitives
// for gfx950 (wave64): DPP prefix scans, ballots, lane reads, LDS fences.
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

// uniform in (0,1): top 52 bits of the 64-bit word hi:lo plus half a step,
// ((w >> 12) + 1/2) 2^-52; evaluated as hi 2^-32 + ((lo >> 12) + 1/2) 2^-52,
// whose terms and sum are exact in FP64 (53 significant bits at most)
__host__ __device__ inline double u01(uint32_t lo, uint32_t hi) {
  return fma((double)hi, 0x1p-32, ((double)(lo >> 12) + 0.5) * 0x1p-52);
}

// ---------------------------------------------------------------------------
// wavefront primitives (64 lanes)
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }

// order LDS accesses of the lanes of one wave
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// workgroup barrier that orders LDS only (global memory is not waited for)
__device__ inline void block_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ inline double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, BANK_MASK, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, BANK_MASK, true);
  return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__device__ inline int readlane_i(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }
__device__ inline float readlane_t(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ inline double readlane_t(double x, int lane) { return readlane_d(x, lane); }

// a wave-uniform 32-bit value returned unchanged but hidden from the
// optimizer: what is derived from it is recomputed where it is used rather
// than hoisted out of an enclosing loop and held (or spilled) for the loop's
// whole duration
template <typename T>
__device__ inline T opaque_s(T x) {
  static_assert(sizeof(T) == 4, "32-bit values");
  asm volatile("" : "+s"(x));
  return x;
}
// opaque_s for a value that may be held in a vector register at the point of
// use (uniform, but not provably so to the compiler): through a VGPR, then
// the first lane
template <typename T>
__device__ inline T opaque_u(T x) {
  static_assert(sizeof(T) == 4, "32-bit values");
  int v = __builtin_bit_cast(int, x);
  asm volatile("" : "+v"(v));
  return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(v));
}
// the same for a per-lane 32-bit value (kept in a vector register)
template <typename T>
__device__ inline T opaque_v(T x) {
  static_assert(sizeof(T) == 4, "32-bit values");
  asm volatile("" : "+v"(x));
  return x;
}

template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ inline float dpp_f(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, BANK_MASK, true));
}

// inclusive prefix sum over the 64 lanes: shifts of 1, 2, 4, 8 inside rows of
// 16 lanes, then row broadcasts of lanes 15 and 31 (gfx9 DPP)
__device__ inline float wave_incl_scan(float x) {
  x += dpp_f<0x111, 0xf, 0xf>(x);  // row_shr:1
  x += dpp_f<0x112, 0xf, 0xf>(x);  // row_shr:2
  x += dpp_f<0x114, 0xf, 0xf>(x);  // row_shr:4
  x += dpp_f<0x118, 0xf, 0xf>(x);  // row_shr:8
  x += dpp_f<0x142, 0xa, 0xf>(x);  // row_bcast:15 into rows 1, 3
  x += dpp_f<0x143, 0xc, 0xf>(x);  // row_bcast:31 into rows 2, 3
  return x;
}
__device__ inline double wave_incl_scan(double x) {
  x += dpp_d<0x111, 0xf, 0xf>(x);  // row_shr:1
  x += dpp_d<0x112, 0xf, 0xf>(x);  // row_shr:2
  x += dpp_d<0x114, 0xf, 0xf>(x);  // row_shr:4
  x += dpp_d<0x118, 0xf, 0xf>(x);  // row_shr:8
  x += dpp_d<0x142, 0xa, 0xf>(x);  // row_bcast:15 into rows 1, 3
  x += dpp_d<0x143, 0xc, 0xf>(x);  // row_bcast:31 into rows 2, 3
  return x;
}

// maximum over the 64 lanes (non-negative inputs), returned on every lane
__device__ inline double wave_max_nonneg(double x) {
  x = fmax(x, dpp_d<0x111, 0xf, 0xf>(x));
  x = fmax(x, dpp_d<0x112, 0xf, 0xf>(x));
  x = fmax(x, dpp_d<0x114, 0xf, 0xf>(x));
  x = fmax(x, dpp_d<0x118, 0xf, 0xf>(x));
  x = fmax(x, dpp_d<0x142, 0xa, 0xf>(x));
  x = fmax(x, dpp_d<0x143, 0xc, 0xf>(x));
  return readlane_d(x, 63);
}

__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ inline int first_set(uint64_t b) { return b ? __builtin_ctzll(b) : -1; }
__device__ inline int last_set(uint64_t b) { return b ? 63 - __builtin_clzll(b) : -1; }

}  // namespace mcd
