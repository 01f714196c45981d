// collide.hip -- the per-cell collision Monte Carlo of the representative-
// particle method (Zsom & Dullemond 2008, adopted by the paper, Summary):
// build the row sums r_i = sum_j r_ij of the cell's rate matrix, then repeat
// events: exponential waiting time from the total rate R, choose i by the
// cumulative row sums, choose j by the cumulative rates of row i, apply the
// outcome (sticking / erosion / fragmentation) to i only, update every row
// sum incrementally for the changed particle and recompute row i.
//
// A cell is processed by a team of T waves (T = 1 or 4).  The cell's n
// particles are laid out in canonical order j = 0..n-1; team lane t owns the
// contiguous slots j = t*K .. t*K + K - 1 (K = ceil(n / 64T)), so the
// cumulative rate of j is the team prefix of the lanes' partial sums plus a
// short in-lane prefix.  Particle records live in LDS as structure-of-arrays
// indexed by s = q*64T + t (slot q of lane t): lanes of a wave touch
// consecutive words.  Row sums (FP64), the per-event row values and the
// column values stay in registers of the owning lane.
#include "device_common.hpp"
#include "internal.hpp"

namespace mcd {

template <typename RT>
struct Region {
  RT *f;          // 10 arrays of cap: m, im, a, St, h, q1, vr, vp, vz, nd
  double *m64;    // exact masses
  double *M64;    // swarm masses
  int32_t *idx;   // global particle index
  void *scratch;  // team reduction scratch
  int cap;

  __device__ Region(char *base, int cap_) : cap(cap_) {
    f = (RT *)base;
    m64 = (double *)(base + (size_t)10 * cap * sizeof(RT));
    M64 = m64 + cap;
    idx = (int32_t *)(M64 + cap);
    scratch = (void *)(idx + cap);
  }
  __device__ Rec<RT> load(int s) const {
    Rec<RT> r;
    r.m = f[s];
    r.im = f[cap + s];
    r.a = f[2 * cap + s];
    r.St = f[3 * cap + s];
    r.h = f[4 * cap + s];
    r.q1 = f[5 * cap + s];
    r.vr = f[6 * cap + s];
    r.vp = f[7 * cap + s];
    r.vz = f[8 * cap + s];
    r.nd = f[9 * cap + s];
    return r;
  }
  __device__ void store(int s, const Rec<RT> &r) {
    f[s] = r.m;
    f[cap + s] = r.im;
    f[2 * cap + s] = r.a;
    f[3 * cap + s] = r.St;
    f[4 * cap + s] = r.h;
    f[5 * cap + s] = r.q1;
    f[6 * cap + s] = r.vr;
    f[7 * cap + s] = r.vp;
    f[8 * cap + s] = r.vz;
    f[9 * cap + s] = r.nd;
  }
};

// Choose the first slot whose cumulative value exceeds target.  v[] are the
// caller lane's K values (in canonical order), part their sum, incl / excl
// the team's inclusive / exclusive prefix of part.  If rounding leaves no
// prefix above the target, the last nonzero entry is taken.  Returns the
// chosen slot q (uniform) and sets owner (team lane) and the owner's payload
// value pay[q] (uniform).
template <int KMAX, int T, typename PT>
__device__ inline int team_select(Team<T> &tm, double incl, double excl, double part,
                                  const double *v, const PT *pay, int K, double target,
                                  int &owner, double &payload) {
  int fb;
  // a lane with an empty partial is never chosen (the team prefix is not
  // exactly monotone under rounding)
  const int first = tm.first_lane(incl > target && part > 0.0, part > 0.0, &fb);
  const int src = first >= 0 ? first : fb;
  int qsel = -1;
  double pv = 0.0;
  if (tm.tl == src) {
    double cum = excl;
    int last = -1;
    bool found = false;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (q < K && !found) {
        if (v[q] > 0.0) {
          last = q;
          pv = (double)pay[q];
        }
        cum += v[q];
        if (first >= 0 && cum > target) {
          qsel = q;
          pv = (double)pay[q];
          found = true;
        }
      }
    }
    if (!found) {
      qsel = last;
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q == last) pv = (double)pay[q];
    }
  }
  tm.bcast(src < 0 ? 0 : src, qsel, pv);
  owner = src;
  payload = pv;
  return qsel;
}

template <typename RT, int KMAX, int T>
__device__ void process_cell(const CollideArgs &A, int cell, char *base, int cap, int wave,
                             int lane, uint32_t step) {
  const int s0 = A.cell_start[cell];
  const int n = A.cell_start[cell + 1] - s0;
  if (n <= 0) return;
  constexpr int TL = 64 * T;
  const int K = (n + TL - 1) / TL;
  Region<RT> R(base, cap);
  Team<T> tm(wave, lane, R.scratch);
  const int tl = tm.tl;
  if (K > KMAX || K * TL > cap) {
    if (tl == 0) atomicOr(&A.state->flags, FLAG_CAPACITY);
    return;
  }

  Gas g;
  gas_from_primaries(A.P, A.gas + (size_t)cell * 6, g);
  const PairConst<RT> pc = make_pair_const<RT>(A.P, g);
  if (!(g.V > 0.0)) {
    if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_VOLUME);
    return;
  }

  // ---- load members, choose the cell's rate scale, build records --------
  double m64[KMAX], M64[KMAX];
  int idx[KMAX];
  double ndmax = 0.0;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const int j = tl * K + q;
    idx[q] = -1;
    m64[q] = 1.0;
    M64[q] = 0.0;
    if (q < K && j < n) {
      idx[q] = A.order[s0 + j];
      m64[q] = A.m[idx[q]];
      M64[q] = A.M[idx[q]];
      ndmax = fmax(ndmax, M64[q] / (m64[q] * g.V));
    }
  }
  double scale = 1.0;  // rates are carried as r * scale (FP32 range)
  if (sizeof(RT) == 4) {
    ndmax = tm.max(ndmax);
    int e2 = 0;
    frexp(ndmax, &e2);
    scale = ldexp(1.0, -e2);
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const int j = tl * K + q;
    if (q < K && j < n) {
      const int s = q * TL + tl;
      R.store(s, make_rec<RT>(A.P, g, m64[q], M64[q], scale));
      R.m64[s] = m64[q];
      R.M64[s] = M64[q];
      R.idx[s] = idx[q];
    }
  }
  tm.sync();

  // ---- row sums r_i = sum_k r_ik, k in canonical order ------------------
  double r[KMAX];
  const int lanes_used = (n + K - 1) / K;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    r[q] = 0.0;
    if (q < K && tl * K + q < n) {
      const Rec<RT> mine = R.load(q * TL + tl);
      RT acc = (RT)0;
      for (int t2 = 0; t2 < lanes_used; ++t2) {
        for (int q2 = 0; q2 < K; ++q2) {
          if (t2 * K + q2 >= n) break;
          const Rec<RT> rk = R.load(q2 * TL + t2);
          RT dv;
          const RT Kx = pair_kernel(pc, mine, rk, dv);
          acc += swarm_rate(pc, mine, rk, Kx);
        }
      }
      r[q] = (double)acc;
    }
  }

  // ---- events ------------------------------------------------------------
  double t = 0.0;
  int64_t e = 0;
  unsigned long long oc_count[4] = {0ull, 0ull, 0ull, 0ull};
  const uint32_t c32 = (uint32_t)cell;
  for (;;) {
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < K) part += r[q];
    double excl, Rtot;
    const double incl = tm.incl_scan(part, excl, Rtot);
    if (!(Rtot > 0.0) || !isfinite(Rtot)) {
      if (!isfinite(Rtot) && tl == 0) atomicOr(&A.state->flags, FLAG_BAD_RATE);
      break;
    }
    if (A.max_events > 0 && e >= A.max_events) break;
    const U4 w0 = philox4x32_10(U4{(uint32_t)e, c32, step, 0u}, A.P.key0, A.P.key1);
    const U4 w1 = philox4x32_10(U4{(uint32_t)e, c32, step, 1u}, A.P.key0, A.P.key1);
    const double u1 = u01(w0.x, w0.y), u2 = u01(w0.z, w0.w);
    const double u3 = u01(w1.x, w1.y), u4 = u01(w1.z, w1.w);
    const double tau = -log(u1) / Rtot * scale;  // exponential waiting time, true units
    if (A.dt > 0.0 && t + tau > A.dt) break;   // the next event falls outside the step
    t += tau;

    // -- choose i by cumulative row sums
    int ownI;
    double dummy;
    const int qI = team_select<KMAX, T, double>(tm, incl, excl, part, r, r, K, u2 * Rtot, ownI,
                                               dummy);
    if (qI < 0 || ownI < 0) {
      if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_RATE);
      break;
    }
    const int si = qI * TL + ownI;
    const Rec<RT> ri = R.load(si);
    const double mi = R.m64[si];
    const double Mi = R.M64[si];
    const int gi = R.idx[si];

    // -- row i before the event: r_ij, r_ji and the relative velocities
    RT rji[KMAX], dvv[KMAX];
    double rij[KMAX];
    double part1 = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      rij[q] = 0.0;
      rji[q] = (RT)0;
      dvv[q] = (RT)0;
      if (q < K && tl * K + q < n) {
        const Rec<RT> rq = R.load(q * TL + tl);
        RT dv;
        const RT Kx = pair_kernel(pc, ri, rq, dv);
        rij[q] = (double)swarm_rate(pc, ri, rq, Kx);
        rji[q] = swarm_rate(pc, rq, ri, Kx);
        dvv[q] = dv;
        part1 += rij[q];
      }
    }
    double excl1, Ri;
    const double incl1 = tm.incl_scan(part1, excl1, Ri);
    if (!(Ri > 0.0)) {
      // row i has no partner left (its stored sum was rounding residue):
      // clear it and count a null event
      if (tl == ownI) {
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
          if (q == qI) r[q] = 0.0;
      }
      if (tl == 0 && A.evlog != nullptr && e < A.log_per_cell) {
        int32_t *L = A.evlog + ((size_t)cell * A.log_per_cell + e) * 4;
        L[0] = ownI * K + qI;
        L[1] = -1;
        L[2] = -1;
        L[3] = 0;
      }
      ++e;
      continue;
    }
    int ownJ;
    double dvj;
    const int qJ =
        team_select<KMAX, T, RT>(tm, incl1, excl1, part1, rij, dvv, K, u3 * Ri, ownJ, dvj);
    const int sj = qJ * TL + ownJ;
    const double mj = R.m64[sj];
    const int gj = R.idx[sj];
    const int j_local = ownJ * K + qJ;
    const int i_local = ownI * K + qI;

    // -- outcome (only i changes)
    double mnew;
    const bool fast = !((RT)dvj < (RT)A.P.v_frag);
    const int oc = outcome(A.P, fast, mi, mj, u4, mnew);
    if (!(mnew > 0.0) || !isfinite(mnew)) {
      if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_MASS);
    }
    if (A.comp != nullptr && A.P.n_comp > 0 && (oc == OUT_STICK || oc == OUT_FRAG) &&
        tl < A.P.n_comp) {
      const double wi = mi, wj = group_factor(A.P.dm_max, mi, mj) * mj;
      float *cs = A.comp + (size_t)tl * A.N;
      const double ci = (double)cs[gi], cj = (double)cs[gj];
      cs[gi] = (float)((wi * ci + wj * cj) / (wi + wj));
    }
    const Rec<RT> rin = make_rec<RT>(A.P, g, mnew, Mi, scale);
    tm.sync();  // every lane is done reading the old record of i
    if (tl == 0) {
      R.store(si, rin);
      R.m64[si] = mnew;
      A.m[gi] = mnew;
      if (A.evlog != nullptr && e < A.log_per_cell) {
        int32_t *L = A.evlog + ((size_t)cell * A.log_per_cell + e) * 4;
        L[0] = i_local;
        L[1] = j_local;
        L[2] = oc;
        L[3] = 0;
      }
    }
    tm.sync();

    // -- new row i: incremental update of the other rows, fresh row sum of i
    double part2 = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (q < K && tl * K + q < n) {
        const int s = q * TL + tl;
        const Rec<RT> rq = R.load(s);
        RT dv;
        const RT Kx = pair_kernel(pc, rin, rq, dv);
        part2 += (double)swarm_rate(pc, rin, rq, Kx);
        if (s != si) {
          const double x = (r[q] - (double)rji[q]) + (double)swarm_rate(pc, rq, rin, Kx);
          r[q] = x > 0.0 ? x : 0.0;
        }
      }
    }
    const double ri_new = tm.sum(part2);
    if (tl == ownI) {
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q == qI) r[q] = ri_new;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) oc_count[k] += (oc == k) ? 1ull : 0ull;
    ++e;
  }
  if (tl == 0) {
    atomicAdd(&A.state->events, (unsigned long long)e);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (oc_count[k]) atomicAdd(&A.state->outcomes[k], oc_count[k]);
  }
  tm.sync();  // the region is reused by the next cell
}

// ---------------------------------------------------------------------------
// batched schedule: one persistent launch; big cells on four-wave teams
// (largest first), then small cells on single waves (largest first)
// ---------------------------------------------------------------------------
template <typename RT, int KBIG, int KSMALL>
__global__ __launch_bounds__(256) void collide_batched(CollideArgs A) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_item;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t step = A.state->step;
  if (A.n_big > 0) {
    for (;;) {
      if (threadIdx.x == 0) s_item = atomicAdd(&A.state->big_head, 1);
      __syncthreads();
      const int item = s_item;
      __syncthreads();
      if (item >= A.n_big) break;
      process_cell<RT, KBIG, 4>(A, A.big_list[item], smem, A.big_cap, wave, lane, step);
    }
  }
  char *mine = smem + (size_t)wave * region_bytes<RT>(A.small_cap, 1);
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(&A.state->small_head, 1);
    item = __shfl(item, 0, 64);
    if (item >= A.n_small) break;
    process_cell<RT, KSMALL, 1>(A, A.small_list[item], mine, A.small_cap, 0, lane, step);
  }
}

// plain schedule: one one-wave workgroup per cell
template <typename RT, int KMAX>
__global__ __launch_bounds__(64) void collide_plain(CollideArgs A) {
  extern __shared__ __align__(16) char smem[];
  process_cell<RT, KMAX, 1>(A, blockIdx.x, smem, A.small_cap, 0, threadIdx.x, A.state->step);
}

__global__ void reset_queues(DevState *st) {
  st->big_head = 0;
  st->small_head = 0;
}

// ---------------------------------------------------------------------------
// test path: the full rate matrix of one cell, from the same records and
// pair code as the collision kernel
// ---------------------------------------------------------------------------
template <typename RT>
__global__ __launch_bounds__(256) void rates_cell(CollideArgs A, int cell, double *r_out,
                                                  int64_t ld, double *rowsum) {
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
      RT dv;
      const RT Kx = pair_kernel(pc, ri, rk, dv);
      const RT x = swarm_rate(pc, ri, rk, Kx);
      acc += x;
      r_out[(int64_t)i * ld + k] = (double)x / scale;
    }
    if (rowsum) rowsum[i] = (double)acc / scale;
  }
}

// ---------------------------------------------------------------------------
template <typename RT, int KB, int KS>
static hipError_t run_batched(const CollideArgs &a, int grid_override, hipStream_t s) {
  const size_t lds = std::max(region_bytes<RT>(a.big_cap, 4), 4 * region_bytes<RT>(a.small_cap, 1));
  auto kern = collide_batched<RT, KB, KS>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int units = a.n_big + (a.n_small + 3) / 4;
  int grid = std::min(per_cu * cus, std::max(units, 1));
  if (grid_override > 0) grid = grid_override;
  reset_queues<<<1, 1, 0, s>>>(a.state);
  kern<<<grid, 256, lds, s>>>(a);
  return hipGetLastError();
}

template <typename RT>
static hipError_t run_plain(const CollideArgs &a, int n_cells, hipStream_t s) {
  const size_t lds = region_bytes<RT>(a.small_cap, 1);
  auto kern = collide_plain<RT, 16>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (n_cells > 0) kern<<<n_cells, 64, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_collide(const CollideArgs &a, int precision, int schedule, int n_cells,
                          int max_cell, int grid_override, hipStream_t s) {
  if (schedule == 0) {
    if (max_cell > 64 * 16) return hipErrorInvalidValue;
    return precision == 0 ? run_plain<double>(a, n_cells, s) : run_plain<float>(a, n_cells, s);
  }
  const bool wide = a.big_cap > 256 * 4;
  if (precision == 0)
    return wide ? run_batched<double, 8, 4>(a, grid_override, s)
                : run_batched<double, 4, 4>(a, grid_override, s);
  return wide ? run_batched<float, 8, 4>(a, grid_override, s)
              : run_batched<float, 4, 4>(a, grid_override, s);
}

hipError_t launch_rates_cell(const CollideArgs &a, int precision, int cell, double *r_out,
                             int64_t ld, double *rowsum_out, hipStream_t s) {
  if (precision == 0)
    rates_cell<double><<<1, 256, 0, s>>>(a, cell, r_out, ld, rowsum_out);
  else
    rates_cell<float><<<1, 256, 0, s>>>(a, cell, r_out, ld, rowsum_out);
  return hipGetLastError();
}

}  // namespace mcd
