// collide_device.hpp -- the per-cell collision Monte Carlo of the representative-
// particle method (Zsom & Dullemond 2008, adopted by the paper, Summary):
// build the row sums r_i = sum_j r_ij of the cell's rate matrix, then repeat
// events: exponential waiting time from the total rate R, choose i by the
// cumulative row sums, choose j by the cumulative rates of row i, apply the
// outcome (sticking / erosion / fragmentation) to i only, update every row
// sum incrementally for the changed particle and recompute row i.
//
// A cell is processed by a team of nw waves (1, or 4 for cells above the
// single-wave threshold, 256 particles by default); the two team shapes are
// separate instantiations of the cell body.  The cell's n particles are in
// canonical order j = 0..n-1; team lane t owns the contiguous slots
// j = t*K .. t*K+K-1 (K = ceil(n/(64 nw))), so the cumulative rate of j is the
// team prefix of the lanes' partial sums plus a short in-lane prefix.  Prefix
// sums are FP64 DPP scans in both forms; four-wave teams exchange wave totals
// through LDS (one barrier per scan).  A selection is made by the wave whose
// prefix range holds the target -- every wave finds it from the exchanged
// totals -- and published with one more barrier.  The uniforms of 64 events
// are drawn at once, one event per lane.  Particle records live in LDS as
// packed vectors indexed by s = q*64nw + t (slot q of lane t), so a wave reads
// consecutive 16-byte words.  Row sums (FP64), the per-event row values,
// masses and particle indices stay in registers of the owning lane; masses go
// back to HBM once, when the cell is done.  In the FP32 form the starting row
// sums evaluate each unordered pair once (build_rows_pairwise*); the FP64 form
// sums every row in canonical order.  The batched kernel carries the
// composition mix and the event log only in the variant launched for runs
// that use them.
//
// The cell body and the kernel templates; collide.hip launches them, and
// collide_ilp.hip holds the one instantiation built with a different
// instruction schedule.
#pragma once

#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace mcd {

// ---------------------------------------------------------------------------
// packed LDS records
// ---------------------------------------------------------------------------
template <typename RT>
struct RecStore;

template <>
struct RecStore<float> {
  float4 *A;  // im, a, St, h
  float4 *B;  // q1, vr, vp, vz
  float4 *C;  // nd, m, ist, Mn
  __device__ RecStore(char *base, int cap)
      : A((float4 *)base), B((float4 *)base + cap), C((float4 *)base + 2 * cap) {}
  __device__ Rec<float> load(int s) const {
    const float4 a = A[s], b = B[s], c = C[s];
    Rec<float> r;
    r.im = a.x; r.a = a.y; r.St = a.z; r.h = a.w;
    r.q1 = b.x; r.vr = b.y; r.vp = b.z; r.vz = b.w;
    r.nd = c.x; r.m = c.y; r.ist = c.z; r.Mn = c.w;
    return r;
  }
  __device__ void store(int s, const Rec<float> &r) const {
    A[s] = make_float4(r.im, r.a, r.St, r.h);
    B[s] = make_float4(r.q1, r.vr, r.vp, r.vz);
    C[s] = make_float4(r.nd, r.m, r.ist, r.Mn);
  }
};

template <>
struct RecStore<double> {
  double2 *D;  // 6 arrays: (im, a) (St, h) (q1, vr) (vp, vz) (nd, m) (ist, -)
  int cap;
  __device__ RecStore(char *base, int cap_) : D((double2 *)base), cap(cap_) {}
  __device__ Rec<double> load(int s) const {
    const double2 a = D[s], b = D[cap + s], c = D[2 * cap + s], d = D[3 * cap + s],
                  e = D[4 * cap + s], f = D[5 * cap + s];
    Rec<double> r;
    r.im = a.x; r.a = a.y; r.St = b.x; r.h = b.y; r.q1 = c.x; r.vr = c.y;
    r.vp = d.x; r.vz = d.y; r.nd = e.x; r.m = e.y; r.ist = f.x;
    r.Mn = 0.0;  // not held: the FP64 state is rebuilt from M
    return r;
  }
  __device__ void store(int s, const Rec<double> &r) const {
    D[s] = make_double2(r.im, r.a);
    D[cap + s] = make_double2(r.St, r.h);
    D[2 * cap + s] = make_double2(r.q1, r.vr);
    D[3 * cap + s] = make_double2(r.vp, r.vz);
    D[4 * cap + s] = make_double2(r.nd, r.m);
    D[5 * cap + s] = make_double2(r.ist, 0.0);
  }
};

// record of an empty slot: zero number density, so every rate against it
// vanishes; finite values elsewhere
template <typename RT>
__device__ inline Rec<RT> empty_rec() {
  Rec<RT> r;
  r.m = r.im = r.St = r.ist = (RT)1;
  r.a = r.h = r.vr = r.vp = r.vz = r.nd = r.Mn = (RT)0;
  r.q1 = (RT)0.5;
  return r;
}

// both directed rates of a pair and the relative velocity
template <typename RT, bool FAST>
struct PairEval {
  __device__ static void run(const PairConst<RT> &c, const Rec<RT> &x, const Rec<RT> &y, RT &dv,
                             RT &rxy, RT &ryx) {
    const RT K = pair_kernel(c, x, y, dv);
    rxy = swarm_rate(c, x, y, K);
    ryx = swarm_rate(c, y, x, K);
  }
};
template <>
struct PairEval<float, true> {
  __device__ static void run(const PairConst<float> &c, const Rec<float> &x, const Rec<float> &y,
                             float &dv, float &rxy, float &ryx) {
    pair_rates_all(c, x, y, dv, rxy, ryx);
  }
};

// ---------------------------------------------------------------------------
// row sums of a one-wave FP32 cell, each unordered pair evaluated once
// ---------------------------------------------------------------------------
// Lane l holds slots (q, l), q < K.  Step 0 pairs the lane's own slots; step
// d = 1..32 pairs lane l with lane (l + d) mod 64 (at d = 32 only lanes below
// 32 evaluate, so every pair of lanes meets once).  r_xy goes to the lane's
// own sums; r_yx to an accumulator of the partner lane's sums that moves one
// lane down after every step (DPP wave rotation), so that the accumulator of
// lane X is always held by the lane currently paired with X; after step 32 it
// sits at lane X - 32 and returns with one exchange of the wave's halves.
// Sums are in FP32, in an order that differs from the canonical one; slots
// past the cell's particles get 0.
template <int KMAX>
__device__ inline void build_rows_pairwise(const RecStore<float> &R, const PairConst<float> &pc,
                                           int K, int lane, int n, double r[KMAX]) {
  Rec<float> mine[KMAX];
  float acc[KMAX], pacc[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    acc[q] = 0.0f;
    pacc[q] = 0.0f;
    if (q < K) mine[q] = R.load(q * 64 + lane);
  }
#pragma unroll
  for (int I = 0; I < KMAX; ++I) {
#pragma unroll
    for (int J = I; J < KMAX; ++J) {
      if (J < K) {
        float dv, rxy, ryx;
        pair_rates_all(pc, mine[I], mine[J], dv, rxy, ryx);
        acc[I] += rxy;
        if (J != I) acc[J] += ryx;
      }
    }
  }
#pragma unroll 1
  for (int d = 1; d <= 32; ++d) {
    const int c = (lane + d) & 63;
    Rec<float> pr[KMAX];
#pragma unroll
    for (int J = 0; J < KMAX; ++J)
      if (J < K) pr[J] = R.load(J * 64 + c);
    const bool take = d < 32 || lane < 32;
#pragma unroll
    for (int I = 0; I < KMAX; ++I) {
#pragma unroll
      for (int J = 0; J < KMAX; ++J) {
        if (I < K && J < K) {
          float dv, rxy, ryx;
          pair_rates_all(pc, mine[I], pr[J], dv, rxy, ryx);
          acc[I] += take ? rxy : 0.0f;
          pacc[J] += take ? ryx : 0.0f;
        }
      }
    }
    if (d < 32) {
#pragma unroll
      for (int J = 0; J < KMAX; ++J)  // lane l takes lane l + 1's accumulators
        pacc[J] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(pacc[J]), 0x134,
                                                             0xf, 0xf, false));
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const float home = __shfl_xor(pacc[q], 32, 64);
    r[q] = (q < K && lane * K + q < n) ? (double)(acc[q] + home) : 0.0;
  }
}

// Four-wave FP32 teams: the same scheme over the team's 256 lanes.  Wave a
// first pairs its own lanes as above; then in phases p = 1..3 it pairs lane
// l with lane (l + d) mod 64 of wave b = (a + p) mod 4, for d = 0..31 if
// a < b and d = 1..32 if a > b (the two waves of a pair split the 64 lane
// offsets between them).  After each phase the partner accumulators, which
// moved one lane per step as above, go to wave b through the exchange buffer
// in two rounds of two slots (a barrier after each write and before reuse).
template <int KMAX>
__device__ inline void build_rows_pairwise_team(const RecStore<float> &R, const PairConst<float> &pc,
                                                int K, int wave, int lane, int n, float2 *xbuf,
                                                double r[KMAX]) {
  static_assert(KMAX % 2 == 0, "partner sums go over in pairs of slots");
  constexpr int TL = 256;
  const int own = wave * 64;
  Rec<float> mine[KMAX];
  float acc[KMAX], pacc[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    acc[q] = 0.0f;
    pacc[q] = 0.0f;
    if (q < K) mine[q] = R.load(q * TL + own + lane);
  }
#pragma unroll
  for (int I = 0; I < KMAX; ++I) {
#pragma unroll
    for (int J = I; J < KMAX; ++J) {
      if (J < K) {
        float dv, rxy, ryx;
        pair_rates_all(pc, mine[I], mine[J], dv, rxy, ryx);
        acc[I] += rxy;
        if (J != I) acc[J] += ryx;
      }
    }
  }
  // the other lanes of the own wave
#pragma unroll 1
  for (int d = 1; d <= 32; ++d) {
    const int c = (lane + d) & 63;
    Rec<float> pr[KMAX];
#pragma unroll
    for (int J = 0; J < KMAX; ++J)
      if (J < K) pr[J] = R.load(J * TL + own + c);
    const bool take = d < 32 || lane < 32;
#pragma unroll
    for (int I = 0; I < KMAX; ++I) {
#pragma unroll
      for (int J = 0; J < KMAX; ++J) {
        if (I < K && J < K) {
          float dv, rxy, ryx;
          pair_rates_all(pc, mine[I], pr[J], dv, rxy, ryx);
          acc[I] += take ? rxy : 0.0f;
          pacc[J] += take ? ryx : 0.0f;
        }
      }
    }
    if (d < 32) {
#pragma unroll
      for (int J = 0; J < KMAX; ++J)
        pacc[J] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(pacc[J]), 0x134,
                                                             0xf, 0xf, false));
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    acc[q] += __shfl_xor(pacc[q], 32, 64);
    pacc[q] = 0.0f;
  }
  // the lanes of the other three waves
#pragma unroll 1
  for (int p = 1; p <= 3; ++p) {
    const int b = (wave + p) & 3;
    const int d0 = wave < b ? 0 : 1;
#pragma unroll 1
    for (int st = 0; st < 32; ++st) {
      const int c = (lane + d0 + st) & 63;
      Rec<float> pr[KMAX];
#pragma unroll
      for (int J = 0; J < KMAX; ++J)
        if (J < K) pr[J] = R.load(J * TL + b * 64 + c);
#pragma unroll
      for (int I = 0; I < KMAX; ++I) {
#pragma unroll
        for (int J = 0; J < KMAX; ++J) {
          if (I < K && J < K) {
            float dv, rxy, ryx;
            pair_rates_all(pc, mine[I], pr[J], dv, rxy, ryx);
            acc[I] += rxy;
            pacc[J] += ryx;
          }
        }
      }
      if (st < 31) {
#pragma unroll
        for (int J = 0; J < KMAX; ++J)
          pacc[J] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(pacc[J]), 0x134,
                                                               0xf, 0xf, false));
      }
    }
    // lane l now holds the sums of lane (l + d0 + 31) mod 64 of wave b; they
    // go over in two rounds of two slots
#pragma unroll
    for (int h = 0; h < KMAX; h += 2) {
      xbuf[b * 64 + ((lane + d0 + 31) & 63)] = make_float2(pacc[h], pacc[h + 1]);
      block_lds_sync();
      const float2 in = xbuf[own + lane];
      acc[h] += in.x;
      acc[h + 1] += in.y;
      block_lds_sync();
    }
#pragma unroll
    for (int q = 0; q < KMAX; ++q) pacc[q] = 0.0f;
  }
  const int tl = own + lane;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) r[q] = (q < K && tl * K + q < n) ? (double)acc[q] : 0.0;
}

// ---------------------------------------------------------------------------
// team: nw waves of one workgroup, runtime size
// ---------------------------------------------------------------------------
struct Team {
  int nw, wave, lane, tl;
  TeamScratch *S;
  int phase;
  __device__ void sync() const {
    if (nw > 1)
      block_lds_sync();
    else
      wave_lds_sync();
  }
  // the four wave totals of exchange slot k (two 16-byte LDS reads)
  __device__ void totals4(int k, double t[4]) const {
    const double2 a = ((const double2 *)S->tot[phase])[2 * k];
    const double2 b = ((const double2 *)S->tot[phase])[2 * k + 1];
    t[0] = a.x;
    t[1] = a.y;
    t[2] = b.x;
    t[3] = b.y;
  }
  // team-inclusive prefix of x over team lanes; total on every lane.  Teams
  // have one wave or four; the offset and total add the wave totals in wave
  // order
  __device__ double scan(double x, double &total) {
    const double inc = wave_incl_scan(x);
    const double wt = readlane_d(inc, 63);
    if (nw == 1) {
      total = wt;
      return inc;
    }
    phase ^= 1;
    if (lane == 63) S->tot[phase][wave] = wt;
    block_lds_sync();
    double t[4];
    totals4(0, t);
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (w < wave) off += t[w];
      tot += t[w];
    }
    total = tot;
    return off + inc;
  }
  // team-inclusive prefix of a plus the totals of a and b (one exchange); b
  // is summed over each wave in its own precision (BT), then in FP64
  template <typename BT>
  __device__ double scan2(double a, BT b, double &tot_a, double &tot_b) {
    const double ia = wave_incl_scan(a);
    const BT ib = wave_incl_scan(b);
    const double wa = readlane_d(ia, 63), wb = (double)readlane_t(ib, 63);
    if (nw == 1) {
      tot_a = wa;
      tot_b = wb;
      return ia;
    }
    phase ^= 1;
    if (lane == 63) {
      S->tot[phase][wave] = wa;
      S->tot[phase][4 + wave] = wb;
    }
    block_lds_sync();
    double ta4[4], tb4[4];
    totals4(0, ta4);
    totals4(1, tb4);
    double off = 0.0, ta = 0.0, tb = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (w < wave) off += ta4[w];
      ta += ta4[w];
      tb += tb4[w];
    }
    tot_a = ta;
    tot_b = tb;
    return off + ia;
  }
};

// particle state after a collision: FP64 formulas for the FP64 path, the
// FP32 formulas with per-cell FP32 factors for the mixed path
template <typename RT>
struct RecAfter;
template <>
struct RecAfter<double> {
  __device__ static Rec<double> get(const Model &P, const TeamScratch *S, double m, double M,
                                    double) {
    return make_rec<double>(P, S->gas, m, M, 1.0);
  }
};
template <>
struct RecAfter<float> {
  __device__ static Rec<float> get(const Model &, const TeamScratch *S, double m, double,
                                   float Mn) {
    return make_rec_f(S->cf, m, Mn);
  }
};

// ---------------------------------------------------------------------------
// selection: the first slot whose cumulative value exceeds a target
// ---------------------------------------------------------------------------
// Search inside one wave.  v[] are the lane's K values in canonical order,
// part their sum, incl the team-inclusive prefix of part.  The chosen lane is
// the first with incl > target and a nonzero partial (the team prefix is not
// exactly monotone under rounding), else the wave's last lane with a nonzero
// partial; inside it, the first slot whose running sum exceeds the target,
// else its last nonzero slot.  Fills c (team lane, slot, payloads a0[q],
// a1[q], ai[q], and whether a lane passed the target) uniformly over the
// wave; false if no lane of the wave has a nonzero partial.
template <int KMAX, typename VT, typename PT>
__device__ inline bool wave_pick(int wave, double incl, double part, const VT *v, int K,
                                 double target, const double *a0, const PT *a1, const int *ai,
                                 Cand &c) {
  const bool pos = part > 0.0;
  const uint64_t bf = ballot(pos);
  if (bf == 0) return false;
  const int first = first_set(ballot(pos && incl > target));
  const int src = first >= 0 ? first : last_set(bf);
  // every lane searches its own slots as if it owned the pick (no divergent
  // code); the owner's slot is read afterwards, then its payloads with a
  // wave-uniform slot index
  double cum = incl - part;
  int qhit = -1, last = -1;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q < K) {
      last = v[q] > (VT)0 ? q : last;
      cum += (double)v[q];
      qhit = (qhit < 0 && cum > target) ? q : qhit;
    }
  }
  const int qs = readlane_i((first >= 0 && qhit >= 0) ? qhit : last, src);
  c.q = qs;
  c.lane = wave * 64 + src;
  c.hit = first >= 0 ? 1 : 0;
  c.p0 = c.p1 = 0.0;
  c.gi = -1;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q == qs) {
      c.p0 = readlane_d(a0[q], src);
      c.p1 = readlane_d((double)a1[q], src);
      c.gi = readlane_i(ai[q], src);
    }
  }
  return true;
}

// The wave of a multi-wave team that holds the target: the first whose
// team-inclusive prefix at its last lane exceeds it.  That prefix is rebuilt
// from the wave totals of the latest exchange with the same FP64 operations
// the lanes used (offset of the earlier waves, plus the wave's total, plus
// delta from team lane 64 fix_wave on), so every wave finds the same owner
// without another exchange.  -1 if no wave's prefix exceeds the target.
__device__ inline int owner_wave(const Team &tm, double target, int fix_wave, double delta) {
  double t[4];
  tm.totals4(0, t);
  double off = 0.0;
  int ow = -1;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    double cum = off + t[w];
    if (w >= fix_wave) cum += delta;
    if (ow < 0 && cum > target) ow = w;
    off += t[w];
  }
  return ow;
}

// Every wave searches and publishes its candidate; the team takes the first
// wave with a lane past the target, else the last wave with any nonzero
// partial.  q < 0: nothing to pick.
template <int KMAX, typename VT, typename PT>
__device__ inline Cand pick_all_waves(Team &tm, double incl, double part, const VT *v, int K,
                                      double target, const double *a0, const PT *a1,
                                      const int *ai) {
  Cand h{0.0, 0.0, -1, -1, 0, -1};
  if (!wave_pick<KMAX>(tm.wave, incl, part, v, K, target, a0, a1, ai, h)) h.q = -1;
  tm.phase ^= 1;
  if (tm.lane == 0) tm.S->cand[tm.phase][tm.wave] = h;
  block_lds_sync();
  int wsel = -1;
  for (int w = tm.nw - 1; w >= 0; --w) {
    const Cand &x = tm.S->cand[tm.phase][w];
    if (x.q >= 0 && x.hit) wsel = w;
  }
  if (wsel < 0) {
    for (int w = 0; w < tm.nw; ++w)
      if (tm.S->cand[tm.phase][w].q >= 0) wsel = w;
  }
  if (wsel < 0) return Cand{0.0, 0.0, -1, -1, 0, -1};
  return tm.S->cand[tm.phase][wsel];
}

// Team-wide selection: one wave searches (the owner of the target) and
// publishes; if rounding leaves no lane of that wave past the target, every
// wave searches (pick_all_waves).  The same result on every lane of the team.
template <int KMAX, typename VT, typename PT>
__device__ inline Cand team_pick(Team &tm, double incl, double part, const VT *v, int K,
                                 double target, int fix_wave, double delta, const double *a0,
                                 const PT *a1, const int *ai) {
  Cand c{0.0, 0.0, -1, -1, 0, -1};
  if (tm.nw == 1) {
    if (!wave_pick<KMAX>(0, incl, part, v, K, target, a0, a1, ai, c)) c.q = -1;
    return c;
  }
  const int ow = owner_wave(tm, target, fix_wave, delta);
  tm.phase ^= 1;
  if (tm.wave == ow) {
    if (!wave_pick<KMAX>(tm.wave, incl, part, v, K, target, a0, a1, ai, c) || !c.hit) c.q = -1;
    if (tm.lane == 0) tm.S->cand[tm.phase][0] = c;
  }
  block_lds_sync();
  if (ow >= 0) {
    c = tm.S->cand[tm.phase][0];
    if (c.q >= 0) return c;
  }
  return pick_all_waves<KMAX>(tm, incl, part, v, K, target, a0, a1, ai);
}

// Outcome of an event for i (mass mi, swarm mass Mi; the FP32 form takes the
// record's Mn instead) hitting j's swarm (mass mj) at relative velocity dvj:
// new mass, outcome code and i's new record.
// The writer also applies the side effects: the anomaly flag and the
// mass-weighted composition of i on sticking or fragmentation (lanes below
// n_comp, one component each).
// PROB: the probabilistic fragmentation criteria (a kernel variant of its
// own, so that the sharp criterion carries none of their special functions);
// u5 is their uniform, from Philox (e, cell, step, 3).  The FP64 form takes
// the probability in FP64; the mixed form, whose relative velocity is FP32,
// in FP32
template <typename RT, bool PROB>
__device__ inline int event_outcome(const CollideArgs &A, const TeamScratch *S, double mi,
                                    double mj, double Mi, RT Mn, RT dvj, double u4, double u5,
                                    int gi, int gj, int lane, bool writer, double &mnew,
                                    Rec<RT> &rin) {
  const OutcomeConst &P = S->oc;
  bool fast;
  if constexpr (PROB) {
    fast = u5 < (double)frag_probability(P, dvj);
  } else {
    fast = !(dvj < (RT)P.v_frag);
  }
  const int oc = outcome<sizeof(RT) == 8>(P, fast, mi, mj, u4, mnew);
  if (writer && (!(mnew > 0.0) || !isfinite(mnew)) && lane == 0)
    atomicOr(&A.state->flags, FLAG_BAD_MASS);
  rin = RecAfter<RT>::get(A.P, S, mnew, Mi, Mn);
  return oc;
}

// Composition of i after a sticking or fragmenting event: mass-weighted mix
// of i's fractions (weight m_i) and j's (weight g m_j), one component per
// lane below n_comp.  The fractions are loaded as soon as i and j are known
// (comp_load) and the mix is stored early in the next event, once its i is
// chosen, or when the cell ends (comp_store): the loads then have the rest of
// the event and the next event's selection of i to arrive instead of
// stalling the chain.  The next event's own loads come after that store, and
// a load of a lane after its own store to the same address reads the store.
struct CompMix {
  float cI, cJ;
  bool on;
};
__device__ inline CompMix comp_load(const CollideArgs &A, int lane, bool writer, int gi, int gj) {
  CompMix c{0.0f, 0.0f, false};
  if (writer && A.comp != nullptr && lane < A.P.n_comp) {
    // the component's base is formed here, per event, not held (or spilled)
    // across the event loop
    const float *cs = A.comp + (size_t)opaque_v(lane) * A.N;
    c.cI = cs[gi];
    c.cJ = cs[gj];
    c.on = true;
  }
  return c;
}
template <bool EXACT>
__device__ inline void comp_store(const CollideArgs &A, const CompMix &c, int lane, int oc, int gi,
                                  double mi, double mj) {
  if (c.on && (oc == OUT_STICK || oc == OUT_FRAG)) {
    // the grouped mass g m_j as the outcome formed it
    double wj;
    if (EXACT) {
      wj = group_factor(A.P.dm_max, mi, mj) * mj;
    } else {
      const double d = A.P.dm_max * mi;
      wj = (A.P.dm_max > 0.0 && d > mj) ? d : mj;
    }
    A.comp[(size_t)opaque_v(lane) * A.N + gi] =
        (float)((mi * (double)c.cI + wj * (double)c.cJ) / (mi + wj));
  }
}

__device__ inline void log_event(const CollideArgs &A, int cell, uint32_t e, int i_local,
                                 int j_local, int oc) {
  if (A.evlog != nullptr && (int64_t)e < A.log_per_cell) {
    int32_t *L = A.evlog + ((size_t)cell * A.log_per_cell + e) * 4;
    L[0] = i_local;
    L[1] = j_local;
    L[2] = oc;
    L[3] = 0;
  }
}

// the event budget a kernel is compiled for: a fixed number of events per
// cell (dt = 0), a time limit dt > 0, or either, read from the arguments
enum : int { kFixedCount = 0, kTimeLimited = 1, kEitherLimit = 2 };

// AUX: the composition mix and the event log are compiled in (a launch with
// fractions to track or events to record); without them the event loop
// carries neither.  LIMIT: a kernel compiled for fixed counts only carries no
// waiting times (their logarithm, the time test, the priority rule)
template <typename RT, int KMAX, bool FAST, bool PROB, bool AUX, int NW, int LIMIT = kEitherLimit>
__device__ void process_cell(const CollideArgs &A, int cell, char *base, int cap, int wave,
                             int lane, uint32_t step) {
  constexpr int nw = NW;  // waves of the team: 1, or 4 (a compile-time shape per cell body)
  const int s0 = __builtin_amdgcn_readfirstlane(A.cell_start[cell]);
  const int n = __builtin_amdgcn_readfirstlane(A.cell_start[cell + 1]) - s0;
  if (n <= 0) return;
  const int TL = 64 * nw;
  const int K = (n + TL - 1) / TL;
  const RecStore<RT> R(base, cap);
  Team tm;
  tm.nw = nw;
  tm.wave = wave;
  tm.lane = lane;
  tm.tl = wave * 64 + lane;
  tm.S = (TeamScratch *)(base + (size_t)cap * rec_bytes<RT>());
  tm.phase = 0;
  const int tl = tm.tl;
  if (K > KMAX || K * TL > cap) {
    if (tl == 0) atomicOr(&A.state->flags, FLAG_CAPACITY);
    return;
  }
  Gas g;
  {
    // grid sizes opaque per cell: the node lookups' bounds are formed here
    // instead of being held through every cell of a persistent launch
    Model Pl = A.P;
    Pl.grid.nr = opaque_u(Pl.grid.nr);
    Pl.grid.nz = opaque_u(Pl.grid.nz);
    gas_from_primaries(Pl, A.gas + (size_t)cell * 6, g);
  }
  if (!(g.V > 0.0)) {
    if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_VOLUME);
    return;
  }
  const PairConst<RT> pc = make_pair_const<RT>(A.P, g);

  // ---- members: masses and indices stay in the owning lane's registers ---
  double m64[KMAX];
  int gix[KMAX];
  double ndmax = 0.0;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const int j = tl * K + q;
    gix[q] = -1;
    m64[q] = 1.0;
    if (q < K && j < n) {
      gix[q] = A.order[s0 + j];
      m64[q] = A.m[gix[q]];
      ndmax = fmax(ndmax, A.M[gix[q]] / (m64[q] * g.V));
    }
  }
  double scale = 1.0;  // FP32 rates are carried as r * scale, a power of two
  if (sizeof(RT) == 4) {
    ndmax = wave_max_nonneg(ndmax);
    if (nw > 1) {
      if (lane == 0) tm.S->tot[0][wave] = ndmax;
      block_lds_sync();
      for (int w = 0; w < nw; ++w) ndmax = fmax(ndmax, tm.S->tot[0][w]);
      block_lds_sync();
    }
    int e2 = 0;
    frexp(ndmax, &e2);
    scale = ldexp(1.0, -e2);
  }
  if (tl == 0) {
    tm.S->gas = g;
    tm.S->cf = make_cellf(A.P, g, scale);
    tm.S->oc = make_outcome_const(A.P);
  }
  uint32_t valid = 0;  // bit q: slot q holds a particle
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q < K) {
      const bool v = tl * K + q < n;
      valid |= v ? (1u << q) : 0u;
      R.store(q * TL + tl, v ? make_rec<RT>(A.P, g, m64[q], A.M[gix[q]], scale) : empty_rec<RT>());
    }
  }
  tm.sync();

  // ---- row sums r_i = sum_k r_ik ------------------------------------------
  // The FP32 form evaluates each unordered pair once (build_rows_pairwise,
  // build_rows_pairwise_team).  Otherwise partners k = 0..n-1 are read once per
  // group of G own slots and paired with each of them (independent
  // evaluations), and each row adds its terms in canonical order.
  double r[KMAX];
  bool built = false;
  if constexpr (sizeof(RT) == 4 && FAST && KMAX == 4) {
    if (nw == 1)
      build_rows_pairwise<KMAX>(R, pc, K, lane, n, r);
    else
      build_rows_pairwise_team<KMAX>(R, pc, K, wave, lane, n,
                                     (float2 *)(base + xbuf_offset<RT>(cap)), r);
    built = true;
  }
  if (!built) {
    constexpr int G = sizeof(RT) == 4 ? 4 : 2;
    static_assert(KMAX % G == 0, "slot groups");
#pragma unroll
    for (int q0 = 0; q0 < KMAX; q0 += G) {
      Rec<RT> mine[G];
      RT acc[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        acc[g] = (RT)0;
        if (q0 + g < K) mine[g] = R.load((q0 + g) * TL + tl);
      }
      if (q0 < K) {
        int t2 = 0, q2 = 0;
        for (int k = 0; k < n; ++k) {
          const Rec<RT> rk = R.load(q2 * TL + t2);
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (q0 + g < K) {
              RT dv, rxy, ryx;
              PairEval<RT, FAST>::run(pc, mine[g], rk, dv, rxy, ryx);
              acc[g] += rxy;
            }
          }
          if (++q2 == K) {
            q2 = 0;
            ++t2;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
        r[q0 + g] = (q0 + g < K && tl * K + q0 + g < n) ? (double)acc[g] : 0.0;
    }
  }

  if (A.rowsum_dump != nullptr) {
    // test path: the starting row sums as built above, unscaled, at the
    // members' positions in the cell order; no events
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < K && tl * K + q < n) A.rowsum_dump[s0 + tl * K + q] = r[q] / scale;
    tm.sync();
    return;
  }

  // ---- events ------------------------------------------------------------
  double t = 0.0;
  uint32_t e = 0;  // events so far (fewer than 2^32 per cell and step)
  uint32_t oc_count[4] = {0u, 0u, 0u, 0u};
  const uint32_t c32 = (uint32_t)cell;
  const bool timed = LIMIT == kEitherLimit ? A.dt > 0.0 : LIMIT == kTimeLimited;
  const uint32_t emax = A.max_events > 0 ? (uint32_t)A.max_events : 0xFFFFFFFFu;
  double part = 0.0, Rtot;
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (q < K) part += r[q];
  double incl = tm.scan(part, Rtot);
  // time-limited steps: a cell whose expected event count R dt is large is a
  // long serial chain that can outlast every other cell of the step, so its
  // waves get a higher issue priority on their SIMD (the rest fill in around
  // them); back to the default when the cell is done
  if (timed) {
    const double expect = Rtot / scale * A.dt;
    if (expect >= 256.0)
      __builtin_amdgcn_s_setprio(3);
    else if (expect >= 64.0)
      __builtin_amdgcn_s_setprio(2);
    else if (expect >= 16.0)
      __builtin_amdgcn_s_setprio(1);
  }
  // lanes from team lane 64 fix_wave on carry delta on top of the latest
  // scanned prefix (the new row sum of the previous event's i)
  int fix_wave = nw;
  double delta = 0.0;
  // uniforms of 64 consecutive events: lane l holds -ln u1, u2, u3, u4 of
  // event e0 + l from Philox(e0 + l, cell, step, 0) and (.., 1)
  double nlu1 = 0.0, uu2 = 0.0, uu3 = 0.0, uu4 = 0.0, uu5 = 0.0;
  uint32_t e0 = 0u - 64u;  // first event of the current batch (none yet)
  // the previous event's composition mix, not yet stored
  CompMix pcm{0.0f, 0.0f, false};
  int p_oc = 0, p_gi = 0;
  double p_mi = 0.0, p_mj = 0.0;
  const int K_cell = K, lane_cell = lane, wave_cell = wave;
  for (;;) {
    // K and the lane / wave indices per event: tests such as q < K, w < wave
    // or lane == 63 are made where they are needed instead of being kept as
    // lane masks across the loop
    const int K = opaque_s(K_cell);
    tm.lane = opaque_v(lane_cell);
    tm.wave = opaque_s(wave_cell);
    if (!(Rtot > 0.0) || !isfinite(Rtot)) {
      if (!isfinite(Rtot)) {
        if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_RATE);
        break;
      }
      // the running total (the last scan plus the change of r_i) can round
      // to zero while a row sum still holds a positive remainder: the cell
      // is done only when a fresh sum of the row sums is zero, as in the
      // method's definition of R
      if (fix_wave == nw) break;
      part = 0.0;
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < K) part += r[q];
      incl = tm.scan(part, Rtot);
      fix_wave = nw;
      delta = 0.0;
      if (!(Rtot > 0.0)) break;
    }
    if (e >= emax) break;
    if (e - e0 >= 64) {
      e0 = e;
      const uint32_t ec = (uint32_t)(e + lane);
      // the key schedule is formed here, once per 64 events, not held
      const uint32_t k0 = opaque_u(A.P.key0), k1 = opaque_u(A.P.key1);
      const U4 w0 = philox4x32_10(U4{ec, c32, step, 0u}, k0, k1);
      const U4 w1 = philox4x32_10(U4{ec, c32, step, 1u}, k0, k1);
      if (timed) nlu1 = -log(u01(w0.x, w0.y));
      uu2 = u01(w0.z, w0.w);
      uu3 = u01(w1.x, w1.y);
      uu4 = u01(w1.z, w1.w);
      if constexpr (PROB) {  // the fragmentation uniform u5
        const U4 w3 = philox4x32_10(U4{ec, c32, step, 3u}, k0, k1);
        uu5 = u01(w3.x, w3.y);
      }
    }
    const int rl = (int)(e - e0);
    double t_next = t;
    if (timed) {
      // exponential waiting time; the FP32 form takes 1/R from the hardware
      // estimate and one Newton step
      double tau;
      if constexpr (sizeof(RT) == 4) {
        double ir = __builtin_amdgcn_rcp(Rtot);
        ir = fma(fma(-Rtot, ir, 1.0), ir, ir);
        tau = readlane_d(nlu1, rl) * ir * scale;
      } else {
        tau = readlane_d(nlu1, rl) / Rtot * scale;
      }
      if (t + tau > A.dt) break;  // the next event falls outside the step
      t_next = t + tau;
    }

    // -- choose i by cumulative row sums (payloads: m_i, old r_i, index)
    const Cand ci = team_pick<KMAX>(tm, incl, part, r, K, readlane_d(uu2, rl) * Rtot, fix_wave,
                                    delta, m64, r, gix);
    if (ci.q < 0) {
      // no row sum is positive in the running prefixes: decide on a fresh
      // sum (a total of rounding remainders ends the cell; a positive fresh
      // total retries the event on the fresh prefixes)
      if (fix_wave != nw) {
        part = 0.0;
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
          if (q < K) part += r[q];
        incl = tm.scan(part, Rtot);
        fix_wave = nw;
        delta = 0.0;
        if (!(Rtot > 0.0)) break;
        continue;
      }
      if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_RATE);
      break;
    }
    if constexpr (AUX) {
      if (pcm.on) {
        comp_store<sizeof(RT) == 8>(A, pcm, lane, p_oc, p_gi, p_mi, p_mj);
        pcm.on = false;
      }
    }
    t = t_next;
    const int si = ci.q * TL + ci.lane;
    const int i_local = ci.lane * K + ci.q;
    const double mi = ci.p0, ri_old = ci.p1;
    const int gi = ci.gi;
    // the FP64 state of i is rebuilt from its swarm mass (the load overlaps
    // row i); the FP32 record carries it
    const double Mi = sizeof(RT) == 8 ? A.M[gi] : 0.0;
    const Rec<RT> ri = R.load(si);

    // -- row i before the event: r_ij, r_ji and the relative velocities
    RT rij[KMAX], rji[KMAX], dvv[KMAX];
    double part1 = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      rij[q] = (RT)0;
      rji[q] = (RT)0;
      dvv[q] = (RT)0;
      if (q < K) {  // empty slots have zero density: rij = 0
        const Rec<RT> rq = R.load(q * TL + tl);
        PairEval<RT, FAST>::run(pc, ri, rq, dvv[q], rij[q], rji[q]);
      }
      part1 += (double)rij[q];
    }
    double Ri;
    const double incl1 = tm.scan(part1, Ri);
    if (!(Ri > 0.0)) {
      // row i has no partner left (its stored sum was rounding residue):
      // clear it and count a null event
      if (tl == ci.lane) {
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
          if (q == ci.q) r[q] = 0.0;
      }
      if constexpr (AUX) {
        if (tl == 0) log_event(A, cell, e, i_local, -1, -1);
      }
      ++e;
      part = 0.0;
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < K) part += r[q];
      incl = tm.scan(part, Rtot);
      fix_wave = nw;
      delta = 0.0;
      continue;
    }

    // -- choose j (payloads: m_j, relative velocity, index), then the outcome
    // (only i changes), computed alike by every wave; wave 0 writes
    const Cand cj = team_pick<KMAX>(tm, incl1, part1, rij, K, readlane_d(uu3, rl) * Ri, nw, 0.0,
                                    m64, dvv, gix);
    CompMix cm{0.0f, 0.0f, false};
    if constexpr (AUX) cm = comp_load(A, lane, wave == 0, gi, cj.gi);
    double mnew = 0.0;
    Rec<RT> rin;
    const int oc = event_outcome<RT, PROB>(A, tm.S, mi, cj.p0, Mi, ri.Mn, (RT)cj.p1,
                                           readlane_d(uu4, rl),
                                           PROB ? readlane_d(uu5, rl) : 0.0, gi, cj.gi, lane,
                                           wave == 0, mnew, rin);
    if constexpr (AUX) {
      if (tl == 0) log_event(A, cell, e, i_local, cj.lane * K + cj.q, oc);
    }
    // the owner of i keeps the new mass and record; it alone reads the slot
    // until the next exchange
    if (tl == ci.lane) {
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q == ci.q) m64[q] = mnew;
      R.store(si, rin);
    }

    // -- new row i: incremental update of the other rows, fresh row sum of i
    // the fresh row sum of i: in the rate precision within a wave (the FP32
    // tree adds no more than the rates' own rounding), then FP64
    RT part2 = (RT)0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (q < K) {
        const int s = q * TL + tl;
        const Rec<RT> rq = R.load(s);
        RT dv, a_iq, a_qi;
        PairEval<RT, FAST>::run(pc, rin, rq, dv, a_iq, a_qi);
        part2 += a_iq;
        // FP64: old term out, new term in, as the oracle orders them; FP32:
        // the change of r_qi in FP32 (one rounding of a difference far
        // below the row sum), then one FP64 addition
        const double x = sizeof(RT) == 8 ? (r[q] - (double)rji[q]) + (double)a_qi
                                         : r[q] + (double)(a_qi - rji[q]);
        const bool upd = s != si && ((valid >> q) & 1u);
        r[q] = upd ? (x > 0.0 ? x : 0.0) : r[q];
      }
    }
    // next event's prefix of the row sums and the new r_i in one exchange;
    // the owner's slot still holds the old r_i and is corrected afterwards
    part = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < K) part += r[q];
    double ri_new;
    incl = tm.scan2(part, part2, Rtot, ri_new);
    delta = ri_new - ri_old;
    fix_wave = ci.lane >> 6;
    if (tl >= ci.lane) incl += delta;
    Rtot += delta;
    if (tl == ci.lane) {
      part += delta;
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q == ci.q) r[q] = ri_new;
    }
    if constexpr (AUX) {
      pcm = cm;
      p_oc = oc;
      p_gi = gi;
      p_mi = mi;
      p_mj = cj.p0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) oc_count[k] += (oc == k) ? 1u : 0u;
    ++e;
  }
  if constexpr (AUX) {
    if (pcm.on) comp_store<sizeof(RT) == 8>(A, pcm, lane, p_oc, p_gi, p_mi, p_mj);
  }
  // masses back to HBM
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (q < K && tl * K + q < n) A.m[gix[q]] = m64[q];
  if (tl == 0) {
    atomicAdd(&A.state->events, (unsigned long long)e);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (oc_count[k]) atomicAdd(&A.state->outcomes[k], (unsigned long long)oc_count[k]);
  }
  __builtin_amdgcn_s_setprio(0);
  tm.sync();  // the region is reused by the next cell
}

// ---------------------------------------------------------------------------
// batched schedule: one persistent launch of four-wave workgroups; big cells
// on four-wave teams (largest first), then small cells on single waves
// (largest first), each wave popping its own work
// ---------------------------------------------------------------------------
template <typename RT, int KMAX, bool FAST, bool PROB, bool AUX, int LIMIT = kEitherLimit>
__global__ __launch_bounds__(256, sizeof(RT) == 4 ? 3 : 2) void collide_batched(CollideArgs A) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint32_t step = A.state->step;
  const size_t small_bytes = region_bytes<RT>(A.small_cap, 1);
  // list lengths from the device plan (zero for a grid that failed validation)
  const int n_big = __builtin_amdgcn_readfirstlane(A.plan->n_big);
  const int n_small = __builtin_amdgcn_readfirstlane(A.plan->n_small);
  int nw = n_big > 0 ? 4 : 1;
  for (;;) {
    int cell = -1;
    if (nw == 4) {
      if (threadIdx.x == 0) s_item = atomicAdd(&A.state->big_head, 1);
      __syncthreads();
      const int item = __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();
      if (item < n_big)
        cell = __builtin_amdgcn_readfirstlane(A.big_list[item]);
      else
        nw = 1;
    }
    if (nw == 1) {
      int item = 0;
      if (lane == 0) item = atomicAdd(&A.state->small_head, 1);
      item = readlane_i(item, 0);
      if (item >= n_small) break;
      cell = __builtin_amdgcn_readfirstlane(A.small_list[item]);
    }
    if (nw == 4)
      process_cell<RT, KMAX, FAST, PROB, AUX, 4, LIMIT>(A, cell, smem, A.big_cap, wave, lane, step);
    else
      process_cell<RT, KMAX, FAST, PROB, AUX, 1, LIMIT>(A, cell, smem + (size_t)wave * small_bytes,
                                                  A.small_cap, 0, lane, step);
  }
}

// plain schedule: one four-wave workgroup per cell, cells in index order
template <typename RT, int KMAX, bool FAST, bool PROB>
__global__ __launch_bounds__(256) void collide_plain(CollideArgs A) {
  extern __shared__ __align__(16) char smem[];
  if (A.plan->bad) return;  // an explicit grid that failed validation
  // the composition mix and the event log are compiled in; they apply when
  // fractions are given or a log is set
  process_cell<RT, KMAX, FAST, PROB, true, 4>(A, blockIdx.x, smem, A.big_cap,
                                              __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                                              threadIdx.x & 63, A.state->step);
}

}  // namespace mcd
