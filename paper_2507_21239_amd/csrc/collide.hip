// collide.hip -- the per-cell collision Monte Carlo of the representative-
// particle method (Zsom & Dullemond 2008, adopted by the paper, Summary):
// build the row sums r_i = sum_j r_ij of the cell's rate matrix, then repeat
// events: exponential waiting time from the total rate R, choose i by the
// cumulative row sums, choose j by the cumulative rates of row i, apply the
// outcome (sticking / erosion / fragmentation) to i only, update every row
// sum incrementally for the changed particle and recompute row i.
//
// A cell is processed by a team of nw waves (1, or 4 for cells above 256
// particles).  The cell's n particles are in canonical order j = 0..n-1; team
// lane t owns the contiguous slots j = t*K .. t*K+K-1 (K = ceil(n/(64 nw))),
// so the cumulative rate of j is the team prefix of the lanes' partial sums
// plus a short in-lane prefix.  Prefix sums are FP64 DPP scans; four-wave
// teams exchange wave totals through LDS (two barriers per selection, one
// for the new row sum).  Particle records live in LDS as packed vectors
// indexed by s = q*64nw + t (slot q of lane t), so a wave reads consecutive
// 16-byte words.  Row sums (FP64), the per-event row values, masses and
// particle indices stay in registers of the owning lane; masses go back to
// HBM once, when the cell is done.
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
  float4 *C;  // nd, m, ist, -
  __device__ RecStore(char *base, int cap)
      : A((float4 *)base), B((float4 *)base + cap), C((float4 *)base + 2 * cap) {}
  __device__ Rec<float> load(int s) const {
    const float4 a = A[s], b = B[s], c = C[s];
    Rec<float> r;
    r.im = a.x; r.a = a.y; r.St = a.z; r.h = a.w;
    r.q1 = b.x; r.vr = b.y; r.vp = b.z; r.vz = b.w;
    r.nd = c.x; r.m = c.y; r.ist = c.z;
    return r;
  }
  __device__ void store(int s, const Rec<float> &r) const {
    A[s] = make_float4(r.im, r.a, r.St, r.h);
    B[s] = make_float4(r.q1, r.vr, r.vp, r.vz);
    C[s] = make_float4(r.nd, r.m, r.ist, 0.0f);
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
  r.a = r.h = r.vr = r.vp = r.vz = r.nd = (RT)0;
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
  // team-inclusive prefix of x over team lanes; total on every lane
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
    double off = 0.0, tot = 0.0;
    for (int w = 0; w < nw; ++w) {
      const double v = S->tot[phase][w];
      if (w < wave) off += v;
      tot += v;
    }
    total = tot;
    return off + inc;
  }
  // team-inclusive prefix of a plus the totals of a and b (one exchange)
  __device__ double scan2(double a, double b, double &tot_a, double &tot_b) {
    const double ia = wave_incl_scan(a);
    const double ib = wave_incl_scan(b);
    const double wa = readlane_d(ia, 63), wb = readlane_d(ib, 63);
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
    double off = 0.0, ta = 0.0, tb = 0.0;
    for (int w = 0; w < nw; ++w) {
      const double v = S->tot[phase][w];
      if (w < wave) off += v;
      ta += v;
      tb += S->tot[phase][4 + w];
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
  __device__ static Rec<double> get(const Model &P, const TeamScratch *S, double m, double M) {
    return make_rec<double>(P, S->gas, m, M, 1.0);
  }
};
template <>
struct RecAfter<float> {
  __device__ static Rec<float> get(const Model &, const TeamScratch *S, double m, double M) {
    return make_rec_f(S->cf, m, M);
  }
};

// Pick the first slot whose cumulative value exceeds target.  v[] are the
// lane's K values in canonical order, part their sum, incl the team-inclusive
// prefix of part.  A lane with an empty partial is never chosen (the team
// prefix is not exactly monotone under rounding); if rounding leaves no
// prefix above the target, the last nonzero entry is taken.  Returns the
// chosen slot, its owner and the owner's payloads a0[q], a1[q], a2[q], ai[q]
// on every lane of the team.
template <int KMAX, typename VT, typename P2>
__device__ inline Cand team_pick(Team &tm, double incl, double part, const VT *v, int K,
                                 double target, const double *a0, const double *a1,
                                 const P2 *a2, const int *ai) {
  const bool hit = incl > target && part > 0.0;
  const uint64_t bh = ballot(hit), bf = ballot(part > 0.0);
  const int first = first_set(bh);
  const int src = first >= 0 ? first : last_set(bf);
  // every lane searches its own slots as if it owned the pick (no divergent
  // code); the owner's answer is read afterwards
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
  const int qsel = (first >= 0 && qhit >= 0) ? qhit : last;
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  int gi = -1;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const bool m = q == qsel;
    p0 = m ? a0[q] : p0;
    p1 = m ? a1[q] : p1;
    p2 = m ? (double)a2[q] : p2;
    gi = m ? ai[q] : gi;
  }
  Cand o{0.0, 0.0, 0.0, -1, -1, first >= 0 ? 1 : 0, -1};
  if (src < 0) {
    if (tm.nw == 1) return o;
  } else {
    o.q = readlane_i(qsel, src);
    o.lane = tm.wave * 64 + src;
    o.gi = readlane_i(gi, src);
    o.p0 = readlane_d(p0, src);
    o.p1 = readlane_d(p1, src);
    o.p2 = readlane_d(p2, src);
    if (tm.nw == 1) return o;
  }
  tm.phase ^= 1;
  if (tm.lane == 0) tm.S->cand[tm.phase][tm.wave] = o;
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
  if (wsel < 0) {
    Cand z{0.0, 0.0, 0.0, -1, -1, 0, -1};
    return z;
  }
  return tm.S->cand[tm.phase][wsel];
}

template <typename RT, int KMAX, bool FAST>
__device__ void process_cell(const CollideArgs &A, int cell, char *base, int cap, int nw, int wave,
                             int lane, uint32_t step) {
  const int s0 = A.cell_start[cell];
  const int n = A.cell_start[cell + 1] - s0;
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
  gas_from_primaries(A.P, A.gas + (size_t)cell * 6, g);
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

  // ---- row sums r_i = sum_k r_ik, k in canonical order ------------------
  double r[KMAX];
  const int lanes_used = (n + K - 1) / K;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) r[q] = 0.0;
#pragma unroll 1
  for (int q = 0; q < K; ++q) {
    if (tl * K + q >= n) break;
    const Rec<RT> mine = R.load(q * TL + tl);
    RT acc = (RT)0;
    for (int t2 = 0; t2 < lanes_used; ++t2) {
      for (int q2 = 0; q2 < K; ++q2) {
        if (t2 * K + q2 >= n) break;
        const Rec<RT> rk = R.load(q2 * TL + t2);
        RT dv, rxy, ryx;
        PairEval<RT, FAST>::run(pc, mine, rk, dv, rxy, ryx);
        acc += rxy;
      }
    }
#pragma unroll
    for (int qq = 0; qq < KMAX; ++qq)
      if (qq == q) r[qq] = (double)acc;
  }

  // ---- events ------------------------------------------------------------
  double t = 0.0;
  int64_t e = 0;
  uint32_t oc_count[4] = {0u, 0u, 0u, 0u};
  const uint32_t c32 = (uint32_t)cell;
  const bool timed = A.dt > 0.0;
  double part = 0.0, Rtot;
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (q < K) part += r[q];
  double incl = tm.scan(part, Rtot);
  // random words of 64 consecutive events: lane l holds Philox(e0 + l, cell,
  // step, 0) and Philox(e0 + l, cell, step, 1); an event reads its lane
  U4 rw0{0u, 0u, 0u, 0u}, rw1{0u, 0u, 0u, 0u};
  int64_t e0 = -64;
  for (;;) {
    if (!(Rtot > 0.0) || !isfinite(Rtot)) {
      if (!isfinite(Rtot) && tl == 0) atomicOr(&A.state->flags, FLAG_BAD_RATE);
      break;
    }
    if (A.max_events > 0 && e >= A.max_events) break;
    if (e - e0 >= 64) {
      e0 = e;
      const uint32_t ec = (uint32_t)(e + lane);
      rw0 = philox4x32_10(U4{ec, c32, step, 0u}, A.P.key0, A.P.key1);
      rw1 = philox4x32_10(U4{ec, c32, step, 1u}, A.P.key0, A.P.key1);
    }
    const int rl = (int)(e - e0);
    if (timed) {
      const double u1 = u01((uint32_t)readlane_i((int)rw0.x, rl), (uint32_t)readlane_i((int)rw0.y, rl));
      const double tau = -log(u1) / Rtot * scale;  // exponential waiting time
      if (t + tau > A.dt) break;  // the next event falls outside the step
      t += tau;
    }
    const double u2 = u01((uint32_t)readlane_i((int)rw0.z, rl), (uint32_t)readlane_i((int)rw0.w, rl));
    const double u3 = u01((uint32_t)readlane_i((int)rw1.x, rl), (uint32_t)readlane_i((int)rw1.y, rl));
    const double u4 = u01((uint32_t)readlane_i((int)rw1.z, rl), (uint32_t)readlane_i((int)rw1.w, rl));

    // -- choose i by cumulative row sums (payloads: m_i, index)
    const Cand ci = team_pick<KMAX, double, double>(tm, incl, part, r, K, u2 * Rtot, m64, r, m64,
                                                    gix);
    if (ci.q < 0) {
      if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_RATE);
      break;
    }
    const int si = ci.q * TL + ci.lane;
    const int i_local = ci.lane * K + ci.q;
    const double mi = ci.p0, ri_old = ci.p1;
    const int gi = ci.gi;
    const double Mi = A.M[gi];  // needed after the outcome: the load overlaps row i
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
      if (tl == 0 && A.evlog != nullptr && e < A.log_per_cell) {
        int32_t *L = A.evlog + ((size_t)cell * A.log_per_cell + e) * 4;
        L[0] = i_local;
        L[1] = -1;
        L[2] = -1;
        L[3] = 0;
      }
      ++e;
      part = 0.0;
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < K) part += r[q];
      incl = tm.scan(part, Rtot);
      continue;
    }
    // -- choose j (payloads: m_j, relative velocity, index)
    const Cand cj = team_pick<KMAX, RT, RT>(tm, incl1, part1, rij, K, u3 * Ri, m64, m64, dvv, gix);
    const int j_local = cj.lane * K + cj.q;
    const double mj = cj.p0;
    const RT dvj = (RT)cj.p2;
    const int gj = cj.gi;

    // -- outcome (only i changes)
    double mnew;
    const bool fast = !(dvj < (RT)A.P.v_frag);
    const int oc = outcome(A.P, fast, mi, mj, u4, mnew);
    if (!(mnew > 0.0) || !isfinite(mnew)) {
      if (tl == 0) atomicOr(&A.state->flags, FLAG_BAD_MASS);
    }
    if (A.comp != nullptr && A.P.n_comp > 0 && (oc == OUT_STICK || oc == OUT_FRAG) &&
        tl < A.P.n_comp) {
      const double wi = mi, wj = group_factor(A.P.dm_max, mi, mj) * mj;
      float *cs = A.comp + (size_t)tl * A.N;
      const double cI = (double)cs[gi], cJ = (double)cs[gj];
      cs[gi] = (float)((wi * cI + wj * cJ) / (wi + wj));
    }
    const Rec<RT> rin = RecAfter<RT>::get(A.P, tm.S, mnew, Mi);
    if (tl == ci.lane) {
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q == ci.q) m64[q] = mnew;
    }
    if (tl == 0) {
      R.store(si, rin);
      if (A.evlog != nullptr && e < A.log_per_cell) {
        int32_t *L = A.evlog + ((size_t)cell * A.log_per_cell + e) * 4;
        L[0] = i_local;
        L[1] = j_local;
        L[2] = oc;
        L[3] = 0;
      }
    }

    // -- new row i: incremental update of the other rows, fresh row sum of i
    double part2 = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (q < K) {
        const int s = q * TL + tl;
        const Rec<RT> rq = s == si ? rin : R.load(s);
        RT dv, a_iq, a_qi;
        PairEval<RT, FAST>::run(pc, rin, rq, dv, a_iq, a_qi);
        part2 += (double)a_iq;
        const double x = (r[q] - (double)rji[q]) + (double)a_qi;
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
    const double delta = ri_new - ri_old;
    if (tl >= ci.lane) incl += delta;
    Rtot += delta;
    if (tl == ci.lane) {
      part += delta;
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q == ci.q) r[q] = ri_new;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) oc_count[k] += (oc == k) ? 1u : 0u;
    ++e;
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
  tm.sync();  // the region is reused by the next cell
}

// ---------------------------------------------------------------------------
// batched schedule: one persistent launch of four-wave workgroups; big cells
// on four-wave teams (largest first), then small cells on single waves
// (largest first), each wave popping its own work
// ---------------------------------------------------------------------------
template <typename RT, int KMAX, bool FAST>
__global__ __launch_bounds__(256, sizeof(RT) == 4 ? 3 : 2) void collide_batched(CollideArgs A) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_item;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t step = A.state->step;
  const size_t small_bytes = region_bytes<RT>(A.small_cap, 1);
  int nw = A.n_big > 0 ? 4 : 1;
  for (;;) {
    int cell = -1;
    if (nw == 4) {
      if (threadIdx.x == 0) s_item = atomicAdd(&A.state->big_head, 1);
      __syncthreads();
      const int item = s_item;
      __syncthreads();
      if (item < A.n_big)
        cell = A.big_list[item];
      else
        nw = 1;
    }
    if (nw == 1) {
      int item = 0;
      if (lane == 0) item = atomicAdd(&A.state->small_head, 1);
      item = readlane_i(item, 0);
      if (item >= A.n_small) break;
      cell = A.small_list[item];
    }
    char *base = nw == 4 ? smem : smem + (size_t)wave * small_bytes;
    process_cell<RT, KMAX, FAST>(A, cell, base, nw == 4 ? A.big_cap : A.small_cap, nw,
                                 nw == 4 ? wave : 0, lane, step);
  }
}

// plain schedule: one four-wave workgroup per cell, cells in index order
template <typename RT, int KMAX, bool FAST>
__global__ __launch_bounds__(256) void collide_plain(CollideArgs A) {
  extern __shared__ __align__(16) char smem[];
  process_cell<RT, KMAX, FAST>(A, blockIdx.x, smem, A.big_cap, 4, threadIdx.x >> 6, threadIdx.x & 63,
                         A.state->step);
}

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

template <typename RT, int KMAX, bool FAST>
static hipError_t run_batched(const CollideArgs &a, int grid_override, hipStream_t s) {
  const size_t lds = std::max(region_bytes<RT>(a.big_cap, 4), 4 * region_bytes<RT>(a.small_cap, 1));
  auto kern = collide_batched<RT, KMAX, FAST>;
  hipError_t e = prepare(kern, lds);
  int dev = 0, cus = 0, per_cu = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
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

template <typename RT, int KMAX, bool FAST>
static hipError_t run_plain(const CollideArgs &a, int n_cells, hipStream_t s) {
  const size_t lds = region_bytes<RT>(a.big_cap, 4);
  auto kern = collide_plain<RT, KMAX, FAST>;
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

hipError_t launch_collide(const CollideArgs &a, int precision, int schedule, int n_cells,
                          int max_cell, int grid_override, hipStream_t s) {
  const bool wide = max_cell > 1024;
  const bool fast = fast_path(a, precision);
  if (schedule == 0) {
    if (precision == 0)
      return wide ? run_plain<double, 8, false>(a, n_cells, s)
                  : run_plain<double, 4, false>(a, n_cells, s);
    if (fast)
      return wide ? run_plain<float, 8, true>(a, n_cells, s)
                  : run_plain<float, 4, true>(a, n_cells, s);
    return wide ? run_plain<float, 8, false>(a, n_cells, s)
                : run_plain<float, 4, false>(a, n_cells, s);
  }
  if (precision == 0)
    return wide ? run_batched<double, 8, false>(a, grid_override, s)
                : run_batched<double, 4, false>(a, grid_override, s);
  if (fast)
    return wide ? run_batched<float, 8, true>(a, grid_override, s)
                : run_batched<float, 4, true>(a, grid_override, s);
  return wide ? run_batched<float, 8, false>(a, grid_override, s)
              : run_batched<float, 4, false>(a, grid_override, s);
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
