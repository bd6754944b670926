// Complete clipping: lower bound of a.x + c over box ∩ {G x + h <= 0} by
// coordinate ascent over the Lagrange multipliers (Alg. 1, eq. 4).  Each
// step maximises the 1-D dual of Thm 3.1 for one constraint g.x + h <= 0
// with the other multipliers fixed:
//   D(beta) = min_box (a' + beta g).x + c' + beta h  (concave, piecewise linear)
// Its slope just right of beta is  m + sum_{q_j > beta} w_j,  where
// m = min_box(g.x + h), q_j = -a'_j / g_j are the breakpoints and
// w_j = |g_j| (hi_j - lo_j).  So beta* = 0 when the slope at 0+ is <= 0, else
// beta* is the breakpoint q* where the slope changes sign: the smallest
// positive breakpoint with  sum_{q_j > q*} w_j <= -m  (a weighted quantile).
// m > 0 means the constraint is empty over the box (+inf).  Slopes within a
// small tolerance of zero count as zero, so near-ties between maximisers go
// to the smallest one (see the tolerance at its use).
//
// GPU mapping: one team per problem -- a wave64 for n <= 1024, a 256-thread
// workgroup for n <= 4096 -- whose member t owns coordinates t, t + T, ...
// (EPL per member, T the team size) and keeps a' and the box in registers.  The weighted quantile is found without sorting by bisection
// over the float64 bit patterns of the breakpoints (positive doubles order
// like their bit patterns): each round picks the largest breakpoint at or
// below the midpoint and tests it with two wave-wide sums; a hit ends the
// search and otherwise the bit range halves, so at most 63 rounds are needed
// and about log2(#breakpoints) are typical.
//
// The returned bound D(beta) is valid for any beta >= 0 (weak duality); it is
// evaluated in float64, moved down by a rigorous bound on its rounding (and by
// the error bound of the objective plane itself) and rounded down to float32.
#include <type_traits>

#include "cv_common.h"
#include "cv_internal.h"
#include "cv_team.h"

namespace {

constexpr int CA_KMAX = CV_TEAM_KMAX;

// What the search keeps per candidate beside its breakpoint: workgroup teams
// (LDS to spare at three workgroups per CU) the float64 weight itself, wave
// teams |g_j| in float32 (their four teams' slices share one workgroup's
// LDS), from which each round forms the weight.
template <class Team>
using ca_wt = typename std::conditional<Team::PER_BLOCK == 1, double, float>::type;

// Weighted quantile: the smallest candidate q* with W(> q*) <= S, where
// W(> p) sums the weights of candidates above p.  The search keeps an open
// interval (lo, hi) of float64 bit patterns with W(> lo) > S >= W(>= hi) and
// probes a split point inside it: where the known weights put the crossing
// (interpolation, clamped to [1/16, 15/16] of the interval) on each of the
// first 16 rounds and on even rounds after them, the midpoint on the odd rounds
// after them.  Every round shrinks the interval to at most 15/16 and, past
// round 16, it at least halves every two rounds, so the 64-bit range closes
// within 16 + 2 * 65 rounds (typical searches end in 5-8 rounds; interpolating
// on every early round takes 15-20 % fewer than alternating from the start).
// A probe takes the largest candidate p at or below the split point; W(> p)
// decides the side and, only when W(> p) <= S, W(>= p) > S identifies p = q*.
// The breakpoints and the candidates' weights sit in the team's LDS slice
// (element e of member t at e*T + t; non-candidates hold -inf and 0), which
// keeps them out of the registers of the common path that needs no search:
// the float64 weight |g_j| (hi_j - lo_j) itself (workgroup teams), or |g_j|,
// from which each round forms that weight with the box in registers (wave
// teams).  Either way it is the value the caller summed, so every decision
// is taken on exact float64 weights.
// qmax, qmin: the largest and smallest candidate (team-wide), wpos the sum
// of the candidates' weights.
template <class Team, int EPL>
__device__ double ca_select(const Team& tm, const double* sq, const ca_wt<Team>* sg,
                            const float (&xl)[EPL], const float (&xh)[EPL], double S,
                            double wpos, double qmax, double qmin) {
  constexpr int T = Team::SIZE;
  unsigned long long blo = (unsigned long long)__double_as_longlong(qmin) - 1ull;
  unsigned long long bhi = (unsigned long long)__double_as_longlong(qmax) + 1ull;
  double wlo = wpos, whi = 0.0;  // W(> lo), W(>= hi)
#pragma unroll 1
  for (int it = 0; it < 160; ++it) {
    const unsigned long long span = bhi - blo;
    if (span <= 1ull) break;
    unsigned long long off = span / 2ull;
    if (it < 16 || (it & 1) == 0) {
      double f = (wlo - S) / (wlo - whi);
      f = fmin(fmax(f, 0.0625), 0.9375);
      off = (unsigned long long)((double)span * f);
    }
    off = off < 1ull ? 1ull : (off >= span ? span - 1ull : off);
    const double lo_v = __longlong_as_double((long long)blo);
    const double mv = __longlong_as_double((long long)(blo + off));
    double p = -INFINITY;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const double q = sq[e * T + tm.t];
      if (q > lo_v && q <= mv) p = fmax(p, q);
    }
    p = tm.max(p);
    if (p == -INFINITY) {  // no candidate in (lo, mv]: W(> mv) = W(> lo)
      blo += off;
      continue;
    }
    // W(> p) and W(>= p) in one reduction
    double wg = 0.0, wge = 0.0, zero = 0.0;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const double q = sq[e * T + tm.t];
      double w;
      if constexpr (Team::PER_BLOCK == 1) w = sg[e * T + tm.t];
      else w = (double)sg[e * T + tm.t] * ((double)xh[e] - (double)xl[e]);
      if (q > p) wg += w;
      if (q >= p) wge += w;
    }
    tm.sum3(wg, wge, zero);
    if (wg > S) {  // q* > p, and nothing lies in (p, mv]
      blo += off;
      wlo = wg;
      continue;
    }
    if (wge > S) return p;
    bhi = (unsigned long long)__double_as_longlong(p);
    whi = wge;
  }
  return __longlong_as_double((long long)bhi);
}

// One problem on one team.  a: objective coefficients (member-strided), c
// its intercept; on return a holds a + beta^T G.  Returns the rigorous
// float64 lower bound (before the final float32 rounding) or +inf when empty.
// The rounding-error scale sum_j (|a_j| + sum_k beta_k |g_kj|) max(|lo_j|,|hi_j|)
// is accumulated per constraint (beta_k times that constraint's own
// sum_j |g_kj| max(|lo_j|,|hi_j|)), so no per-coordinate scale is kept.
// xstar (optional) receives the minimising corner of the final dual; it may
// alias the objective row in memory, which is read for the kink test first.
// Member k fetches constraint k's row pointer, sign and offset up front, so a
// constraint costs one dependent load (its row) instead of a chain.
template <class Team, int EPL>
__device__ double ca_core(const Team& tm, int n, double (&a)[EPL], double c, double e_in,
                          const float* lo_b, const float* hi_b, const CvCons* cons, int b,
                          int passes, bool& empty, float* beta_out, double* xstar,
                          double* beta, double* sq, ca_wt<Team>* sw) {
  constexpr int T = Team::SIZE;
  const int t = tm.t;
  float xl[EPL], xh[EPL];
  double Ea = 0.0;
  const cv_buf blo = cv_buffer(lo_b, 4u * n), bhi = cv_buffer(hi_b, 4u * n);
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int j = t + T * e;
    xl[e] = buf_f32(blo, 4 * j);
    xh[e] = buf_f32(bhi, 4 * j);
    Ea += fabs(a[e]) * fabs_max(xl[e], xh[e]);
  }
  double cabs = fabs(c), Eb = 0.0;
  const int cnt = cons ? cons_count(*cons, b) : 0;
  const float* my_row = nullptr;
  float my_scale = 0.0f;
  double my_h = 0.0;
  if (t < cnt) cons_row(*cons, b, t, n, my_row, my_scale, my_h);
  tm.publish(my_row, my_scale, my_h, cnt);
  Ea = tm.sum(Ea);
  // beta: this team's slice of LDS (all members hold and write equal values)
  for (int k = 0; k < cnt; ++k) beta[k] = 0.0;
  empty = false;
#pragma unroll 1
  for (int pass = 0; pass < passes && !empty; ++pass) {
#pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const float* row;
      float scale;
      double h;
      tm.meta(my_row, my_scale, my_h, k, row, scale, h);
      if (!row) continue;
      // the shared statistics of this (subdomain, constraint), loaded first so
      // their latency overlaps the row's
      CvKStat st{};
      if (cons->kstats) st = cons->kstats[(size_t)b * cons->kmax + k];
      const cv_buf brow = cv_buffer(row, 4u * n);
      int vb = 4 * t;
      cv_opaque(vb);
      float g[EPL];  // constraint coefficients are float32 values
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        g[e] = scale * buf_f32(brow, vb + 4 * T * e);
        cv_opaque(xl[e]);
        cv_opaque(xh[e]);
      }
      const double bold = beta[k];
      if (bold != 0.0) {  // later passes: drop this constraint's own multiplier
#pragma unroll
        for (int e = 0; e < EPL; ++e) a[e] -= bold * (double)g[e];
      }
      // m, its error scales, and the weight of the coordinates whose
      // breakpoint q_j = -a_j/g_j is positive (a_j and g_j of opposite
      // signs), without dividing; breakpoints are formed only when that
      // weight exceeds -m, i.e. when beta* > 0 is possible.  Weights are
      // summed in float64 (products of float32 values are exact in float64,
      // so min(g lo, g hi) = g * (g >= 0 ? min(lo, hi) : max(lo, hi))
      // exactly; the opposite-sign test is branch-free, and a skipped weight
      // adds +0.0 to a non-negative sum, which leaves it unchanged).
      double m = 0.0, em = 0.0, tmax = 0.0;
      if (cons->kstats) {  // m, em and tmax of this (subdomain, constraint) computed once
        m = st.m;
        em = st.em;
        tmax = (double)st.tmax;
      } else {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const double gg = (double)g[e];
          const float xs = g[e] >= 0.0f ? fminf(xl[e], xh[e]) : fmaxf(xl[e], xh[e]);
          m += gg * (double)xs;
          const double te = fabs(gg) * (double)fmaxf(fabsf(xl[e]), fabsf(xh[e]));
          em += te;
          tmax = fmax(tmax, te);
        }
        tm.sum_sum_max(m, em, tmax);
      }
      // The weight of the coordinates whose breakpoint is positive, W(> 0).
      // Workgroup teams (rows over 1024 wide, where most constraints need a
      // search) screen it in float32: each weight |g_j| (hi_j - lo_j) is then
      // within 2^-23 of its value and a member's sum of up to 16 of them
      // within 15 * 2^-24 more, so the team sum `ws` is within 2^-19 ws of the
      // exact one, and only when that does not settle `ws > S` is the exact
      // float64 sum formed; the decision is the exact one either way.  Wave
      // teams sum in float64 directly (measured faster there: the screen
      // costs them registers).
      constexpr bool SCREEN = Team::PER_BLOCK == 1;
      double ws = 0.0;
      if constexpr (SCREEN) {
        float w32 = 0.0f;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const bool opp = (g[e] != 0.0f) & (a[e] != 0.0) & (signbit(a[e]) != signbit(g[e]));
          const float wf = fabsf(g[e]) * (xh[e] - xl[e]);
          w32 += opp ? wf : 0.0f;
        }
        ws = tm.sum((double)w32);
      } else {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const double wd = fabs((double)g[e]) * ((double)xh[e] - (double)xl[e]);
          const bool opp = (g[e] != 0.0f) & (a[e] != 0.0) & (signbit(a[e]) != signbit(g[e]));
          ws += opp ? wd : 0.0;
        }
        ws = tm.sum(ws);
      }
      m += h;
      if (bold != 0.0) {
        c -= bold * h;
        Eb += bold * em;
        cabs += bold * fabs(h);
      }
      if (m - cv_gamma(n + 1) * (em + fabs(h)) * CV_ERR_SLACK > 0.0) {
        empty = true;
        break;
      }
      // Slopes within `tol` of zero count as zero, so near-ties go to the
      // smaller multiplier.  Relaxed clipping by this constraint leaves the
      // dual exactly flat where only the clipped coordinate i's breakpoint is
      // ahead (its weight is -m), but the float32 end of that coordinate is
      // rounded outward, which leaves a slope of up to one float32 ulp of the
      // end times |g_i| <= 2^-23 tmax; the float64 sums add at most
      // gamma_{2n+8} (em + |h| + wsg).
      const double tol = 2.384185791015625e-07 * tmax + cv_gamma(2 * n + 8) * (em + fabs(h) + ws);
      const double S = -m + tol;
      bool search = ws > S + (SCREEN ? 0x1p-18 * ws : 0.0);
      if (SCREEN && !search && ws > S - 0x1p-18 * ws) {  // too close to call in float32
        double wsg = 0.0;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const double wd = fabs((double)g[e]) * ((double)xh[e] - (double)xl[e]);
          const bool opp = (g[e] != 0.0f) & (a[e] != 0.0) & (signbit(a[e]) != signbit(g[e]));
          wsg += opp ? wd : 0.0;
        }
        search = tm.sum(wsg) > S;
      }
      double bk = 0.0;
      if (search) {
        // breakpoints and the exact candidate set (a division may underflow
        // to q = 0, which is not a candidate), staged in LDS for the search
        // with |g_j|; the candidates' total weight and their range, reduced
        // together
        double wpos = 0.0, qmax = -INFINITY, nqmin = -INFINITY;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          double qe = -INFINITY;
          ca_wt<Team> ge = 0;
          if (g[e] != 0.0f) {
            const double q = -a[e] / (double)g[e];
            const double w = (double)fabsf(g[e]) * ((double)xh[e] - (double)xl[e]);
            if (q > 0.0 && w > 0.0) {
              qe = q;
              if constexpr (Team::PER_BLOCK == 1) ge = w;
              else ge = fabsf(g[e]);
              wpos += w;
              qmax = fmax(qmax, q);
              nqmin = fmax(nqmin, -q);
            }
          }
          sq[e * T + t] = qe;
          sw[e * T + t] = ge;
        }
        tm.max_max_sum(qmax, nqmin, wpos);
        if (wpos > S) bk = ca_select<Team, EPL>(tm, sq, sw, xl, xh, S, wpos, qmax, -nqmin);
      }
      beta[k] = bk;
      if (bk != 0.0) {
        // the row is re-read (cache hit) rather than kept live over the search
        int vb2 = 4 * t;
        cv_opaque(vb2);
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const float gr = scale * buf_f32(brow, vb2 + 4 * T * e);
          a[e] += bk * (double)gr;
        }
        c += bk * h;
        Eb += bk * em;
        cabs += bk * fabs(h);
      }
    }
  }
  if (empty) return INFINITY;
  double d = 0.0;
#pragma unroll
  for (int e = 0; e < EPL; ++e) d += fmin(a[e] * (double)xl[e], a[e] * (double)xh[e]);
  d = tm.sum(d) + c;
  const double err = (cv_gamma(n + 2 * passes * cnt + 8) * (Ea + Eb + cabs) + e_in) * CV_ERR_SLACK;
  if (beta_out && t < cons->kmax) {  // by slot: position o holds slot cons_slot(o)
    const int slot = cons_slot(*cons, b, t);
    if (slot >= 0) beta_out[slot] = t < cnt ? (float)beta[t] : 0.0f;
  }
  if (xstar) {
    // kink test: |a'_j| <= 2^-40 (|a_j| + sum_k beta_k |g_kj|); the scale
    // only sets a threshold far from both sides of the test, so float32
    // holds it (a kink leaves |a'_j| at rounding level, ~2^-50 of the scale)
    float sc[EPL];
    const cv_buf bx = cv_buffer(xstar, 8u * n);
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int j = t + T * e;
      sc[e] = (float)fabs(buf_f64(bx, 8 * j));
    }
    for (int k = 0; k < cnt; ++k) {
      if (beta[k] == 0.0) continue;
      const float* row;
      float scale;
      double h;
      tm.meta(my_row, my_scale, my_h, k, row, scale, h);
      if (!row) continue;
      const cv_buf brow = cv_buffer(row, 4u * n);
      int vb = 4 * t;
      cv_opaque(vb);
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        sc[e] += (float)beta[k] * fabsf(buf_f32(brow, vb + 4 * T * e));
      }
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int j = t + T * e;
      if (j < n) {
        const bool kink = fabs(a[e]) <= 9.094947017729282e-13 * (double)sc[e];  // 2^-40
        xstar[j] = kink ? 0.5 * ((double)xl[e] + (double)xh[e])
                        : (a[e] > 0.0 ? (double)xl[e] : (double)xh[e]);
      }
    }
  }
  return d - err;
}

// Per (subdomain, constraint position): m = min over the box of g.x (h not
// included), em = sum_j |g_j| max(|lo_j|,|hi_j|) and the largest of those
// terms, with the same team shape and summation order as ca_core computes
// them (so both give the same values); complete clipping of every objective
// row of the subdomain reads them instead of recomputing them.
template <class Team, int EPL>
__global__ __launch_bounds__(256) void k_cons_stats(int B, int n, CvCons cons,
                                                    const float* __restrict__ lo,
                                                    const float* __restrict__ hi,
                                                    CvKStat* stats) {
  __shared__ double red[24];
  __shared__ const float* mrow[CV_TEAM_KMAX];
  __shared__ float mscale[CV_TEAM_KMAX];
  __shared__ double mh[CV_TEAM_KMAX];
  const Team tm = make_team<Team>(red, mrow, mscale, mh);
  constexpr int T = Team::SIZE;
  const int b = xcd_block(blockIdx.x, gridDim.x) * Team::PER_BLOCK + Team::index_in_block();
  if (b >= B) return;
  float xl[EPL], xh[EPL];
  const cv_buf blo = cv_buffer(lo + (size_t)b * n, 4u * n), bhi = cv_buffer(hi + (size_t)b * n, 4u * n);
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int j = tm.t + T * e;
    xl[e] = buf_f32(blo, 4 * j);
    xh[e] = buf_f32(bhi, 4 * j);
  }
  const int cnt = cons_count(cons, b);
  const float* my_row = nullptr;
  float my_scale = 0.0f;
  double my_h = 0.0;
  if (tm.t < cnt) cons_row(cons, b, tm.t, n, my_row, my_scale, my_h);
  tm.publish(my_row, my_scale, my_h, cnt);
#pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const float* row;
    float scale;
    double h;
    tm.meta(my_row, my_scale, my_h, k, row, scale, h);
    if (!row) continue;
    const cv_buf brow = cv_buffer(row, 4u * n);
    int vb = 4 * tm.t;
    cv_opaque(vb);
    double m = 0.0, em = 0.0, tmax = 0.0;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const float g = scale * buf_f32(brow, vb + 4 * T * e);
      const double gg = (double)g;
      const float xs = g >= 0.0f ? fminf(xl[e], xh[e]) : fmaxf(xl[e], xh[e]);
      m += gg * (double)xs;
      const double te = fabs(gg) * (double)fmaxf(fabsf(xl[e]), fabsf(xh[e]));
      em += te;
      tmax = fmax(tmax, te);
    }
    tm.sum_sum_max(m, em, tmax);
    if (tm.t == 0) stats[(size_t)b * cons.kmax + k] = CvKStat{m, em, ru32(tmax), 0.0f};
  }
}

// LDS of a workgroup: beta, the search slices and the team scratch, with
// the team of member threadIdx.x.
template <class Team, int EPL>
struct CaShared {
  double beta[Team::PER_BLOCK * CA_KMAX];
  double q[Team::PER_BLOCK * Team::SIZE * EPL];
  ca_wt<Team> w[Team::PER_BLOCK * Team::SIZE * EPL];
  double red[24];
  const float* mrow[CA_KMAX];
  float mscale[CA_KMAX];
  double mh[CA_KMAX];
};
template <class Team, int EPL>
__device__ __forceinline__ Team team_of(CaShared<Team, EPL>& sh) {
  if constexpr (Team::PER_BLOCK == 1)
    return Team{(int)threadIdx.x, sh.red, sh.mrow, sh.mscale, sh.mh};
  else
    return Team{(int)(threadIdx.x & 63)};
}
template <class Team, int EPL>
__device__ __forceinline__ double* beta_slice(CaShared<Team, EPL>& sh) {
  return sh.beta + Team::index_in_block() * CA_KMAX;
}
template <class Team, int EPL>
__device__ __forceinline__ double* q_slice(CaShared<Team, EPL>& sh) {
  return sh.q + Team::index_in_block() * Team::SIZE * EPL;
}
template <class Team, int EPL>
__device__ __forceinline__ ca_wt<Team>* w_slice(CaShared<Team, EPL>& sh) {
  return sh.w + Team::index_in_block() * Team::SIZE * EPL;
}

// Workgroups per CU that k_ca_rows asks the register allocator for: three.
// At four, a 13-coordinate wave team spills its objective row inside the
// constraint loop, and a 12-coordinate workgroup team spills about 40
// registers to memory (measured on 3072-wide rows: 4.19 ms at four, 3.69 ms
// at three).
template <class Team, int EPL>
constexpr int ca_rows_blocks() {
  return 3;
}

// Final planes: rows r = (b, m) of the backward pass output.
template <class Team, int EPL>
__global__ __launch_bounds__(256, (ca_rows_blocks<Team, EPL>())) void k_ca_rows(int R, int M, int n, CvCons cons, int passes,
                                                 double* Ax, const double* __restrict__ rowc,
                                                 const double* __restrict__ rowerr,
                                                 const float* __restrict__ lo,
                                                 const float* __restrict__ hi, uint8_t* infeasible,
                                                 float* lb, float* beta_out, int write_xstar,
                                                 float* best, int best_init) {
  __shared__ CaShared<Team, EPL> sh;
  const Team tm = team_of(sh);
  constexpr int T = Team::SIZE;
  // the M rows of a subdomain share its box and constraint rows: keep
  // neighbouring rows on one XCD
  const int r = xcd_block(blockIdx.x, gridDim.x) * Team::PER_BLOCK + Team::index_in_block();
  if (r >= R) return;
  const int b = r / M;
  double* arow = Ax + (size_t)r * n;
  const cv_buf ba = cv_buffer(arow, 8u * n);
  if (infeasible && infeasible[b]) {
    if (tm.t == 0) {
      lb[r] = INFINITY;
      if (best) best[r] = INFINITY;
    }
    return;
  }
  double a[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int j = tm.t + T * e;
    a[e] = buf_f64(ba, 8 * j);
  }
  bool empty;
  const double L = ca_core<Team, EPL>(tm, n, a, rowc[r], rowerr[r], lo + (size_t)b * n,
                                      hi + (size_t)b * n, &cons, b, passes, empty,
                                      beta_out ? beta_out + (size_t)r * cons.kmax : nullptr,
                                      write_xstar ? arow : nullptr, beta_slice(sh), q_slice(sh),
                                      w_slice(sh));
  if (tm.t == 0) {
    float v = INFINITY;
    if (empty) {
      if (infeasible) infeasible[b] = 1;
    } else {
      v = fmaxf(lb[r], rd32(L));
    }
    lb[r] = v;
    if (best) best[r] = best_init ? v : fmaxf(best[r], v);
  }
}

template <class Team, int EPL>
__global__ __launch_bounds__(256, 2) void k_ca_generic(int B, int P, int n, const float* __restrict__ A,
                                                    int A_shared, const float* __restrict__ cv,
                                                    const float* __restrict__ lo,
                                                    const float* __restrict__ hi, CvCons cons,
                                                    int has_cons, int passes, float* lb, float* ub,
                                                    float* beta_out, uint8_t* infeasible) {
  __shared__ CaShared<Team, EPL> sh;
  const Team tm = team_of(sh);
  constexpr int T = Team::SIZE;
  const long long pid = (long long)blockIdx.x * Team::PER_BLOCK + Team::index_in_block();
  if (pid >= (long long)B * P) return;
  const int b = (int)(pid / P), p = (int)(pid % P);
  const size_t arow = A_shared ? (size_t)p : (size_t)pid;
  const float* ap = A + arow * n;
  const double c = (double)cv[arow];
  const float* lb_ = lo + (size_t)b * n;
  const float* hb_ = hi + (size_t)b * n;
  double a[EPL];
  double dmin = 0.0, dmax = 0.0, ea = 0.0;
  const cv_buf bap = cv_buffer(ap, 4u * n), blb = cv_buffer(lb_, 4u * n), bhb = cv_buffer(hb_, 4u * n);
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int j = tm.t + T * e;
    a[e] = (double)buf_f32(bap, 4 * j);
    const double x0 = (double)buf_f32(blb, 4 * j), x1 = (double)buf_f32(bhb, 4 * j);
    dmin += fmin(a[e] * x0, a[e] * x1);
    dmax += fmax(a[e] * x0, a[e] * x1);
    ea += fabs(a[e]) * fmax(fabs(x0), fabs(x1));
  }
  tm.sum3(dmin, dmax, ea);
  const double e0 = cv_gamma(n + 1) * (ea + fabs(c)) * CV_ERR_SLACK;
  float out = rd32(dmin + c - e0);
  bool empty = false;
  if (has_cons) {
    const double L = ca_core<Team, EPL>(tm, n, a, c, 0.0, lb_, hb_, &cons, b, passes, empty,
                                        beta_out ? beta_out + (size_t)pid * cons.kmax : nullptr,
                                        nullptr, beta_slice(sh), q_slice(sh), w_slice(sh));
    if (!empty) out = fmaxf(out, rd32(L));
  }
  if (tm.t == 0) {
    lb[pid] = empty ? INFINITY : out;
    if (ub) ub[pid] = ru32(dmax + c + e0);
    if (empty && infeasible) infeasible[b] = 1;
  }
}

// Intermediate neurons: lower plane (side 0) and negated upper plane (side 1) of every
// root-unstable neuron still unstable in subdomain b.
template <class Team, int EPL>
__global__ __launch_bounds__(256, 2) void k_ca_neurons(int B, int Umax, int n, CvProps props,
                                                    CvCons cons, int passes,
                                                    const float* __restrict__ lo,
                                                    const float* __restrict__ hi,
                                                    const float* __restrict__ l,
                                                    const float* __restrict__ u, int Nh,
                                                    const uint8_t* __restrict__ infeasible,
                                                    const uint8_t* __restrict__ select,
                                                    float* Ltmp) {
  __shared__ CaShared<Team, EPL> sh;
  const Team tm = team_of(sh);
  constexpr int T = Team::SIZE;
  const long long id =
      (long long)xcd_block(blockIdx.x, gridDim.x) * Team::PER_BLOCK + Team::index_in_block();
  if (id >= (long long)B * Umax * 2) return;
  const int side = (int)(id & 1);
  const long long bc = id >> 1;
  const int b = (int)(bc / Umax), q = (int)(bc % Umax);
  const RootDev& rd = prop_of(props, b);
  if (q >= rd.U) {  // past this property's unstable neurons
    if (tm.t == 0) Ltmp[id] = -INFINITY;
    return;
  }
  const int j = rd.uidx[q];
  const float lj = l[(size_t)b * Nh + j], uj = u[(size_t)b * Nh + j];
  if ((infeasible && infeasible[b]) || !(lj < 0.0f && uj > 0.0f) ||
      (select && !select[(size_t)b * Nh + j])) {
    if (tm.t == 0) Ltmp[id] = -INFINITY;
    return;
  }
  const float* ap = uniform_ptr((side ? rd.A_hi : rd.A_lo) + (size_t)(rd.prow ? q : j) * n);
  const double c = side ? -rd.c_hi[j] : rd.c_lo[j];
  double a[EPL];
  const cv_buf bap = cv_buffer(ap, 4u * n);
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int jj = tm.t + T * e;
    const double v = (double)buf_f32(bap, 4 * jj);
    a[e] = side ? -v : v;
  }
  bool empty;
  const double L = ca_core<Team, EPL>(tm, n, a, c, 0.0, lo + (size_t)b * n, hi + (size_t)b * n,
                                      &cons, b, passes, empty, nullptr, nullptr, beta_slice(sh),
                                      q_slice(sh), w_slice(sh));
  if (tm.t == 0) Ltmp[id] = empty ? INFINITY : rd32(L);
}

}  // namespace

hipError_t launch_cons_stats(int B, int n, const CvCons& cons, const float* lo, const float* hi,
                             CvKStat* stats, hipStream_t s) {
  if (B <= 0 || cons.kmax <= 0) return hipSuccess;
  if (cons.kmax > CA_KMAX) return hipErrorInvalidValue;
  CV_DISPATCH_TEAM(n, hipLaunchKernelGGL((k_cons_stats<TM, E>), dim3(team_blocks(B, TM::PER_BLOCK)),
                                       dim3(256), 0, s, B, n, cons, lo, hi, stats));
  return hipGetLastError();
}

hipError_t launch_ca_rows(int R, int M, int n, const CvCons& cons, int passes, double* Ax,
                          const double* rowc, const double* rowerr, const float* lo,
                          const float* hi, uint8_t* infeasible, float* lb, float* beta_out,
                          int write_xstar, float* best, int best_init, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  if (cons.kmax > CA_KMAX) return hipErrorInvalidValue;
  CV_DISPATCH_TEAM(n, hipLaunchKernelGGL((k_ca_rows<TM, E>), dim3(team_blocks(R, TM::PER_BLOCK)),
                                       dim3(256), 0, s, R, M, n, cons, passes, Ax, rowc, rowerr,
                                       lo, hi, infeasible, lb, beta_out, write_xstar, best,
                                       best_init));
  return hipGetLastError();
}

hipError_t launch_ca_generic(int B, int P, int n, const float* A, int A_shared, const float* c,
                             const float* lo, const float* hi, const CvCons* cons, int passes,
                             float* lb, float* ub, float* beta_out, uint8_t* infeasible,
                             hipStream_t s) {
  const long long tot = (long long)B * P;
  if (tot <= 0) return hipSuccess;
  CvCons cc{};
  if (cons) {
    cc = *cons;
    if (cc.kmax > CA_KMAX) return hipErrorInvalidValue;
  }
  CV_DISPATCH_TEAM(n, hipLaunchKernelGGL((k_ca_generic<TM, E>), dim3(team_blocks(tot, TM::PER_BLOCK)),
                                       dim3(256), 0, s, B, P, n, A, A_shared, c, lo, hi, cc,
                                       cons ? 1 : 0, passes, lb, ub, beta_out, infeasible));
  return hipGetLastError();
}

hipError_t launch_ca_neurons(int B, int Umax, int n, CvProps props,
                             const CvCons& cons, int passes, const float* lo, const float* hi,
                             const float* l, const float* u, int Nh, const uint8_t* infeasible,
                             const uint8_t* select, float* Ltmp, hipStream_t s) {
  const long long tot = (long long)B * Umax * 2;
  if (tot <= 0) return hipSuccess;
  if (cons.kmax > CA_KMAX) return hipErrorInvalidValue;
  CV_DISPATCH_TEAM(n, hipLaunchKernelGGL((k_ca_neurons<TM, E>), dim3(team_blocks(tot, TM::PER_BLOCK)),
                                       dim3(256), 0, s, B, Umax, n, props, cons, passes, lo, hi,
                                       l, u, Nh, infeasible, select, Ltmp));
  return hipGetLastError();
}
