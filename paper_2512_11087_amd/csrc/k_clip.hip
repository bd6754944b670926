// Relaxed clipping of subdomain boxes by linear constraints G x + h <= 0
// (Thm 3.2; parallel form Alg. 2, sequential form Alg. 3).
//
// One team per subdomain -- a wave64 for n <= 1024 (four subdomains per
// workgroup), a 256-thread workgroup up to 4096; member t owns coordinates
// t, t + T, ... of the box (kept in registers), so the per-constraint
// reduction m = min over the box of g.x + h is the only cross-thread step.
// Constraint rows are read either from the cached root planes (split form,
// eqs. 9-10) or from a dense G.
//
// Soundness in floating point: m is evaluated in float64 with products of
// float32 values (exact) and a rigorous bound e on the rounding of the sum;
// m_lo = m - e is a certain lower bound of the exact m.  The box is empty
// only if m_lo > 0.  The new bounds lo_i - m_lo/g_i (g_i > 0, an upper bound)
// and hi_i - m_lo/g_i (g_i < 0, a lower bound) are loosened by a margin that
// covers their own float64 rounding and rounded outward to float32, so the
// float32 box always contains the exact clipped box.
#include "cv_common.h"
#include "cv_internal.h"
#include "cv_team.h"

namespace {

// One team per subdomain (a wave for n <= 1024, a workgroup up to 4096);
// member t owns coordinates t, t + T, ... of the box in registers, loaded
// with range-checked buffer loads (no branch per element).
template <class Team, int EPL>
__global__ __launch_bounds__(256) void k_clip(int B, int n, CvCons cons, float* lo, float* hi,
                                              uint8_t* infeasible, int mode) {
  __shared__ double red[24];
  __shared__ const float* mrow[CV_TEAM_KMAX];
  __shared__ float mscale[CV_TEAM_KMAX];
  __shared__ double mh[CV_TEAM_KMAX];
  const Team tm = make_team<Team>(red, mrow, mscale, mh);
  constexpr int T = Team::SIZE;
  const int t = tm.t;
  const int b = blockIdx.x * Team::PER_BLOCK + Team::index_in_block();
  if (b >= B) return;
  float* lob = lo + (size_t)b * n;
  float* hib = hi + (size_t)b * n;
  const cv_buf blo = cv_buffer(lob, 4u * n), bhi = cv_buffer(hib, 4u * n);
  float olo[EPL], ohi[EPL], nlo[EPL], nhi[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int j = t + T * e;
    olo[e] = buf_f32(blo, 4 * j);
    ohi[e] = buf_f32(bhi, 4 * j);
    nlo[e] = olo[e];
    nhi[e] = ohi[e];
  }
  const int cnt = cons_count(cons, b);
  // member k fetches constraint k's row pointer, sign and offset up front
  // (up to CV_TEAM_KMAX constraints; beyond, each is fetched in the loop)
  const float* my_row = nullptr;
  float my_scale = 0.0f;
  double my_h = 0.0;
  if (t < cnt && t < CV_TEAM_KMAX) cons_row(cons, b, t, n, my_row, my_scale, my_h);
  tm.publish(my_row, my_scale, my_h, cnt < CV_TEAM_KMAX ? cnt : CV_TEAM_KMAX);
  bool empty = false;
#pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const float* row;
    float scale;
    double h;
    if (k < CV_TEAM_KMAX)
      tm.meta(my_row, my_scale, my_h, k, row, scale, h);
    else
      cons_row(cons, b, k, n, row, scale, h);
    row = uniform_ptr(row);  // the same constraint for the whole team
    if (!row) continue;
    const cv_buf brow = cv_buffer(row, 4u * n);
    float g[EPL];
    double m = 0.0, err = 0.0, zero = 0.0;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      g[e] = scale * buf_f32(brow, 4 * (t + T * e));
      const double x0 = mode ? (double)nlo[e] : (double)olo[e];
      const double x1 = mode ? (double)nhi[e] : (double)ohi[e];
      const double gg = (double)g[e];
      m += fmin(gg * x0, gg * x1);
      err += fabs(gg) * fmax(fabs(x0), fabs(x1));
    }
    tm.sum3(m, err, zero);
    m += h;
    const double mlo = m - cv_gamma(n + 1) * (err + fabs(h)) * CV_ERR_SLACK;
    if (mlo > 0.0) {
      empty = true;
      break;
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const double gg = (double)g[e];
      if (gg > 0.0) {
        const double base = mode ? (double)nlo[e] : (double)olo[e];
        const double d = mlo / gg;
        const double v = base - d + (fabs(base) + fabs(d)) * (4.0 * CV_U64);
        nhi[e] = fminf(nhi[e], ru32(v));
      } else if (gg < 0.0) {
        const double base = mode ? (double)nhi[e] : (double)ohi[e];
        const double d = mlo / gg;
        const double v = base - d - (fabs(base) + fabs(d)) * (4.0 * CV_U64);
        nlo[e] = fmaxf(nlo[e], rd32(v));
      }
    }
  }
  double bad = 0.0;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int j = t + T * e;
    if (j < n) {
      lob[j] = nlo[e];
      hib[j] = nhi[e];
      if (nlo[e] > nhi[e]) bad = 1.0;
    }
  }
  bad = tm.max(bad);
  if (t == 0) infeasible[b] = (empty || bad > 0.0) ? 1 : 0;
}

// Constraint importance order (heuristics appendix): position -> slot for
// each subdomain, the used slots sorted by the distance |g.xc + h| / ||g||_2
// of their hyperplane from the centre xc of the box, closest first; ties keep
// the list order, slots without a hyperplane (g = 0, ignored) go last, unused
// slots keep their place.  One wave per subdomain, lane k ranks slot k
// (kmax <= 64); the sums are float64 (products of float32 values are exact).
__global__ __launch_bounds__(256) void k_cons_order(int B, int n, CvCons cons,
                                                    const float* __restrict__ lo,
                                                    const float* __restrict__ hi, int32_t* order) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (b >= B) return;
  const int kmax = cons.kmax;
  const int cnt = cons_count(cons, b);
  const float* lb = lo + (size_t)b * n;
  const float* hb = hi + (size_t)b * n;
  double mine = INFINITY;
  for (int k = 0; k < cnt; ++k) {
    const float* row;
    float scale;
    double h;
    cons_row_slot(cons, b, k, n, row, scale, h);
    double sv = 0.0, nn = 0.0;
    if (row) {
      for (int j = lane; j < n; j += 64) {
        const double g = (double)(scale * row[j]);
        sv += g * (0.5 * ((double)lb[j] + (double)hb[j]));
        nn += g * g;
      }
    }
    sv = wave_sum(sv);
    nn = wave_sum(nn);
    double d = (row && nn > 0.0) ? fabs(sv + h) / sqrt(nn) : INFINITY;
    if (!(d == d)) d = INFINITY;
    if (lane == k) mine = d;
  }
  int r = 0;
  for (int j = 0; j < cnt; ++j) {
    const double dj = lane_f64(mine, j);
    r += (dj < mine || (dj == mine && j < lane)) ? 1 : 0;
  }
  if (lane < cnt)
    order[(size_t)b * kmax + r] = lane;
  else if (lane < kmax)
    order[(size_t)b * kmax + lane] = lane;
}

}  // namespace

hipError_t launch_cons_order(int B, int n, const CvCons& cons, const float* lo, const float* hi,
                             int32_t* order, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (cons.kmax > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cons_order, dim3((B + 3) / 4), dim3(256), 0, s, B, n, cons, lo, hi, order);
  return hipGetLastError();
}

hipError_t launch_clip(int B, int n, const CvCons& cons, float* lo, float* hi, uint8_t* infeasible,
                       int mode, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  CV_DISPATCH_TEAM(n, hipLaunchKernelGGL((k_clip<TM, E>), dim3(team_blocks(B, TM::PER_BLOCK)),
                                         dim3(256), 0, s, B, n, cons, lo, hi, infeasible, mode));
  return hipGetLastError();
}
