// Relaxed clipping of subdomain boxes by linear constraints G x + h <= 0
// (Thm 3.2; parallel form Alg. 2, sequential form Alg. 3).
//
// One 256-thread workgroup per subdomain; thread t owns coordinates
// t, t + 256, ... of the box (kept in registers), so the per-constraint
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

namespace {

constexpr int CT = 256;
constexpr int EPT = 16;  // coordinates per thread: n <= 4096

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sh[w * 2] = a;
    sh[w * 2 + 1] = b;
  }
  __syncthreads();
  a = sh[0] + sh[2] + sh[4] + sh[6];
  b = sh[1] + sh[3] + sh[5] + sh[7];
}

__global__ __launch_bounds__(CT) void k_clip(int B, int n, CvCons cons, float* lo, float* hi,
                                             uint8_t* infeasible, int mode) {
  __shared__ double sh[8];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  float olo[EPT], ohi[EPT], nlo[EPT], nhi[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + q * CT;
    olo[q] = ld_or0(lo + (size_t)b * n, i, n);
    ohi[q] = ld_or0(hi + (size_t)b * n, i, n);
    nlo[q] = olo[q];
    nhi[q] = ohi[q];
  }
  const int cnt = cons_count(cons, b);
  bool empty = false;
  for (int k = 0; k < cnt; ++k) {
    const float* row;
    float scale;
    double h;
    cons_row(cons, b, k, n, row, scale, h);
    if (!row) continue;
    float g[EPT];
    double m = 0.0, e = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int i = tid + q * CT;
      g[q] = scale * ld_or0(row, i, n);
      const double x0 = mode ? (double)nlo[q] : (double)olo[q];
      const double x1 = mode ? (double)nhi[q] : (double)ohi[q];
      const double gg = (double)g[q];
      m += fmin(gg * x0, gg * x1);
      e += fabs(gg) * fmax(fabs(x0), fabs(x1));
    }
    block_sum2(m, e, sh);
    m += h;
    const double mlo = m - cv_gamma(n + 1) * (e + fabs(h)) * CV_ERR_SLACK;
    if (mlo > 0.0) {
      empty = true;
      break;
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const double gg = (double)g[q];
      if (gg > 0.0) {
        const double base = mode ? (double)nlo[q] : (double)olo[q];
        const double d = mlo / gg;
        const double v = base - d + (fabs(base) + fabs(d)) * (4.0 * CV_U64);
        nhi[q] = fminf(nhi[q], ru32(v));
      } else if (gg < 0.0) {
        const double base = mode ? (double)nhi[q] : (double)ohi[q];
        const double d = mlo / gg;
        const double v = base - d - (fabs(base) + fabs(d)) * (4.0 * CV_U64);
        nlo[q] = fmaxf(nlo[q], rd32(v));
      }
    }
  }
  int bad = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + q * CT;
    if (i < n) {
      lo[(size_t)b * n + i] = nlo[q];
      hi[(size_t)b * n + i] = nhi[q];
      bad |= (nlo[q] > nhi[q]) ? 1 : 0;
    }
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) infeasible[b] = (empty || bad) ? 1 : 0;
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
  if (n > CT * EPT) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_clip, dim3(B), dim3(CT), 0, s, B, n, cons, lo, hi, infeasible, mode);
  return hipGetLastError();
}
