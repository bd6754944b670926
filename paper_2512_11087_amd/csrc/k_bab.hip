// Branching steps of the two branch-and-bound loops around the hot path.
//
// ReLU (activation) branching, Alg. 5: every parent subdomain is split on
// one unstable neuron (l < 0 < u) not split yet -- the one with the largest
// BaBSR intercept score  max(0,-l) max(0,u) / (u - l) * weight  (float64,
// ties to the lower index) -- into child 2b (branch z <= 0, sign -1) and
// child 2b + 1 (branch z >= 0, sign +1), which carry the parent's splits
// plus the new one and the parent's box.  A parent without such a neuron
// gets chosen = -1 and children identical to itself.
//
// Input branching, Alg. 4: every parent box is halved along the dimension
// with the largest (hi_d - lo_d) * sum_m |A_md| (A: the parent's final
// planes, ties to the lower index) at the float32 midpoint, so the halves
// share their cut; both children keep the parent's planes as constraints.
//
// One wave per parent; the argmax is a wave reduction of (score, -index).
#include "cv_common.h"
#include "cv_internal.h"

namespace {

// Larger score wins; equal scores: smaller index.
__device__ __forceinline__ void argmax_step(double& s, int& i, double s2, int i2) {
  if (s2 > s || (s2 == s && i2 < i)) {
    s = s2;
    i = i2;
  }
}
__device__ __forceinline__ void wave_argmax(double& s, int& i) {
  for (int d = 1; d < 64; d <<= 1) {
    const double s2 = __shfl_xor(s, d);
    const int i2 = __shfl_xor(i, d);
    argmax_step(s, i, s2, i2);
  }
}

__global__ __launch_bounds__(256) void k_branch_relu(int B, int Nh, const float* __restrict__ l,
                                                     const float* __restrict__ u,
                                                     const float* __restrict__ wall, CvProps props,
                                                     int kin,
                                                     const int32_t* __restrict__ neuron,
                                                     const int8_t* __restrict__ sign,
                                                     const int32_t* __restrict__ count, int n0,
                                                     const float* __restrict__ lo,
                                                     const float* __restrict__ hi, int kout,
                                                     int32_t* chosen, int32_t* neuron2,
                                                     int8_t* sign2, int32_t* count2, float* lo2,
                                                     float* hi2) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (b >= B) return;
  const float* __restrict__ weight = wall + (size_t)prop_index(props, b) * Nh;  // [P, Nh]
  int cnt = count ? count[b] : kin;
  cnt = cnt < 0 ? 0 : (cnt > kin ? kin : cnt);
  const float* lb = l + (size_t)b * Nh;
  const float* ub = u + (size_t)b * Nh;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int j = lane; j < Nh; j += 64) {
    const double lj = (double)lb[j], uj = (double)ub[j];
    if (!(lj < 0.0 && uj > 0.0)) continue;
    bool split = false;
    for (int k = 0; k < cnt; ++k) split |= neuron[(size_t)b * kin + k] == j;
    if (split) continue;
    const double sc = (-lj) * uj / (uj - lj) * (double)weight[j];
    argmax_step(best, bi, sc, j);
  }
  wave_argmax(best, bi);
  const int ch = (best >= 0.0 && cnt < kout) ? bi : -1;  // -1: nothing to split or no free slot
  if (lane == 0) chosen[b] = ch;
  for (int side = 0; side < 2; ++side) {
    const size_t r = (size_t)2 * b + side;
    for (int k = lane; k < kout; k += 64) {
      int32_t nv = 0;
      int8_t sv = 0;
      if (k < cnt) {
        nv = neuron[(size_t)b * kin + k];
        sv = sign[(size_t)b * kin + k];
      } else if (k == cnt && ch >= 0) {
        nv = ch;
        sv = side ? 1 : -1;
      }
      neuron2[r * kout + k] = nv;
      sign2[r * kout + k] = sv;
    }
    if (lane == 0) count2[r] = cnt + (ch >= 0 ? 1 : 0);
    for (int j = lane; j < n0; j += 64) {
      lo2[r * n0 + j] = lo[(size_t)b * n0 + j];
      hi2[r * n0 + j] = hi[(size_t)b * n0 + j];
    }
  }
}

__global__ __launch_bounds__(256) void k_branch_input(int B, int M, int n0,
                                                      const float* __restrict__ lo,
                                                      const float* __restrict__ hi,
                                                      const float* __restrict__ A, int32_t* dim,
                                                      float* lo2, float* hi2) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (b >= B) return;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int j = lane; j < n0; j += 64) {
    double w = 0.0;
    for (int m = 0; m < M; ++m) w += fabs((double)A[((size_t)b * M + m) * n0 + j]);
    const double sc = ((double)hi[(size_t)b * n0 + j] - (double)lo[(size_t)b * n0 + j]) * w;
    argmax_step(best, bi, sc, j);
  }
  wave_argmax(best, bi);
  const int d = bi;
  if (lane == 0) dim[b] = d;
  const float mid = 0.5f * (lo[(size_t)b * n0 + d] + hi[(size_t)b * n0 + d]);
  for (int side = 0; side < 2; ++side) {
    const size_t r = (size_t)2 * b + side;
    for (int j = lane; j < n0; j += 64) {
      float a = lo[(size_t)b * n0 + j], c = hi[(size_t)b * n0 + j];
      if (j == d) {
        if (side == 0) c = mid;
        else a = mid;
      }
      lo2[r * n0 + j] = a;
      hi2[r * n0 + j] = c;
    }
  }
}

}  // namespace

hipError_t launch_branch_relu(int B, int Nh, const float* l, const float* u, const float* weight,
                              CvProps props, int kin, const int32_t* neuron, const int8_t* sign,
                              const int32_t* count, int n0, const float* lo, const float* hi,
                              int kout, int32_t* chosen, int32_t* neuron2, int8_t* sign2,
                              int32_t* count2, float* lo2, float* hi2, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_branch_relu, dim3((B + 3) / 4), dim3(256), 0, s, B, Nh, l, u, weight, props, kin,
                     neuron, sign, count, n0, lo, hi, kout, chosen, neuron2, sign2, count2, lo2,
                     hi2);
  return hipGetLastError();
}

hipError_t launch_branch_input(int B, int M, int n0, const float* lo, const float* hi,
                               const float* A, int32_t* dim, float* lo2, float* hi2,
                               hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_branch_input, dim3((B + 3) / 4), dim3(256), 0, s, B, M, n0, lo, hi, A, dim,
                     lo2, hi2);
  return hipGetLastError();
}
