// Device helpers shared by the clip-and-verify kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#define CV_WAVE 64

// ------------------------------------------------------------ rounding
// Largest float32 <= d (rd32) and smallest float32 >= d (ru32).  The
// conversion rounds to nearest; one step toward the required side fixes
// the cases where nearest went the wrong way.  NaN passes through.
__device__ __forceinline__ float rd32(double d) {
  float f = (float)d;
  if ((double)f > d) f = nextafterf(f, -INFINITY);
  return f;
}
__device__ __forceinline__ float ru32(double d) {
  float f = (float)d;
  if ((double)f < d) f = nextafterf(f, INFINITY);
  return f;
}

// Unit roundoff of float64 and a generous bound gamma(K) on the relative
// error of a K-term float64 dot product evaluated in any order (each of the
// K products and K-1 additions rounds once; the factor 2 also covers an
// accumulation that is not round-to-nearest).
#define CV_U64 1.1102230246251565e-16
__host__ __device__ __forceinline__ double cv_gamma(int K) {
  return (2.0 * (double)K + 16.0) * CV_U64;
}
// Relative slack applied to an error bound computed in float64 so the
// rounding of its own evaluation is covered.
#define CV_ERR_SLACK (1.0 + 1.0e-12)

// ------------------------------------------------------ wave reductions
// Butterfly steps inside each 16-lane row use DPP lane permutes (xor 1, xor 2,
// half-row mirror, row mirror: each step combines two disjoint partial sums),
// then the four row results are read with readlane into scalar registers, so
// the result is wave-uniform.  float64 values move as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
#define CV_DPP_XOR1 0xB1
#define CV_DPP_XOR2 0x4E
#define CV_DPP_HALF_MIRROR 0x141
#define CV_DPP_MIRROR 0x140

// Sum over the 16 lanes of each row (every lane of the row gets it).
__device__ __forceinline__ double group16_sum(double v) {
  v += dpp_f64<CV_DPP_XOR1>(v);
  v += dpp_f64<CV_DPP_XOR2>(v);
  v += dpp_f64<CV_DPP_HALF_MIRROR>(v);
  v += dpp_f64<CV_DPP_MIRROR>(v);
  return v;
}
__device__ __forceinline__ double group16_max(double v) {
  v = fmax(v, dpp_f64<CV_DPP_XOR1>(v));
  v = fmax(v, dpp_f64<CV_DPP_XOR2>(v));
  v = fmax(v, dpp_f64<CV_DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp_f64<CV_DPP_MIRROR>(v));
  return v;
}
__device__ __forceinline__ double group16_min(double v) {
  v = fmin(v, dpp_f64<CV_DPP_XOR1>(v));
  v = fmin(v, dpp_f64<CV_DPP_XOR2>(v));
  v = fmin(v, dpp_f64<CV_DPP_HALF_MIRROR>(v));
  v = fmin(v, dpp_f64<CV_DPP_MIRROR>(v));
  return v;
}
// Whole-wave reductions; all lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v = group16_sum(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
  v = group16_max(v);
  return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) {
  v = group16_min(v);
  return fmin(fmin(lane_f64(v, 0), lane_f64(v, 16)), fmin(lane_f64(v, 32), lane_f64(v, 48)));
}

// ---------------------------------------------------- ReLU relaxation
// Relaxation of one ReLU neuron for a row whose coefficient on the neuron's
// output is psi (Lemma A.3; upper line = Planet line):
//   l >= 0: slope 1, intercept 0          u <= 0: slope 0, intercept 0
//   unstable, psi >= 0: slope alpha, 0    unstable, psi < 0: upper line
// For the upper line the slope is s = u/(u-l) (any rounding) and the
// intercept is chosen so that s z + t >= relu(z) at both ends z = l and
// z = u, which by convexity of relu makes the line valid on [l, u]:
//   t >= -s l   and   t >= u - s u,
// each evaluated in float64 and moved up by a margin that covers its
// rounding.  `lower` is set when alpha is the slope (the entries the slope
// gradient acts on).
struct Relax {
  double s, t;
  bool lower;
};
__device__ __forceinline__ Relax relu_relax(double psi, float lf, float uf, double alpha) {
  Relax r;
  const double l = (double)lf, u = (double)uf;
  r.lower = false;
  if (l >= 0.0) { r.s = 1.0; r.t = 0.0; return r; }
  if (u <= 0.0) { r.s = 0.0; r.t = 0.0; return r; }
  if (psi >= 0.0) { r.s = alpha; r.t = 0.0; r.lower = true; return r; }
  const double s = u / (u - l);
  const double t1 = -s * l;
  const double t2 = u - s * u;
  const double t = fmax(t1, t2);
  r.s = s;
  r.t = t + (u - l) * (4.0 * CV_U64);
  return r;
}

// The same relaxation split into a per-neuron part, computed once per
// (subdomain, neuron) and stored as float32: (slope, intercept) of the line
// used when alpha does not apply -- (1, 0) active, (0, 0) inactive, the
// upper line of an unstable neuron (intercept > 0, which marks it unstable)
// -- and the per-row choice by the sign of psi.  For the upper line the
// float32 slope s is taken as given and the intercept is computed from it
// (t >= -s l and t >= u - s u, as in relu_relax) and rounded up, so the
// stored line is itself a valid upper line.
__device__ __forceinline__ float2 relax_line(float lf, float uf) {
  const double l = (double)lf, u = (double)uf;
  if (l >= 0.0) return make_float2(1.0f, 0.0f);
  if (u <= 0.0) return make_float2(0.0f, 0.0f);
  const float s32 = (float)(u / (u - l));
  const double s = (double)s32;
  const double t = fmax(-s * l, u - s * u) + (u - l) * (4.0 * CV_U64);
  return make_float2(s32, ru32(t));
}
__device__ __forceinline__ Relax relax_apply(double psi, float2 line, double alpha) {
  Relax r;
  r.lower = line.y > 0.0f && psi >= 0.0;
  r.s = r.lower ? alpha : (double)line.x;
  r.t = r.lower ? 0.0 : (double)line.y;
  return r;
}

// float32 image of a float64 coefficient that keeps the sign decision
// psi >= 0 of relu_relax (a negative value never becomes -0.0).
__device__ __forceinline__ float trace32(double psi) {
  float f = (float)psi;
  if (psi < 0.0 && !(f < 0.0f)) f = -1.17549435e-38f;
  return f;
}

__device__ __forceinline__ double fabs_max(float a, float b) {
  return fmax(fabs((double)a), fabs((double)b));
}
