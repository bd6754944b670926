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
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, CV_WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, CV_WAVE));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, CV_WAVE));
  return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, CV_WAVE);
  return v;
}
// Sum over the 16 lanes that share (lane / 16): the lanes of one row group
// of an MFMA 16x16 output block.
__device__ __forceinline__ double group16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, CV_WAVE);
  return v;
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
