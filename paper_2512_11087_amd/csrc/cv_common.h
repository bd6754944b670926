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
// A pointer every lane holds alike, moved to scalar registers (so that a
// buffer resource built from it is scalar: a resource in vector registers
// makes the compiler loop over its distinct values around every load).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t u = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (T*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
// A float64 value every lane holds alike, moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
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
// Three independent sums in one pass (their permute chains interleave).
__device__ __forceinline__ void wave_sum3(double& a, double& b, double& c) {
  a += dpp_f64<CV_DPP_XOR1>(a);
  b += dpp_f64<CV_DPP_XOR1>(b);
  c += dpp_f64<CV_DPP_XOR1>(c);
  a += dpp_f64<CV_DPP_XOR2>(a);
  b += dpp_f64<CV_DPP_XOR2>(b);
  c += dpp_f64<CV_DPP_XOR2>(c);
  a += dpp_f64<CV_DPP_HALF_MIRROR>(a);
  b += dpp_f64<CV_DPP_HALF_MIRROR>(b);
  c += dpp_f64<CV_DPP_HALF_MIRROR>(c);
  a += dpp_f64<CV_DPP_MIRROR>(a);
  b += dpp_f64<CV_DPP_MIRROR>(b);
  c += dpp_f64<CV_DPP_MIRROR>(c);
  a = (lane_f64(a, 0) + lane_f64(a, 16)) + (lane_f64(a, 32) + lane_f64(a, 48));
  b = (lane_f64(b, 0) + lane_f64(b, 16)) + (lane_f64(b, 32) + lane_f64(b, 48));
  c = (lane_f64(c, 0) + lane_f64(c, 16)) + (lane_f64(c, 32) + lane_f64(c, 48));
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

// Computed in two parts: a per-neuron part -- (slope, intercept) of
// the line used when alpha does not apply: (1, 0) active, (0, 0) inactive,
// the upper line of an unstable neuron (intercept > 0, which marks it
// unstable) -- and the per-row choice by the sign of psi.  Evaluated in
// float64 where it is used (a stored float32 slope and intercept would
// loosen every unstable neuron's line by ~2^-24 of its height, which adds up
// over thousands of neurons; recomputing costs one division per element).
typedef double2 cv_line;
__device__ __forceinline__ cv_line relax_line(float lf, float uf) {
  const double l = (double)lf, u = (double)uf;
  if (l >= 0.0) return make_double2(1.0, 0.0);
  if (u <= 0.0) return make_double2(0.0, 0.0);
  const double s = u / (u - l);
  const double t = fmax(-s * l, u - s * u) + (u - l) * (4.0 * CV_U64);
  return make_double2(s, t);
}
__device__ __forceinline__ Relax relax_apply(double psi, cv_line line, double alpha) {
  Relax r;
  r.lower = line.y > 0.0 && psi >= 0.0;
  r.s = r.lower ? alpha : line.x;
  r.t = r.lower ? 0.0 : line.y;
  return r;
}

// float32 image of a float64 coefficient that keeps the sign decision
// psi >= 0 of relax_apply (a negative value never becomes -0.0).
__device__ __forceinline__ float trace32(double psi) {
  float f = (float)psi;
  if (psi < 0.0 && !(f < 0.0f)) f = -1.17549435e-38f;
  return f;
}

// p[j] for j < n, else 0, without a branch: the index is clamped into
// [0, n) (callers guarantee n >= 1), so the load is always in bounds and is
// issued together with its neighbours; a select then zeroes the tail.  (A
// guarded load `j < n ? p[j] : 0` becomes one branch per load, which
// serialises the loads' latencies.)
__device__ __forceinline__ float ld_or0(const float* p, int j, int n) {
  const float v = p[j < n ? j : n - 1];
  return j < n ? v : 0.0f;
}
__device__ __forceinline__ double ld_or0(const double* p, int j, int n) {
  const double v = p[j < n ? j : n - 1];
  return j < n ? v : 0.0;
}

// Buffer view of `bytes` bytes at a wave-uniform address p.  Raw buffer
// loads past the end return 0 without touching memory (the hardware range
// check of an unstrided buffer resource), so lane-strided rows of any
// length load without branches and keep immediate offsets.  Word 3 of the
// descriptor is the gfx9-family default (32-bit data format).
typedef __amdgpu_buffer_rsrc_t cv_buf;
__device__ __forceinline__ cv_buf cv_buffer(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// Loads at a byte offset (the range check covers the vector offset and the
// instruction's immediate offset, so constants stay in the immediate field).
__device__ __forceinline__ float buf_f32(cv_buf r, int byte_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
__device__ __forceinline__ double buf_f64(cv_buf r, int byte_off) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
  return __hiloint2double((int)v.y, (int)v.x);
}
// Keeps the compiler from hoisting values derived from v out of a loop:
// hoisted conversions and per-element offsets would stay live in registers
// for the whole loop (and offsets hoisted that way no longer fold into the
// immediate offset field of the loads).
// Logical workgroup index for launches whose neighbouring workgroups share
// data (rows of one subdomain, their constraint rows): the hardware hands
// workgroup i to XCD i mod 8, each XCD with its own L2, so renumber the
// workgroups that one XCD runs into a contiguous range of logical indices.
// A bijection of [0, nblocks).
__device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned nblocks) {
  constexpr unsigned NX = 8;
  const unsigned per = nblocks / NX, rem = nblocks % NX;
  const unsigned x = bid % NX, q = bid / NX;
  return x * per + (x < rem ? x : rem) + q;
}

__device__ __forceinline__ void cv_opaque(float& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void cv_opaque(int& v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ double fabs_max(float a, float b) {
  return fmax(fabs((double)a), fabs((double)b));
}
