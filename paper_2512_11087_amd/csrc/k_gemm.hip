// Dense contractions of the hot path on the float64 matrix cores of gfx950
// (v_mfma_f64_16x16x4_f64), with the per-element work fused into the
// epilogue:
//   * backward pass, hidden layer: Psi = Omega W, then the ReLU relaxation
//     of the layer below (Lemma A.3) -> next Omega, plus the row sums that
//     feed the intercept and the rigorous error bound;
//   * backward pass, input layer: A = Omega W1, then the row-wise
//     concretization over the subdomain's box (Lemma A.2);
//   * re-concretization of the cached root planes over every subdomain box
//     ([lo | hi] times the packed plane matrix);
//   * adjoint of the backward pass for the slope gradient, with the Adam
//     step on alpha fused in.
//
// Tiling: a 256-thread workgroup (4 waves) computes a 64 x 256 output tile;
// wave w owns columns [64 w, 64 w + 64) of the tile and all 64 rows, i.e.
// 4 x 4 MFMA blocks of 16 x 16 (64 float64 accumulators per lane).  The K
// dimension is staged through LDS in chunks of 16 (A as float64, B as
// float32 converted when the fragment is formed).  B (the weights or the
// plane matrix) is shared by all subdomains and stays L2/MALL resident; A
// (per-row coefficients) is streamed from HBM once per 256 output columns.
//
// MFMA operand layout (16x16x4, float64; measured on gfx950): lane L supplies
// A[L%16][L/16] and B[L/16][L%16]; accumulator element v of lane L is
// D[L/16 + 4v][L%16] (rows interleaved by 4, unlike the float32 variant).
#include "cv_common.h"
#include "cv_internal.h"

typedef double d4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int GBM = 64, GBN = 256, GBK = 16;
constexpr int NWAVE = 4;
constexpr int WN = GBN / NWAVE;  // columns per wave
constexpr int MI = GBM / 16;
constexpr int NI = WN / 16;
constexpr int SA_LD = GBM + 2;   // float64 elements per staged k-row of A
constexpr int SB_LD = GBN + 4;   // float32 elements per staged k-row of B
constexpr int NSUM_MAX = 3;

struct LoadF64 {
  const double* p;
  int ld;
  __device__ __forceinline__ double operator()(int r, int k) const { return p[(size_t)r * ld + k]; }
};

// Row r of [lo | hi] (the per-subdomain box, 2 n0 columns).
struct LoadBox {
  const float* lo;
  const float* hi;
  int n0;
  __device__ __forceinline__ double operator()(int r, int k) const {
    return k < n0 ? (double)lo[(size_t)r * n0 + k] : (double)hi[(size_t)r * n0 + (k - n0)];
  }
};

template <class LoadA, class Epi>
__global__ __launch_bounds__(256) void k_gemm(int R, int K, int N, LoadA la,
                                              const float* __restrict__ Bm, int ldb, Epi epi,
                                              double* __restrict__ part, int ntiles) {
  __shared__ double sA[GBK * SA_LD];
  __shared__ float sB[GBK * SB_LD];
  __shared__ double sRed[NWAVE * GBM * NSUM_MAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * GBM;
  const int n0 = blockIdx.y * GBN;
  d4_t acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int ar = tid >> 2, akq = (tid & 3) * 4;   // A staging: row, first k
  const int bk = tid >> 4, bc0 = (tid & 15) * 16; // B staging: k, first column
  for (int k0 = 0; k0 < K; k0 += GBK) {
    {
      const int gr = m0 + ar;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gk = k0 + akq + q;
        sA[(akq + q) * SA_LD + ar] = (gr < R && gk < K) ? la(gr, gk) : 0.0;
      }
    }
    {
      const int gk = k0 + bk;
      const float* brow = Bm + (size_t)gk * ldb;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int gc = n0 + bc0 + q;
        sB[bk * SB_LD + bc0 + q] = (gk < K && gc < N) ? brow[gc] : 0.0f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      double af[MI], bf[NI];
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) af[i] = sA[kr * SA_LD + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NI; ++j) bf[j] = (double)sB[kr * SB_LD + wave * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  constexpr int NS = Epi::NSUM;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int lr = i * 16 + (lane >> 4) + 4 * v;
      const int r = m0 + lr;
      double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int c = n0 + wave * WN + j * 16 + (lane & 15);
        if (r < R && c < N) epi.apply(r, c, acc[i][j][v], sums);
      }
      if constexpr (NS > 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const double t = group16_sum(sums[s]);
          if ((lane & 15) == 0) sRed[(wave * GBM + lr) * NS + s] = t;
        }
      }
    }
  }
  if constexpr (NS > 0) {
    __syncthreads();
    if (tid < GBM) {
      const int r = m0 + tid;
      if (r < R) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          double t = 0.0;
#pragma unroll
          for (int w = 0; w < NWAVE; ++w) t += sRed[(w * GBM + tid) * NS + s];
          part[((size_t)r * ntiles + blockIdx.y) * NS + s] = t;
        }
      }
    }
  }
}

// Hidden layer of the backward pass: psi = (Omega W)[r, j] is the coefficient
// of post-activation j of the layer below; relax it, store the next Omega and
// accumulate  sum psi*t (intercept), sum Omega'*b (that layer's bias term) and
// sum |psi| * wrel (error weight).
struct EpiRelax {
  static constexpr int NSUM = 3;
  int M, Nh, off;
  const float* l;
  const float* u;
  const float* alpha;
  double alpha_def;
  const float* bprev;
  const double* wrel;
  double* Om;
  int ldo;
  float* trace;
  __device__ __forceinline__ void apply(int r, int j, double psi, double* s) const {
    const int b = r / M;
    const size_t bi = (size_t)b * Nh + off + j;
    const size_t ri = (size_t)r * Nh + off + j;
    const double al = alpha ? (double)alpha[ri] : alpha_def;
    const Relax rl = relu_relax(psi, l[bi], u[bi], al);
    const double om = psi * rl.s;
    Om[(size_t)r * ldo + j] = om;
    if (trace) trace[ri] = trace32(psi);
    s[0] += psi * rl.t;
    s[1] += om * (double)bprev[j];
    s[2] += fabs(psi) * wrel[j];
  }
};

// Input layer: a = (Omega W1)[r, j] is the coefficient of x_j in the final
// plane; accumulate min(a lo_j, a hi_j) (Lemma A.2) and |a| X0_j (error).
struct EpiFinal {
  static constexpr int NSUM = 2;
  int M, n0;
  const float* lo;
  const float* hi;
  const double* X0;
  double* Ax;
  float* A_out;
  __device__ __forceinline__ void apply(int r, int j, double a, double* s) const {
    const int b = r / M;
    const double xl = (double)lo[(size_t)b * n0 + j], xh = (double)hi[(size_t)b * n0 + j];
    s[0] += fmin(a * xl, a * xh);
    s[1] += fabs(a) * X0[j];
    if (Ax) Ax[(size_t)r * n0 + j] = a;
    if (A_out) A_out[(size_t)r * n0 + j] = (float)a;
  }
};

// Re-concretized bound of cached plane column `col` over box r.
struct EpiPlanes {
  static constexpr int NSUM = 0;
  int U, Nh;
  const float* cP;
  const double* eP;
  const int32_t* uidx;
  const float* l0;
  const float* u0;
  float* l;
  float* u;
  __device__ __forceinline__ void apply(int b, int col, double v, double*) const {
    if (col < U) {
      const int j = uidx[col];
      const double x = v + (double)cP[col] - eP[col];
      l[(size_t)b * Nh + j] = fmaxf(rd32(x), l0[j]);
    } else {
      const int j = uidx[col - U];
      const double x = v + (double)cP[col] + eP[col];
      u[(size_t)b * Nh + j] = fminf(ru32(x), u0[j]);
    }
  }
};

// Adjoint of one hidden layer k: Omega_bar = Psi_bar W_k^T + b_k (acc + b),
// gradient of the alpha of lower-line entries = Omega_bar * Psi (forward
// trace), Psi_bar of the layer above = Omega_bar * slope + intercept, and the
// projected Adam ascent step on alpha.
struct EpiAdj {
  static constexpr int NSUM = 0;
  int M, Nh, off;
  const float* bias;
  const float* l;
  const float* u;
  float* alpha;
  double alpha_def;
  const float* trace;
  const uint8_t* infeasible;
  float* grad;
  float* am;
  float* av;
  double lr, b1, b2, eps, bc1, bc2;
  double* out;
  int ldo;
  __device__ __forceinline__ void apply(int r, int j, double acc, double*) const {
    const int b = r / M;
    const double om = acc + (double)bias[j];
    const size_t ri = (size_t)r * Nh + off + j;
    const size_t bi = (size_t)b * Nh + off + j;
    const double al = alpha ? (double)alpha[ri] : alpha_def;
    const double psi = (double)trace[ri];
    const Relax rl = relu_relax(psi, l[bi], u[bi], al);
    const bool dead = infeasible && infeasible[b];
    const double g = (rl.lower && !dead) ? om * psi : 0.0;
    if (out) out[(size_t)r * ldo + j] = om * rl.s + rl.t;
    if (grad) grad[ri] = (float)g;
    if (lr > 0.0 && alpha) {
      const double m = b1 * (double)am[ri] + (1.0 - b1) * g;
      const double v = b2 * (double)av[ri] + (1.0 - b2) * g * g;
      const double mh = m / bc1, vh = v / bc2;
      double a = al + lr * mh / (sqrt(vh) + eps);
      a = fmin(fmax(a, 0.0), 1.0);
      am[ri] = (float)m;
      av[ri] = (float)v;
      alpha[ri] = (float)a;
    }
  }
};

template <class LoadA, class Epi>
hipError_t run_gemm(int R, int K, int N, LoadA la, const float* Bm, int ldb, Epi epi,
                    double* part, hipStream_t s) {
  if (R <= 0 || N <= 0) return hipSuccess;
  const int nt = (N + GBN - 1) / GBN;
  dim3 grid((R + GBM - 1) / GBM, nt);
  hipLaunchKernelGGL((k_gemm<LoadA, Epi>), grid, dim3(256), 0, s, R, K, N, la, Bm, ldb, epi, part, nt);
  return hipGetLastError();
}

}  // namespace

int gemm_ntiles(int N) { return (N + GBN - 1) / GBN; }

hipError_t launch_gemm_relax(int R, int K, int N, const double* Om, const float* W, int M, int Nh,
                             int off, const float* l, const float* u, const float* alpha,
                             double alpha_def, const float* bprev, const double* wrel,
                             double* Om_out, float* trace, double* part, hipStream_t s) {
  EpiRelax e{M, Nh, off, l, u, alpha, alpha_def, bprev, wrel, Om_out, N, trace};
  return run_gemm(R, K, N, LoadF64{Om, K}, W, N, e, part, s);
}

hipError_t launch_gemm_final(int R, int K, int N, const double* Om, const float* W, int M,
                             const float* lo, const float* hi, const double* X0, double* Ax,
                             float* A_out, double* part, hipStream_t s) {
  EpiFinal e{M, N, lo, hi, X0, Ax, A_out};
  return run_gemm(R, K, N, LoadF64{Om, K}, W, N, e, part, s);
}

hipError_t launch_gemm_planes(int B, int n0, int U, const float* lo, const float* hi,
                              const float* P, const float* cP, const double* eP,
                              const int32_t* uidx, const float* l0, const float* u0, int Nh,
                              float* l, float* u, hipStream_t s) {
  EpiPlanes e{U, Nh, cP, eP, uidx, l0, u0, l, u};
  return run_gemm(B, 2 * n0, 2 * U, LoadBox{lo, hi, n0}, P, 2 * U, e, nullptr, s);
}

hipError_t launch_gemm_adjoint(int R, int K, int N, const double* Abar, const float* Wt,
                               const float* b, int M, int Nh, int off, const float* l,
                               const float* u, float* alpha, double alpha_def,
                               const float* trace, const uint8_t* infeasible, float* grad,
                               float* adam_m, float* adam_v, double lr, double b1, double b2,
                               double eps, int step, double* Psibar_out, hipStream_t s) {
  const double bc1 = 1.0 - pow(b1, (double)step), bc2 = 1.0 - pow(b2, (double)step);
  EpiAdj e{M, Nh, off, b, l, u, alpha, alpha_def, trace, infeasible, grad, adam_m, adam_v,
           lr, b1, b2, eps, bc1, bc2, Psibar_out, N};
  return run_gemm(R, K, N, LoadF64{Abar, K}, Wt, N, e, nullptr, s);
}
