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
// Tiling: a 256-thread workgroup (4 waves) computes a BM x BN output tile
// (Tile<BM, BN>); wave w owns columns [w BN/4, (w+1) BN/4) of the tile and
// all BM rows, i.e. (BM/16) x (BN/64) MFMA blocks of 16 x 16.  The K
// dimension is staged through LDS in chunks of 16 (A as float64, B as
// float32 converted when the fragment is formed), double-buffered.  B (the
// weights or the plane matrix) is shared by all subdomains and stays
// L2/MALL resident; A (per-row coefficients) is streamed from HBM once per
// BN output columns.
//
// MFMA operand layout (16x16x4, float64; measured on gfx950): lane L supplies
// A[L%16][L/16] and B[L/16][L%16]; accumulator element v of lane L is
// D[L/16 + 4v][L%16] (rows interleaved by 4, unlike the float32 variant).
#include <type_traits>

#include <algorithm>
#include "cv_common.h"
#include "cv_internal.h"

typedef double d4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int GBK = 16;
constexpr int NWAVE = 4;
constexpr int NSUM_MAX = 3;

// Output tile of one workgroup: BM rows x BN columns (4 waves side by side).
template <int BM_, int BN_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_;
  static constexpr int WN = BN / NWAVE;   // columns per wave
  static constexpr int MI = BM / 16;
  static constexpr int NI = WN / 16;
  static constexpr int SA_LD = BM + 2;    // float64 elements per staged k-row of A
  static constexpr int SB_LD = BN + 16;   // float32 elements per staged k-row of B (rows 64 B apart in banks)
  static constexpr int APT = BM * GBK / 256;  // A elements staged per thread
  static constexpr int BPT = BN * GBK / 256;  // B elements staged per thread
  static_assert(APT == 2 || APT == 4 || APT == 8, "A staging");
  static_assert(BPT % 4 == 0 && BPT <= 16, "B staging");
};
// Tile shapes, measured at the 784-256x6 shapes (147456 rows x 256 columns):
// narrow tiles keep the accumulators small (32 x 128: 2 x 2 MFMA blocks per
// wave, 16 doubles per lane), so the fused epilogues fit without
// spilling and several workgroups share a CU; their epilogues then overlap
// the other workgroups' MFMA work.  Backward, final and adjoint GEMMs:
// 32 x 128 (main loop 73-81 % of the float64 MFMA peak, vs 67-72 % with
// 64 x 256).  The plane re-concretization (K = 2 n0, N = 2 U, few rows)
// prefers 64 x 128.  Both have 128 columns, which fixes the number of
// column tiles that the row-sum partials are laid out for.
typedef Tile<32, 128> TileDefault;
typedef Tile<64, 128> TilePlanes;
static_assert(TileDefault::BN == TilePlanes::BN, "row-sum partials assume one column tiling");

// A loaders return 4 consecutive k of one row (zeros outside [0,R) x [0,K)).
struct LoadF64 {
  const double* p;
  int ld;
  template <int NV>
  __device__ __forceinline__ void load(int r, int k, int R, int K, double (&v)[NV]) const {
    if (r < R && k + NV - 1 < K && (ld & 1) == 0) {
      const double2* q = reinterpret_cast<const double2*>(p + (size_t)r * ld + k);
#pragma unroll
      for (int t = 0; t < NV / 2; ++t) {
        const double2 x = q[t];
        v[2 * t] = x.x;
        v[2 * t + 1] = x.y;
      }
      return;
    }
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = (r < R && k + t < K) ? p[(size_t)r * ld + k + t] : 0.0;
  }
};

// Row r of [lo | hi] (the per-subdomain box, 2 n0 columns).
struct LoadBox {
  const float* lo;
  const float* hi;
  int n0;
  template <int NV>
  __device__ __forceinline__ void load(int r, int k, int R, int K, double (&v)[NV]) const {
    static_assert(NV % 2 == 0, "pairs");
    if (r < R && (n0 % NV) == 0 && k + NV - 1 < K) {
      const float* src = k < n0 ? lo + (size_t)r * n0 + k : hi + (size_t)r * n0 + (k - n0);
#pragma unroll
      for (int t = 0; t < NV / 2; ++t) {
        const float2 x = reinterpret_cast<const float2*>(src)[t];
        v[2 * t] = x.x;
        v[2 * t + 1] = x.y;
      }
      return;
    }
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int kk = k + t;
      v[t] = (r < R && kk < K)
                 ? (kk < n0 ? (double)lo[(size_t)r * n0 + kk] : (double)hi[(size_t)r * n0 + (kk - n0)])
                 : 0.0;
    }
  }
};

// NV consecutive columns of one row of B (zeros outside).
template <int NV>
__device__ __forceinline__ void load_bn(const float* __restrict__ Bm, int ldb, int gk, int gc, int K,
                                        int N, float (&v)[NV]) {
  const float* row = Bm + (size_t)gk * ldb + gc;
  if (gk < K && gc + NV - 1 < N && (ldb & 3) == 0) {
    const float4* q = reinterpret_cast<const float4*>(row);
#pragma unroll
    for (int t = 0; t < NV / 4; ++t) {
      const float4 x = q[t];
      v[4 * t] = x.x; v[4 * t + 1] = x.y; v[4 * t + 2] = x.z; v[4 * t + 3] = x.w;
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < NV; ++t) v[t] = (gk < K && gc + t < N) ? row[t] : 0.0f;
}

// Software pipeline: while the MFMAs consume K-chunk c from one LDS buffer,
// the global loads of chunk c+1 are in flight into registers; they are
// written to the other buffer afterwards, one barrier per chunk.
// One BM x BN output tile at (m0, n0); its row-sum partials go to column
// tile `tn`.  Ends with LDS free for the next call.
template <class T, class LoadA, class Epi>
__device__ __forceinline__ void gemm_tile(int m0, int n0, int R, int K, int N, const LoadA& la,
                                          const float* __restrict__ Bm, int ldb, const Epi& epi,
                                          double* __restrict__ part, int ntiles, int tn) {
  constexpr int GBM = T::BM, GBN = T::BN, WN = T::WN, MI = T::MI, NI = T::NI;
  constexpr int SA_LD = T::SA_LD, SB_LD = T::SB_LD, APT = T::APT, BPT = T::BPT;
  __shared__ double sA[2][GBK * SA_LD];
  __shared__ float sB[2][GBK * SB_LD];
  __shared__ double sRed[NWAVE * GBM * NSUM_MAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  (void)GBN;
  d4_t acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
  // column blocks of this wave that intersect [0, N) (wave-uniform)
  int nblk = (N - (n0 + wave * WN) + 15) / 16;
  nblk = nblk < 0 ? 0 : (nblk > NI ? NI : nblk);

  constexpr int AQ = GBK / APT;                        // threads per staged row of A
  const int ar = tid / AQ, akq = (tid % AQ) * APT;     // A staging: row, first k
  const int bk = tid >> 4, bc0 = (tid & 15) * BPT;     // B staging: k, first column
  double pa[APT];
  float pb[BPT];
  auto fetch = [&](int k0) {
    la.template load<APT>(m0 + ar, k0 + akq, R, K, pa);
    load_bn<BPT>(Bm, ldb, k0 + bk, n0 + bc0, K, N, pb);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < APT; ++q) sA[buf][(akq + q) * SA_LD + ar] = pa[q];
#pragma unroll
    for (int q = 0; q < BPT; q += 4)
      *reinterpret_cast<float4*>(&sB[buf][bk * SB_LD + bc0 + q]) =
          make_float4(pb[q], pb[q + 1], pb[q + 2], pb[q + 3]);
  };
  const int nch = (K + GBK - 1) / GBK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) fetch((c + 1) * GBK);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      double af[MI], bf[NI];
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) af[i] = sA[buf][kr * SA_LD + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NI; ++j) bf[j] = (double)sB[buf][kr * SB_LD + wave * WN + j * 16 + (lane & 15)];
      if (nblk == NI) {  // full tile: straight-line MFMA issue
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      } else {
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          if (j < nblk) {
#pragma unroll
            for (int i = 0; i < MI; ++i)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (c + 1 < nch) stash(buf ^ 1);
    __syncthreads();
  }

  // Epilogue, in groups of VGROUP accumulator rows: all global loads of a
  // group are issued first (Epi::load), then the group is computed and
  // stored (Epi::apply), so load latency is paid once per group rather than
  // once per element (the stores could otherwise alias later loads).
  constexpr int NS = Epi::NSUM;
  constexpr int VG = Epi::VGROUP;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int v0 = 0; v0 < 4; v0 += VG) {
      typename Epi::Row rw[VG];
      typename Epi::Pre pre[VG][NI];
#pragma unroll
      for (int dv = 0; dv < VG; ++dv) {
        const int r = m0 + i * 16 + (lane >> 4) + 4 * (v0 + dv);
        rw[dv] = epi.row(r < R ? r : R - 1);
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          const int c = n0 + wave * WN + j * 16 + (lane & 15);
          if (r < R && j < nblk && c < N) pre[dv][j] = epi.load(rw[dv], r, c);
        }
      }
#pragma unroll
      for (int dv = 0; dv < VG; ++dv) {
        const int lr = i * 16 + (lane >> 4) + 4 * (v0 + dv);
        const int r = m0 + lr;
        double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          const int c = n0 + wave * WN + j * 16 + (lane & 15);
          if (r < R && j < nblk && c < N) epi.apply(rw[dv], pre[dv][j], r, c, acc[i][j][v0 + dv], sums);
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
          part[((size_t)r * ntiles + tn) * NS + s] = t;
        }
      }
    }
  }
}

// Tile order: workgroup i runs on XCD i mod 8, each XCD with its own L2, so
// the linear grid is renumbered (xcd_block) to give every XCD a contiguous
// range, walked row tile by row tile with all `ntiles` column tiles of a row
// tile next to each other: they run at about the same time on one XCD, and
// the rows of A that all of them read come from HBM once.
__device__ __forceinline__ void tile_of(int ntiles, int& tm, int& tn) {
  const int t = (int)xcd_block(blockIdx.x, gridDim.x);
  tm = t / ntiles;
  tn = t - tm * ntiles;
}

template <class T, int OCC, class LoadA, class Epi>
__global__ __launch_bounds__(256, OCC) void k_gemm(int R, int K, int N, LoadA la,
                                                   const float* __restrict__ Bm, int ldb, Epi epi,
                                                   double* __restrict__ part, int ntiles) {
  int tm, tn;
  tile_of(ntiles, tm, tn);
  gemm_tile<T>(tm * T::BM, tn * T::BN, R, K, N, la, Bm, ldb, epi, part, ntiles, tn);
}

// Hidden layer of the backward pass: psi = (Omega W)[r, j] is the coefficient
// of post-activation j of the layer below; relax it, store the next Omega and
// accumulate  sum psi*t (intercept), sum Omega'*b (that layer's bias term) and
// sum |psi| * wrel (error weight).
// MULTI: rows of several properties (the error weight of each row's
// property is looked up); else one property's weight for every row.
template <bool MULTI>
struct EpiRelax {
  static constexpr int NSUM = 3;
  static constexpr int VGROUP = 4;
  int M, Nh, off;
  const float* lz;   // pre-activation bounds l, u of the layer below [B, Nh]
  const float* uz;
  const float* alpha;
  double alpha_def;
  const float* bprev;
  const double* wrel;  // !MULTI: error weight of layer `layer`
  CvProps props;       // MULTI: per-property error weights
  int layer;
  double* Om;
  int ldo;
  float* trace;
  struct RowS {
    const float* l;
    const float* u;
    size_t ri;
  };
  struct RowM : RowS {
    const double* wrel;
  };
  typedef typename std::conditional<MULTI, RowM, RowS>::type Row;
  __device__ __forceinline__ Row row(int r) const {
    const int b = r / M;
    const RowS rs{lz + (size_t)b * Nh + off, uz + (size_t)b * Nh + off, (size_t)r * Nh + off};
    if constexpr (MULTI) {
      RowM rm;
      static_cast<RowS&>(rm) = rs;
      rm.wrel = prop_of(props, b).wrel[layer];
      return rm;
    } else {
      return rs;
    }
  }
  __device__ __forceinline__ const double* wrel_of(const Row& w) const {
    if constexpr (MULTI) return w.wrel;
    else return wrel;
  }
  struct Pre {
    float l, u, al;
  };
  __device__ __forceinline__ Pre load(const Row& w, int, int j) const {
    return Pre{w.l[j], w.u[j], alpha ? alpha[w.ri + j] : (float)alpha_def};
  }
  __device__ __forceinline__ void apply(const Row& w, const Pre& p, int r, int j, double psi,
                                        double* s) const {
    const size_t ri = w.ri + j;
    const double al = alpha ? (double)p.al : alpha_def;
    const Relax rl = relax_apply(psi, relax_line(p.l, p.u), al);
    const double om = psi * rl.s;
    Om[(size_t)r * ldo + j] = om;
    if (trace) trace[ri] = trace32(psi);
    s[0] += psi * rl.t;
    s[1] += om * (double)bprev[j];
    s[2] += fabs(psi) * wrel_of(w)[j];
  }
};

// Input layer: a = (Omega W1)[r, j] is the coefficient of x_j in the final
// plane; accumulate min(a lo_j, a hi_j) (Lemma A.2) and |a| X0_j (error).
template <bool MULTI>
struct EpiFinal {
  static constexpr int NSUM = 2;
  static constexpr int VGROUP = 4;
  int M, n0;
  const float* lo;
  const float* hi;
  const double* X0;  // !MULTI: max(|lo0|, |hi0|) of the property
  CvProps props;     // MULTI: per property
  double* Ax;
  float* A_out;
  struct RowS {
    const float* lo;
    const float* hi;
  };
  struct RowM : RowS {
    const double* X0;
  };
  typedef typename std::conditional<MULTI, RowM, RowS>::type Row;
  __device__ __forceinline__ Row row(int r) const {
    const int b = r / M;
    const RowS rs{lo + (size_t)b * n0, hi + (size_t)b * n0};
    if constexpr (MULTI) {
      RowM rm;
      static_cast<RowS&>(rm) = rs;
      rm.X0 = prop_of(props, b).X0;
      return rm;
    } else {
      return rs;
    }
  }
  struct Pre {
    float xl, xh;
  };
  __device__ __forceinline__ Pre load(const Row& w, int, int j) const { return Pre{w.lo[j], w.hi[j]}; }
  __device__ __forceinline__ void apply(const Row& w, const Pre& p, int r, int j, double a,
                                        double* s) const {
    const double xl = (double)p.xl, xh = (double)p.xh;
    s[0] += fmin(a * xl, a * xh);
    if constexpr (MULTI) s[1] += fabs(a) * w.X0[j];
    else s[1] += fabs(a) * X0[j];
    if (Ax) Ax[(size_t)r * n0 + j] = a;
    if (A_out) A_out[(size_t)r * n0 + j] = (float)a;
  }
};

// Re-concretized bound of cached plane column `col` over box b; MULTI: for
// the boxes of property p only (rows of other properties are left alone).
template <bool MULTI>
struct EpiPlanes {
  static constexpr int NSUM = 0;
  static constexpr int VGROUP = 4;
  int U, Nh;
  const double* cP;
  const double* eP;
  const int32_t* uidx;
  const float* l0;
  const float* u0;
  float* l;
  float* u;
  CvProps props;
  int p;
  struct RowS {};
  struct RowM {
    bool mine;
  };
  typedef typename std::conditional<MULTI, RowM, RowS>::type Row;
  __device__ __forceinline__ Row row(int b) const {
    if constexpr (MULTI) return RowM{prop_index(props, b) == p};
    else return RowS{};
  }
  struct Pre {};
  __device__ __forceinline__ Pre load(const Row&, int, int) const { return Pre{}; }
  __device__ __forceinline__ void apply(const Row& w, const Pre&, int b, int col, double v,
                                        double*) const {
    if constexpr (MULTI) {
      if (!w.mine) return;
    }
    if (col < U) {
      const int j = uidx[col];
      const double x = v + cP[col] - eP[col];
      l[(size_t)b * Nh + j] = fmaxf(rd32(x), l0[j]);
    } else {
      const int j = uidx[col - U];
      const double x = v + cP[col] + eP[col];
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
  static constexpr int VGROUP = 2;
  int M, Nh, off;
  const float* bias;
  const float* lz;
  const float* uz;
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
  const float* alpha_in;  // slopes read (null: alpha_def everywhere); alpha: where they are written
  bool fresh;             // Adam's moments start at zero (not read)
  struct Row {
    const float* l;
    const float* u;
    size_t ri;
    bool dead;
  };
  __device__ __forceinline__ Row row(int r) const {
    const size_t b = (size_t)(r / M);
    return Row{lz + b * Nh + off, uz + b * Nh + off, (size_t)r * Nh + off,
               infeasible != nullptr && infeasible[b] != 0};
  }
  struct Pre {
    float l, u, psi, al, m, v;
  };
  __device__ __forceinline__ Pre load(const Row& w, int, int j) const {
    const size_t ri = w.ri + j;
    const bool adam = lr > 0.0 && alpha && !fresh;
    return Pre{w.l[j], w.u[j], trace[ri], alpha_in ? alpha_in[ri] : (float)alpha_def,
               adam ? am[ri] : 0.0f, adam ? av[ri] : 0.0f};
  }
  __device__ __forceinline__ void apply(const Row& w, const Pre& p, int r, int j, double acc,
                                        double*) const {
    const double om = acc + (double)bias[j];
    const size_t ri = w.ri + j;
    const double al = alpha_in ? (double)p.al : alpha_def;
    const double psi = (double)p.psi;
    const Relax rl = relax_apply(psi, relax_line(p.l, p.u), al);
    const bool dead = w.dead;
    const double g = (rl.lower && !dead) ? om * psi : 0.0;
    if (out) out[(size_t)r * ldo + j] = om * rl.s + rl.t;
    if (grad) grad[ri] = (float)g;
    if (lr > 0.0 && alpha) {
      const double m = b1 * (double)p.m + (1.0 - b1) * g;
      const double v = b2 * (double)p.v + (1.0 - b2) * g * g;
      const double mh = m / bc1, vh = v / bc2;
      double a = al + lr * mh / (sqrt(vh) + eps);
      a = fmin(fmax(a, 0.0), 1.0);
      am[ri] = (float)m;
      av[ri] = (float)v;
      alpha[ri] = (float)a;
    }
  }
};

// ------------------------------------------------------------ convolutions
// The backward pass through a conv layer is a transposed convolution of each
// row of Omega (and the adjoint a forward convolution), computed directly
// rather than as a product with the layer's dense matrix: float64 FMAs on the
// vector units (whose float64 rate equals the matrix cores' on gfx950), one
// workgroup per row, the same fused epilogues as the GEMMs.  A wave takes a
// task = (channel block, chunk of 64 output positions); the block's weights
// are wave-uniform (scalar loads), each input value read feeds CB FMAs.  A
// row that fits is first staged in LDS with wide coalesced loads, so the
// taps read LDS instead of issuing one dependent global load each.
// Transposed convolution: the lanes of a task share one stride-parity class
// of output positions (iy = cy + s a, ix = cx + s b), so for every tap the
// divisibility (iy + p - ky) % s is uniform and only the ~k^2/s^2 valid taps
// are visited; borders are masked per lane.

// Row sums of a workgroup into the partials of column tile 0 (the other
// tiles of the row get zeros), the layout the GEMM epilogues write.
template <int NS>
__device__ __forceinline__ void conv_row_sums(double (&sums)[NSUM_MAX], double* sred, double* part,
                                              int r, int ntiles) {
  if constexpr (NS > 0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const double t = wave_sum(sums[q]);
      if (lane == 0) sred[wave * NSUM_MAX + q] = t;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
      const int q = threadIdx.x;
      part[((size_t)r * ntiles) * NS + q] =
          (sred[q] + sred[NSUM_MAX + q]) + (sred[2 * NSUM_MAX + q] + sred[3 * NSUM_MAX + q]);
    }
    for (int i = threadIdx.x; i < (ntiles - 1) * NS; i += 256)
      part[((size_t)r * ntiles + 1) * NS + i] = 0.0;
  }
}

// Kernel weights are read through the constant address space: their
// addresses are wave-uniform and nothing in these kernels writes them, so
// they come in by scalar loads and feed the FMAs from SGPRs.
typedef const __attribute__((address_space(4))) double* conv_wptr;

// Largest input row staged in LDS (doubles): 64 KiB keeps two workgroups
// per CU; longer rows are read from global memory directly.
constexpr int CONV_STAGE_MAX = 8192;

// Copy one row into LDS with many loads in flight per thread.
__device__ __forceinline__ void conv_stage(double* __restrict__ dst, const double* __restrict__ src,
                                           int n) {
  int i = threadIdx.x;
  for (; i + 3 * 256 < n; i += 4 * 256) {
    const double a0 = src[i], a1 = src[i + 256], a2 = src[i + 512], a3 = src[i + 768];
    dst[i] = a0;
    dst[i + 256] = a1;
    dst[i + 512] = a2;
    dst[i + 768] = a3;
  }
  for (; i < n; i += 256) dst[i] = src[i];
  __syncthreads();
}

// P positions per lane (lanes take consecutive positions, P groups of 64
// apart): each weight a scalar load brings feeds P * CB FMAs and each wave
// has P input loads in flight per step.
template <class Epi, int CB, bool STAGE, int P>
__global__ __launch_bounds__(256) void k_convt(int R, ConvDesc cd, const double* __restrict__ in,
                                               Epi epi, double* __restrict__ part, int ntiles) {
  extern __shared__ double srow[];
  __shared__ double sred[4 * NSUM_MAX];
  constexpr int NS = Epi::NSUM;
  constexpr int CH = 64 * P;  // positions per task
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t cin = (size_t)cd.ho * cd.wo;
  const double* row = in + (size_t)r * cd.co * cin;
  if constexpr (STAGE) conv_stage(srow, row, (int)(cd.co * cin));
  const double* src = STAGE ? srow : row;
  const int cpad = cd.ptp;
  const int nblk = (cd.ci + CB - 1) / CB;
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
  // tasks: (block, parity class, chunk of CH positions of that class)
  int per_blk = 0;
  for (int cy = 0; cy < cd.s; ++cy)
    for (int cx = 0; cx < cd.s; ++cx) {
      const int ny = (cd.hi - cy + cd.s - 1) / cd.s, nx = (cd.wi - cx + cd.s - 1) / cd.s;
      per_blk += (ny * nx + CH - 1) / CH;
    }
  const int ntask = per_blk * nblk;
  for (int task = wave; task < ntask; task += 4) {
    // decode (uniform): block, class, chunk
    const int blk = task / per_blk;
    int rem = task - blk * per_blk;
    int cy = 0, cx = 0, ny = 0, nx = 0;
    for (int c = 0; c < cd.s * cd.s; ++c) {
      const int y = c / cd.s, x = c % cd.s;
      const int yy = (cd.hi - y + cd.s - 1) / cd.s, xx = (cd.wi - x + cd.s - 1) / cd.s;
      const int nch = (yy * xx + CH - 1) / CH;
      if (rem < nch) {
        cy = y; cx = x; ny = yy; nx = xx;
        break;
      }
      rem -= nch;
    }
    bool live[P];
    int iy[P], ix[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int idx = rem * CH + 64 * p + lane;
      live[p] = idx < ny * nx;
      iy[p] = cy + cd.s * (live[p] ? idx / nx : 0);
      ix[p] = cx + cd.s * (live[p] ? idx % nx : 0);
    }
    const int ci0 = blk * CB;
    double acc[P][CB];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < CB; ++q) acc[p][q] = 0.0;
    const int ky0 = (cy + cd.p) % cd.s, kx0 = (cx + cd.p) % cd.s;
    for (int ky = ky0; ky < cd.k; ky += cd.s) {
      for (int kx = kx0; kx < cd.k; kx += cd.s) {
        int base[P];
        bool v[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          // exact when >= 0: iy + p - ky = s * oy (same class)
          const int oy = (iy[p] + cd.p - ky) / cd.s, ox = (ix[p] + cd.p - kx) / cd.s;
          v[p] = live[p] && iy[p] + cd.p - ky >= 0 && oy < cd.ho && ix[p] + cd.p - kx >= 0 &&
                 ox < cd.wo;
          base[p] = v[p] ? oy * cd.wo + ox : 0;
        }
        const conv_wptr wk = (conv_wptr)(cd.Wb + (ky * cd.k + kx) * cpad + ci0);
        const int wstep = cd.k * cd.k * cpad;
#pragma unroll 2
        for (int co = 0; co < cd.co; ++co) {
          double x[P];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const double x0 = src[co * (int)cin + base[p]];
            x[p] = v[p] ? x0 : 0.0;
          }
          const conv_wptr wq = wk + co * wstep;
#pragma unroll
          for (int q = 0; q < CB; ++q) {
            const double wv = wq[q];
#pragma unroll
            for (int p = 0; p < P; ++p) acc[p][q] += x[p] * wv;
          }
        }
      }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (live[p]) {
#pragma unroll
        for (int q = 0; q < CB; ++q) {
          const int ci = ci0 + q;
          if (ci < cd.ci) {
            const int c = (ci * cd.hi + iy[p]) * cd.wi + ix[p];
            const auto pre = epi.load(w, r, c);
            epi.apply(w, pre, r, c, acc[p][q], sums);
          }
        }
      }
    }
  }
  conv_row_sums<NS>(sums, sred, part, r, ntiles);
}

// Forward convolution of each row (adjoint): out (co, oy, ox) =
// sum over ci and taps of in (ci, oy*s - p + ky, ox*s - p + kx) * W (co, ci, ky, kx).
template <class Epi, int CB, bool STAGE, int P>
__global__ __launch_bounds__(256) void k_convf(int R, ConvDesc cd, const double* __restrict__ in,
                                               Epi epi, double* __restrict__ part, int ntiles) {
  extern __shared__ double srow[];
  __shared__ double sred[4 * NSUM_MAX];
  constexpr int NS = Epi::NSUM;
  constexpr int CH = 64 * P;  // positions per task
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t cin = (size_t)cd.hi * cd.wi;
  const double* row = in + (size_t)r * cd.ci * cin;
  if constexpr (STAGE) conv_stage(srow, row, (int)(cd.ci * cin));
  const double* src = STAGE ? srow : row;
  const int cpad = cd.pfp;
  const int nblk = (cd.co + CB - 1) / CB;
  const int npos = cd.ho * cd.wo, nchunk = (npos + CH - 1) / CH;
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
  for (int task = wave; task < nblk * nchunk; task += 4) {
    const int blk = task / nchunk, chunk = task % nchunk;
    bool live[P];
    int oy[P], ox[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int pos = chunk * CH + 64 * p + lane;
      live[p] = pos < npos;
      oy[p] = live[p] ? pos / cd.wo : 0;
      ox[p] = live[p] ? pos % cd.wo : 0;
    }
    const int co0 = blk * CB;
    double acc[P][CB];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < CB; ++q) acc[p][q] = 0.0;
    for (int ky = 0; ky < cd.k; ++ky) {
      for (int kx = 0; kx < cd.k; ++kx) {
        int base[P];
        bool v[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const int iy = oy[p] * cd.s - cd.p + ky, ix = ox[p] * cd.s - cd.p + kx;
          v[p] = live[p] && iy >= 0 && iy < cd.hi && ix >= 0 && ix < cd.wi;
          base[p] = v[p] ? iy * cd.wi + ix : 0;
        }
        const conv_wptr wk = (conv_wptr)(cd.Wf + (ky * cd.k + kx) * cpad + co0);
        const int wstep = cd.k * cd.k * cpad;
#pragma unroll 2
        for (int ci = 0; ci < cd.ci; ++ci) {
          double x[P];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const double x0 = src[ci * (int)cin + base[p]];
            x[p] = v[p] ? x0 : 0.0;
          }
          const conv_wptr wq = wk + ci * wstep;
#pragma unroll
          for (int q = 0; q < CB; ++q) {
            const double wv = wq[q];
#pragma unroll
            for (int p = 0; p < P; ++p) acc[p][q] += x[p] * wv;
          }
        }
      }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (live[p]) {
#pragma unroll
        for (int q = 0; q < CB; ++q) {
          const int co = co0 + q;
          if (co < cd.co) {
            const int c = (co * cd.ho + oy[p]) * cd.wo + ox[p];
            const auto pre = epi.load(w, r, c);
            epi.apply(w, pre, r, c, acc[p][q], sums);
          }
        }
      }
    }
  }
  conv_row_sums<NS>(sums, sred, part, r, ntiles);
}

// Matrix-core forward convolution of one row per workgroup, as an implicit
// GEMM  D[co, pos] = sum_(tap, ci) W[co, ci, tap] X[ci, pos + tap]  (the
// adjoint's convolution; an autotuner variant beside the vector kernel).
// The row X is staged once in LDS with a zero border wide enough that every
// tap reads inside it, so no load is masked (channels padded to 16, the
// channel stride padded to 16 mod 32 doubles so that a fragment's four lane
// groups read disjoint LDS banks); the kernel comes as pre-laid-out
// A-fragments (coalesced 512-byte loads, four issued together, each shared
// by NQ column tiles).  A wave owns a 16-row tile of output channels and NQ
// 16-column tiles of positions: lane L feeds B[L/16][L%16] = X[channel group
// + L/16, position L%16 of the tile] and receives D[L/16 + 4v][L%16].  The
// contraction accumulates every output in the same order as the vector
// kernel (tap-major, then input channel), so the two give identical results.
template <class Epi, int NQ>
__global__ __launch_bounds__(256, 4) void k_convf_mfma(int R, ConvDesc cd, const double* __restrict__ in,
                                                       Epi epi) {
  extern __shared__ double xs[];
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lk = lane >> 4, lc = lane & 15;
  const int H = cd.hi, W = cd.wi, PT = cd.fPT, HP = cd.fHP, WP = cd.fWP, plane = cd.fPL;
  {
    const double* row = in + (size_t)r * cd.ci * H * W;
    const int nst = cd.ci16 * plane;
    for (int i = threadIdx.x; i < nst; i += 256) {
      const int c = i / plane, o = i % plane, y = o / WP, x = o % WP;
      const int yy = y - PT, xx = x - PT;
      double v = 0.0;
      if (c < cd.ci && y < HP && yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = row[((size_t)c * H + yy) * W + xx];
      xs[i] = v;
    }
  }
  __syncthreads();
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
  const int MT = (cd.co + 15) / 16;
  const int CG = cd.ci16 / 4;  // channel groups of 4, a multiple of 4
  const int npos = cd.ho * cd.wo;
  const int NG = ((npos + 15) / 16 + NQ - 1) / NQ;
  // work units: (row tile, NQ column tiles); column tiles past the last
  // position compute clamped copies that are not stored
  for (int u = wave; u < MT * NG; u += 4) {
    const int mt = u / NG, nt0 = (u % NG) * NQ;
    int pb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int pos = (nt0 + q) * 16 + lc;
      pos = pos < npos ? pos : npos - 1;
      pb[q] = lk * plane + (pos / cd.wo * cd.s) * WP + (pos % cd.wo) * cd.s;
    }
    d4_t acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};
    const double* Ab = cd.Af + (size_t)mt * 64 + lane;
    const size_t astep = (size_t)MT * 64;
    for (int t = 0; t < cd.k * cd.k; ++t) {
      const int toff = (t / cd.k) * WP + t % cd.k;
      const double* At_ = Ab + (size_t)t * CG * astep;
      for (int g0 = 0; g0 < CG; g0 += 4) {
        double af[4], bf[4][NQ];
#pragma unroll
        for (int j = 0; j < 4; ++j) af[j] = At_[(size_t)(g0 + j) * astep];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int q = 0; q < NQ; ++q) bf[j][q] = xs[pb[q] + (g0 + j) * 4 * plane + toff];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[j], bf[j][q], acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int pos = (nt0 + q) * 16 + lc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ch = mt * 16 + lk + 4 * v;
        if (ch < cd.co && pos < npos) {
          const int c = ch * npos + pos;
          const auto pre = epi.load(w, r, c);
          epi.apply(w, pre, r, c, acc[q][v], sums);
        }
      }
    }
  }
}

template <class Epi>
void launch_convf_mfma(int R, const ConvDesc& cd, const double* in, Epi epi, hipStream_t s) {
  static_assert(Epi::NSUM == 0, "forward convolution: no row sums");
  const size_t lds = (size_t)cd.ci16 * cd.fPL * 8;
  const int MT = (cd.co + 15) / 16, NT = (cd.ho * cd.wo + 15) / 16;
  // four column tiles per unit unless that leaves a wave without work
  if (MT * ((NT + 3) / 4) >= 4)
    hipLaunchKernelGGL((k_convf_mfma<Epi, 4>), dim3(R), dim3(256), lds, s, R, cd, in, epi);
  else
    hipLaunchKernelGGL((k_convf_mfma<Epi, 2>), dim3(R), dim3(256), lds, s, R, cd, in, epi);
}

// Channel block of a convolution: the largest of 16, 8, 4 that still gives
// every wave of a row a task (fewer channels: the smallest block covering them).
inline int conv_block(int ch, int tasks_per_block) {
  int cb = 16;
  while (cb > 4 && ((ch + cb - 1) / cb) * tasks_per_block < 4) cb >>= 1;
  if (ch <= 4) cb = 4;
  else if (ch <= 8 && cb > 8) cb = 8;
  return cb;
}

// Positions per lane of a direct convolution: 2 where a block's positions
// fill at least two full chunks of 64 per task and the accumulators stay
// within 32 doubles, else 1 (blocks of one position each task would leave
// lanes idle).  `per_blk64` counts a block's tasks at one position per lane.
inline int conv_positions(int cb, int nblk, int npos_min, int per_blk64) {
  if (cb * 2 <= 32 && npos_min >= 128 && nblk * ((per_blk64 + 1) / 2) >= 4) return 2;
  return 1;
}

template <class Epi, int CB, int P>
void launch_convt_p(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                    hipStream_t s) {
  const int n = cd.co * cd.ho * cd.wo;
  if (n <= CONV_STAGE_MAX)
    hipLaunchKernelGGL((k_convt<Epi, CB, true, P>), dim3(R), dim3(256), (size_t)n * 8, s, R, cd, in,
                       epi, part, ntiles);
  else
    hipLaunchKernelGGL((k_convt<Epi, CB, false, P>), dim3(R), dim3(256), 0, s, R, cd, in, epi, part,
                       ntiles);
}

// variant 0: positions per lane by conv_positions; 1, 2, 3: one, two, four.
template <class Epi, int CB>
void launch_convt_cb(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant) {
  // smallest stride-parity class and the tasks of a block at one position per lane
  int per_blk = 0, cls_min = 1 << 30;
  for (int cy = 0; cy < cd.s; ++cy)
    for (int cx = 0; cx < cd.s; ++cx) {
      const int ncls = ((cd.hi - cy + cd.s - 1) / cd.s) * ((cd.wi - cx + cd.s - 1) / cd.s);
      per_blk += (ncls + 63) / 64;
      cls_min = std::min(cls_min, ncls);
    }
  const int P = variant == 1 ? 1 : variant == 2 ? 2 : variant == 3 ? 4
                                  : conv_positions(CB, (cd.ci + CB - 1) / CB, cls_min, per_blk);
  if (P == 4)
    launch_convt_p<Epi, CB, 4>(R, cd, in, epi, part, ntiles, s);
  else if (P == 2)
    launch_convt_p<Epi, CB, 2>(R, cd, in, epi, part, ntiles, s);
  else
    launch_convt_p<Epi, CB, 1>(R, cd, in, epi, part, ntiles, s);
}

template <class Epi, int CB, int P>
void launch_convf_p(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                    hipStream_t s) {
  const int n = cd.ci * cd.hi * cd.wi;
  if (n <= CONV_STAGE_MAX)
    hipLaunchKernelGGL((k_convf<Epi, CB, true, P>), dim3(R), dim3(256), (size_t)n * 8, s, R, cd, in,
                       epi, part, ntiles);
  else
    hipLaunchKernelGGL((k_convf<Epi, CB, false, P>), dim3(R), dim3(256), 0, s, R, cd, in, epi, part,
                       ntiles);
}

template <class Epi, int CB>
void launch_convf_cb(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int P = 0) {
  const int npos = cd.ho * cd.wo;
  if (P == 0) P = conv_positions(CB, (cd.co + CB - 1) / CB, npos, (npos + 63) / 64);
  if (P == 4)
    launch_convf_p<Epi, CB, 4>(R, cd, in, epi, part, ntiles, s);
  else if (P == 2)
    launch_convf_p<Epi, CB, 2>(R, cd, in, epi, part, ntiles, s);
  else
    launch_convf_p<Epi, CB, 1>(R, cd, in, epi, part, ntiles, s);
}

// Transposed convolution; variant (autotuner) 0: positions per lane by the
// shape heuristic, 1/2/3: one, two or four positions per lane.  Every variant
// accumulates each output in the same order.
template <class Epi>
hipError_t run_convt(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant = 0) {
  if (R <= 0) return hipSuccess;
  int per_blk = 0;
  for (int cy = 0; cy < cd.s; ++cy)
    for (int cx = 0; cx < cd.s; ++cx)
      per_blk += (((cd.hi - cy + cd.s - 1) / cd.s) * ((cd.wi - cx + cd.s - 1) / cd.s) + 63) / 64;
  switch (conv_block(cd.ci, per_blk)) {
    case 4: launch_convt_cb<Epi, 4>(R, cd, in, epi, part, ntiles, s, variant); break;
    case 8: launch_convt_cb<Epi, 8>(R, cd, in, epi, part, ntiles, s, variant); break;
    default: launch_convt_cb<Epi, 16>(R, cd, in, epi, part, ntiles, s, variant); break;
  }
  return hipGetLastError();
}

// variant: 0 the vector kernel with the block size of conv_block, 1/2/3
// with blocks of 4/8/16 channels (positions per lane by shape), 4/5 blocks
// of 8/16 channels with four positions per lane, 6 the matrix-core kernel
// (where the layer has one).  The forward convolution has no row sums and
// every variant accumulates each output in the same order, so the choice
// changes no result.
template <class Epi>
hipError_t run_convf(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant = 0) {
  if (R <= 0) return hipSuccess;
  if (variant == 6 && cd.mf) {
    launch_convf_mfma(R, cd, in, epi, s);
    return hipGetLastError();
  }
  const int cb = variant == 1 ? 4 : (variant == 2 || variant == 4) ? 8
                                  : (variant == 3 || variant == 5) ? 16
                                                                   : conv_block(cd.co, (cd.ho * cd.wo + 63) / 64);
  const int P = variant >= 4 ? 4 : 0;
  switch (cb) {
    case 4: launch_convf_cb<Epi, 4>(R, cd, in, epi, part, ntiles, s, P); break;
    case 8: launch_convf_cb<Epi, 8>(R, cd, in, epi, part, ntiles, s, P); break;
    default: launch_convf_cb<Epi, 16>(R, cd, in, epi, part, ntiles, s, P); break;
  }
  return hipGetLastError();
}

// Plane re-concretization of a batch whose boxes belong to several
// properties, each with its own packed plane matrix: a row tile is computed
// once per property present in it (in increasing order; one pass when the
// boxes are grouped by property), with that property's matrix, and each pass
// writes only its own rows.
__device__ __forceinline__ int tile_next_prop(const CvProps& props, int m0, int rows, int after) {
  const int lane = threadIdx.x & 63;
  int best = props.P;
  for (int i = lane; i < rows; i += 64) {
    const int q = prop_index(props, m0 + i);
    if (q > after && q < best) best = q;
  }
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_xor(best, d);
    best = o < best ? o : best;
  }
  return __builtin_amdgcn_readfirstlane(best);
}

template <class T, int OCC>
__global__ __launch_bounds__(256, OCC) void k_gemm_planes(int B, int n0, LoadBox la, CvProps props,
                                                          int Nh, float* l, float* u, int ntiles) {
  int tm, tn;
  tile_of(ntiles, tm, tn);
  const int m0 = tm * T::BM, c0 = tn * T::BN;
  const int rows = min(T::BM, B - m0);
  for (int p = tile_next_prop(props, m0, rows, -1); p < props.P;
       p = tile_next_prop(props, m0, rows, p)) {
    const RootDev& rd = props.tab[p];
    const int N = 2 * rd.U;
    if (c0 >= N) continue;
    EpiPlanes<true> e{rd.U, Nh, rd.cP, rd.eP, rd.uidx, rd.l0, rd.u0, l, u, props, p};
    gemm_tile<T>(m0, c0, B, 2 * n0, N, la, rd.P, N, e, nullptr, 1, 0);
  }
}

template <class T = TileDefault, int OCC = 2, class LoadA, class Epi>
hipError_t run_gemm(int R, int K, int N, LoadA la, const float* Bm, int ldb, Epi epi,
                    double* part, hipStream_t s) {
  if (R <= 0 || N <= 0) return hipSuccess;
  const int nt = (N + T::BN - 1) / T::BN;
  const long long nblk = (long long)((R + T::BM - 1) / T::BM) * nt;
  hipLaunchKernelGGL((k_gemm<T, OCC, LoadA, Epi>), dim3((unsigned)nblk), dim3(256), 0, s, R, K, N,
                     la, Bm, ldb, epi, part, nt);
  return hipGetLastError();
}

// Tile variants the autotuner chooses among for the backward and adjoint
// GEMMs.  The backward ones have 128 columns (the row-sum partials' layout);
// the adjoint may also take 256.  All accumulate every element over K in the
// same order, so they give identical results.
template <class LoadA, class Epi>
hipError_t run_gemm_v(int variant, int R, int K, int N, LoadA la, const float* Bm, int ldb,
                      Epi epi, double* part, hipStream_t s) {
  switch (variant) {
    case 1: return run_gemm<Tile<64, 128>, 2>(R, K, N, la, Bm, ldb, epi, part, s);
    case 2: return run_gemm<Tile<128, 128>, 1>(R, K, N, la, Bm, ldb, epi, part, s);
    case 3:  // 256 columns: each row of A read once at N = 256 (no row sums to lay out)
      if constexpr (Epi::NSUM == 0) return run_gemm<Tile<32, 256>, 2>(R, K, N, la, Bm, ldb, epi, part, s);
      return hipErrorInvalidValue;
    default: return run_gemm<TileDefault, 2>(R, K, N, la, Bm, ldb, epi, part, s);
  }
}

}  // namespace

int gemm_ntiles(int N) { return (N + TileDefault::BN - 1) / TileDefault::BN; }

hipError_t launch_gemm_relax(int R, int K, int N, const double* Om, const float* W,
                             const ConvDesc* conv, int M, int Nh,
                             int off, const float* lz, const float* uz, const float* alpha,
                             double alpha_def, const float* bprev, CvProps props, int layer,
                             double* Om_out, float* trace, double* part, int variant,
                             hipStream_t s) {
  if (props.host) {  // one property: its error weight for every row
    EpiRelax<false> e{M, Nh, off, lz, uz, alpha, alpha_def, bprev, props.host->wrel[layer], props,
                      layer, Om_out, N, trace};
    if (conv) return run_convt(R, *conv, Om, e, part, gemm_ntiles(N), s, variant);
    return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, e, part, s);
  }
  EpiRelax<true> e{M, Nh, off, lz, uz, alpha, alpha_def, bprev, nullptr, props, layer, Om_out, N,
                   trace};
  if (conv) return run_convt(R, *conv, Om, e, part, gemm_ntiles(N), s, variant);
  return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, e, part, s);
}

hipError_t launch_gemm_final(int R, int K, int N, const double* Om, const float* W,
                             const ConvDesc* conv, int M,
                             const float* lo, const float* hi, CvProps props, double* Ax,
                             float* A_out, double* part, int variant, hipStream_t s) {
  if (props.host) {
    EpiFinal<false> e{M, N, lo, hi, props.host->X0, props, Ax, A_out};
    if (conv) return run_convt(R, *conv, Om, e, part, gemm_ntiles(N), s, variant);
    return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, e, part, s);
  }
  EpiFinal<true> e{M, N, lo, hi, nullptr, props, Ax, A_out};
  if (conv) return run_convt(R, *conv, Om, e, part, gemm_ntiles(N), s, variant);
  return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, e, part, s);
}

hipError_t launch_gemm_planes(int B, int n0, int Umax, const float* lo, const float* hi,
                              CvProps props, int Nh, float* l, float* u, hipStream_t s) {
  if (B <= 0 || Umax <= 0) return hipSuccess;
  if (props.host) {  // one property: the plain tiled GEMM with its plane matrix
    const RootDev& rd = *props.host;
    EpiPlanes<false> e{rd.U, Nh, rd.cP, rd.eP, rd.uidx, rd.l0, rd.u0, l, u, props, 0};
    return run_gemm<TilePlanes>(B, 2 * n0, 2 * rd.U, LoadBox{lo, hi, n0}, rd.P, 2 * rd.U, e,
                                nullptr, s);
  }
  const int nt = (2 * Umax + TilePlanes::BN - 1) / TilePlanes::BN;
  const long long nblk = (long long)((B + TilePlanes::BM - 1) / TilePlanes::BM) * nt;
  hipLaunchKernelGGL((k_gemm_planes<TilePlanes, 2>), dim3((unsigned)nblk), dim3(256), 0, s, B, n0,
                     LoadBox{lo, hi, n0}, props, Nh, l, u, nt);
  return hipGetLastError();
}

hipError_t launch_gemm_adjoint(int R, int K, int N, const double* Abar, const float* Wt,
                               const ConvDesc* conv, const float* b, int M, int Nh, int off, const float* lz,
                               const float* uz,
                               float* alpha, const float* alpha_in, double alpha_def,
                               const float* trace, const uint8_t* infeasible, float* grad,
                               float* adam_m, float* adam_v, double lr, double b1, double b2,
                               double eps, int step, bool fresh, double* Psibar_out, int variant,
                               hipStream_t s) {
  const double bc1 = 1.0 - pow(b1, (double)step), bc2 = 1.0 - pow(b2, (double)step);
  EpiAdj e{M, Nh, off, b, lz, uz, alpha, alpha_def, trace, infeasible, grad, adam_m, adam_v,
           lr, b1, b2, eps, bc1, bc2, Psibar_out, N, alpha_in, fresh};
  if (conv) return run_convf(R, *conv, Abar, e, nullptr, 1, s, variant);
  return run_gemm_v(variant, R, K, N, LoadF64{Abar, K}, Wt, N, e, nullptr, s);
}
