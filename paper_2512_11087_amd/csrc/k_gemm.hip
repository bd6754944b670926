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
// load_in (HAS_IN): the same for a row and chunk known to lie inside, with no
// test (fast_ok: the loader's own layout allows it).
struct LoadF64 {
  const double* p;
  int ld;
  static constexpr bool HAS_IN = true;
  __device__ __forceinline__ bool fast_ok() const { return (ld & 1) == 0; }
  template <int NV>
  __device__ __forceinline__ void load_in(int r, int k, double (&v)[NV]) const {
    const double2* q = reinterpret_cast<const double2*>(p + (size_t)r * ld + k);
#pragma unroll
    for (int t = 0; t < NV / 2; ++t) {
      const double2 x = q[t];
      v[2 * t] = x.x;
      v[2 * t + 1] = x.y;
    }
  }
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
  // no untested copy of the main loop for this loader (a second loop copy
  // costs the plane re-concretization a wave per SIMD); load_in exists only
  // so that the shared loop compiles
  static constexpr bool HAS_IN = false;
  template <int NV>
  __device__ __forceinline__ void load_in(int r, int k, double (&v)[NV]) const {
    load<NV>(r, k, 0x7fffffff, 0x7fffffff, v);
  }
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
  // A tile inside the matrix (every row, column and K chunk in range) runs a
  // copy of the main loop whose operand loads have no per-lane test: one
  // uniform branch per tile instead of masked branches around every load.
  auto main_loop = [&](auto inside) {
    constexpr bool IN = decltype(inside)::value;
    auto fetch_c = [&](int k0) {
      if constexpr (IN) {
        la.template load_in<APT>(m0 + ar, k0 + akq, pa);
        const float4* q = reinterpret_cast<const float4*>(Bm + (size_t)(k0 + bk) * ldb + n0 + bc0);
#pragma unroll
        for (int t = 0; t < BPT / 4; ++t) {
          const float4 x = q[t];
          pb[4 * t] = x.x; pb[4 * t + 1] = x.y; pb[4 * t + 2] = x.z; pb[4 * t + 3] = x.w;
        }
      } else {
        fetch(k0);
      }
    };
    fetch_c(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      const int buf = c & 1;
      if (c + 1 < nch) fetch_c((c + 1) * GBK);
#pragma unroll
      for (int kk = 0; kk < GBK; kk += 4) {
        double af[MI], bf[NI];
        const int kr = kk + (lane >> 4);
#pragma unroll
        for (int i = 0; i < MI; ++i) af[i] = sA[buf][kr * SA_LD + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < NI; ++j) bf[j] = (double)sB[buf][kr * SB_LD + wave * WN + j * 16 + (lane & 15)];
        if (IN || nblk == NI) {  // full tile: straight-line MFMA issue
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
  };

  // Epilogue, in groups of VGROUP accumulator rows: all global loads of a
  // group are issued first (Epi::load), then the group is computed and
  // stored (Epi::apply), so load latency is paid once per group rather than
  // once per element (the stores could otherwise alias later loads).
  constexpr int NS = Epi::NSUM;
  constexpr int VG = Epi::VGROUP;
  // Inside a tile that lies in the matrix every element is in range; the
  // epilogues that gain from it (Epi::UNGUARDED_INSIDE) then run without the
  // per-element tests.
  auto epilogue = [&](auto inside) {
  constexpr bool IN = decltype(inside)::value && Epi::UNGUARDED_INSIDE;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int v0 = 0; v0 < 4; v0 += VG) {
      // (FENCE_GROUPS: each group's loads stay in the group, which bounds the
      // registers the epilogue holds)
      if constexpr (Epi::FENCE_GROUPS) __builtin_amdgcn_sched_barrier(0);
      typename Epi::Row rw[VG];
      typename Epi::Pre pre[VG][NI];
#pragma unroll
      for (int dv = 0; dv < VG; ++dv) {
        const int r = m0 + i * 16 + (lane >> 4) + 4 * (v0 + dv);
        rw[dv] = epi.row(IN || r < R ? r : R - 1);
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          const int c = n0 + wave * WN + j * 16 + (lane & 15);
          if (IN || (r < R && j < nblk && c < N)) pre[dv][j] = epi.load(rw[dv], r, c);
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
          if (IN || (r < R && j < nblk && c < N)) epi.apply(rw[dv], pre[dv][j], r, c, acc[i][j][v0 + dv], sums);
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
  };
  if constexpr (LoadA::HAS_IN) {
    const bool in = m0 + GBM <= R && n0 + GBN <= N && K > 0 && K % GBK == 0 && la.fast_ok() && (ldb & 3) == 0;
    if (in)
      main_loop(std::true_type{});
    else
      main_loop(std::false_type{});
    if constexpr (Epi::UNGUARDED_INSIDE) {
      if (in)
        epilogue(std::true_type{});
      else
        epilogue(std::false_type{});
    } else {
      epilogue(std::false_type{});
    }
  } else {
    main_loop(std::false_type{});
    epilogue(std::false_type{});
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
// FULL: slopes read and the trace written (the backward pass of a slope
// step), fixed at compile time; otherwise tested per call.
template <bool MULTI, bool FULL = false>
struct EpiRelax {
  static constexpr int NSUM = 3;
  // groups of two rows: the unguarded form then fits 5 waves per SIMD
  // (84 VGPRs against 100 with four; 0.421 -> 0.414 ms at 784-256x6)
  static constexpr int VGROUP = 2;
  static constexpr bool UNGUARDED_INSIDE = true;
  static constexpr bool FENCE_GROUPS = false;
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
    return Pre{w.l[j], w.u[j], (FULL || alpha) ? alpha[w.ri + j] : (float)alpha_def};
  }
  __device__ __forceinline__ void apply(const Row& w, const Pre& p, int r, int j, double psi,
                                        double* s) const {
    const size_t ri = w.ri + j;
    const double al = (FULL || alpha) ? (double)p.al : alpha_def;
    const Relax rl = relax_apply(psi, relax_line(p.l, p.u), al);
    const double om = psi * rl.s;
    Om[(size_t)r * ldo + j] = om;
    if (FULL || trace) trace[ri] = trace32(psi);
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
  static constexpr bool UNGUARDED_INSIDE = true;
  static constexpr bool FENCE_GROUPS = false;
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
  static constexpr bool UNGUARDED_INSIDE = false;
  static constexpr bool FENCE_GROUPS = false;
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
// FULL: the slope step after the first -- slopes read, Adam's moments read
// and the step taken -- fixed at compile time; otherwise these are tested
// per call (every other use, the convolutions included).  Both forms compute
// the same values.
template <bool FULL>
struct EpiAdjT {
  static constexpr int NSUM = 0;
  static constexpr int VGROUP = 2;
  // unguarded only with the groups fenced: the compiler otherwise hoists the
  // later groups' loads and takes 16 more VGPRs (5 -> 4 waves per SIMD;
  // measured 0.624 -> 0.663 ms at the 784-256x6 shapes, 0.607 -> 0.587 ms
  // fenced)
  static constexpr bool UNGUARDED_INSIDE = true;
  static constexpr bool FENCE_GROUPS = true;
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
  __device__ __forceinline__ bool reads_alpha() const { return FULL || alpha_in != nullptr; }
  __device__ __forceinline__ bool steps() const { return FULL || (lr > 0.0 && alpha); }
  __device__ __forceinline__ Pre load(const Row& w, int, int j) const {
    const size_t ri = w.ri + j;
    const bool adam = FULL || (lr > 0.0 && alpha && !fresh);
    return Pre{w.l[j], w.u[j], trace[ri], reads_alpha() ? alpha_in[ri] : (float)alpha_def,
               adam ? am[ri] : 0.0f, adam ? av[ri] : 0.0f};
  }
  __device__ __forceinline__ void apply(const Row& w, const Pre& p, int r, int j, double acc,
                                        double*) const {
    const double om = acc + (double)bias[j];
    const size_t ri = w.ri + j;
    const double al = reads_alpha() ? (double)p.al : alpha_def;
    const double psi = (double)p.psi;
    const Relax rl = relax_apply(psi, relax_line(p.l, p.u), al);
    const bool dead = w.dead;
    const double g = (rl.lower && !dead) ? om * psi : 0.0;
    if (out) out[(size_t)r * ldo + j] = om * rl.s + rl.t;
    if (grad) grad[ri] = (float)g;
    if (steps()) {
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

typedef EpiAdjT<false> EpiAdj;

// ------------------------------------------------------------ convolutions
// The backward pass through a conv layer is a transposed convolution of each
// row of Omega (and the adjoint a forward convolution), computed directly
// rather than as a product with the layer's dense matrix, with the same
// fused epilogues as the GEMMs.
//
// A workgroup takes one row, a band of output rows at full width (a tile)
// and four tasks, one per wave; a task is a set of output channels times a
// group of output positions.  In the transposed convolution the positions of
// a task share one stride-parity class (iy = s a + cy, ix = s b + cx): only
// the taps ky = cy + p (mod s) reach a class, and its t-th one reaches input
// row oy = a + dy - t, so the taps are uniform over the wave and only the
// ~k^2/s^2 of the class are visited.  The input band the tile reads (halo
// included, zero outside the map) is staged in LDS, CC input channels at a
// time, so every tap reads LDS.
//
// Layers with 16 or more output channels run on the float64 matrix cores
// (v_mfma_f64_16x16x4_f64) as an implicit GEMM per task, D[out channel,
// position] = sum over (input channel, tap) of W X: the MFMA's k runs over
// four input channels at one tap, the B fragment is gathered from the band
// and the A fragment (the kernel slice) is read from the L2-resident
// weights.  The contraction order is: groups of four input channels, then
// taps, then the group's channels.  Narrower layers use the float64 vector
// units: a wave takes CB output channels times 64 P positions, each band
// value read feeds CB FMAs whose weights are wave-uniform (scalar loads);
// order: input channels, then taps.  The staging depth CC (an autotuner
// variant) changes no result.

// Kernel weights are read through the constant address space: their
// addresses are wave-uniform and nothing in these kernels writes them, so
// they come in by scalar loads and feed the FMAs from SGPRs.
typedef const __attribute__((address_space(4))) double* conv_wptr;

// Geometry of one tiled convolution launch (computed on the host).
struct ConvPlan {
  bool mf;            // matrix-core kernel (else vector)
  int P, CB;          // vector kernel: positions per lane, channels per block
  int MT, NQ;         // matrix-core kernel: 16-channel row tiles and 16-position column tiles per task
  int CC;             // input channels per staged chunk (matrix-core: a multiple of 4)
  int TA;             // class rows (forward: output rows) per tile
  int nT;             // tiles per row
  int nch;            // position groups per class and tile
  int nblk;           // channel blocks
  int ntask;          // tasks per tile
  int wgt;            // workgroups per tile
  int SH, SW, plane;  // staged band: rows, columns, doubles per channel
  int dmin;           // transposed: first band row (relative to the tile) and column, input coordinates
  float inv_sh;       // 1 / SH (band row -> channel in the staging loop)
};

// Largest staged band, in doubles: 64 KiB of LDS per workgroup.
constexpr int CONV_BAND_MAX = 8192;

// Stage channels [c0, c0 + nc) of a row (maps Hs x Ws; channels >= nin
// read as zero) over band rows [R0, R0 + SH) and columns [C0, C0 + SW)
// into LDS, channel stride `plane`, zero outside the map.  Thread i takes
// column i mod SW of band rows i / SW, i / SW + 256 / SW, ... (SW <= 256),
// four rows' loads issued before their stores; a load outside the map
// reads the row's first value and is replaced by zero (no branch per load).
__device__ __forceinline__ void conv_band(double* __restrict__ band, const double* __restrict__ src,
                                          int c0, int nc, int nin, int Hs, int Ws, int R0, int C0,
                                          int SH, int SW, int plane, float inv_sh) {
  const int rpp = 256 / SW;
  const int r0 = threadIdx.x / SW;
  if (r0 >= rpp) return;
  const int x = threadIdx.x - r0 * SW;
  const int gx = C0 + x;
  const bool xok = gx >= 0 && gx < Ws;
  const int nrow = nc * SH;
  for (int rb = r0; rb < nrow; rb += 4 * rpp) {
    double v[4];
    int d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = rb + u * rpp;
      // r / SH exactly: (r + 1/2) / SH is at least 1 / (2 SH) from an integer
      const int c = (int)(((float)r + 0.5f) * inv_sh);
      const int y = r - c * SH;
      const int gy = R0 + y;
      const bool ok = r < nrow && xok && gy >= 0 && gy < Hs && c0 + c < nin;
      const size_t gi = ok ? ((size_t)(c0 + c) * Hs + gy) * Ws + gx : 0;
      const double val = src[gi];
      v[u] = ok ? val : 0.0;
      d[u] = r < nrow ? c * plane + y * SW + x : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (d[u] >= 0) band[d[u]] = v[u];
  }
}

// Row sums of a workgroup into partial slot `slot` of the row (the GEMM
// epilogues' layout: ntiles slots per row, summed in order afterwards); the
// workgroup of slot 0 zeroes the slots past the row's last workgroup.
template <int NS>
__device__ __forceinline__ void conv_row_sums(double (&sums)[NSUM_MAX], double* sred, double* part,
                                              int r, int ntiles, int slot, int nslots) {
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
      part[((size_t)r * ntiles + slot) * NS + q] =
          (sred[q] + sred[NSUM_MAX + q]) + (sred[2 * NSUM_MAX + q] + sred[3 * NSUM_MAX + q]);
    }
    if (slot == 0)
      for (int i = threadIdx.x; i < (ntiles - nslots) * NS; i += 256)
        part[((size_t)r * ntiles + nslots) * NS + i] = 0.0;
  }
}

// Workgroup -> (row, tile, workgroup of the tile): the workgroups of a row
// are consecutive on one XCD (xcd_block), so its input is fetched into one L2.
__device__ __forceinline__ void conv_wg(const ConvPlan& pl, int& r, int& slot, int& tile, int& g) {
  const int per_row = pl.nT * pl.wgt;
  const int id = (int)xcd_block(blockIdx.x, gridDim.x);
  r = id / per_row;
  slot = id - r * per_row;
  tile = slot / pl.wgt;
  g = slot - tile * pl.wgt;
}

// Sum over n (channel, tap) pairs of a staged chunk, software-pipelined:
// the LDS inputs and scalar weights of pair j+1 are requested before the
// FMAs of pair j, so their latency overlaps those FMAs (LDS reads and scalar
// loads share one wait counter: waiting for either waits for both).  `it`
// walks the pairs in order: xoff() is the pair's offset in the band,
// wptr() its CB weights, next() moves on.
template <int CB, int P, class It>
__device__ __forceinline__ void conv_pairs(double (&acc)[P][CB], const double* __restrict__ band,
                                           const int (&base)[P], It& it, int n) {
  if (n <= 0) return;
  double xa[P], xb[P], wa[CB], wb[CB];
  auto ld = [&](double (&x)[P], double (&w)[CB]) {
    const int o = it.xoff();
    const conv_wptr wp = it.wptr();
#pragma unroll
    for (int p = 0; p < P; ++p) x[p] = band[base[p] + o];
#pragma unroll
    for (int q = 0; q < CB; ++q) w[q] = wp[q];
    it.next();
  };
  auto fm = [&](const double (&x)[P], const double (&w)[CB]) {
#pragma unroll
    for (int q = 0; q < CB; ++q)
#pragma unroll
      for (int p = 0; p < P; ++p) acc[p][q] += x[p] * w[q];
  };
  ld(xa, wa);
  for (int j = 0;;) {
    if (j + 1 < n) ld(xb, wb);
    fm(xa, wa);
    if (++j == n) break;
    if (j + 1 < n) ld(xa, wa);
    fm(xb, wb);
    if (++j == n) break;
  }
}

// Pairs of the transposed convolution: channel c of the chunk, then the
// class's taps (t, u) in order; the band offset of tap (t, u) is -(t SW + u).
struct ConvtPairs {
  const double* w0;  // weights of the chunk's first channel, block ci0
  int c, t, u, nty, ntx, SW, plane, k, s, ky0, kx0, ptp, wstep;
  __device__ __forceinline__ int xoff() const { return c * plane - (t * SW + u); }
  __device__ __forceinline__ conv_wptr wptr() const {
    return (conv_wptr)(w0 + c * wstep + ((ky0 + s * t) * k + kx0 + s * u) * ptp);
  }
  __device__ __forceinline__ void next() {
    if (++u == ntx) {
      u = 0;
      if (++t == nty) {
        t = 0;
        ++c;
      }
    }
  }
};

// Pairs of the forward convolution: channel, then taps (ky, kx) in order;
// the weights of consecutive pairs are pfp doubles apart.
struct ConvfPairs {
  const double* w;  // weights of the current pair, block co0
  int c, ky, kx, k, SW, plane, pfp;
  __device__ __forceinline__ int xoff() const { return c * plane + ky * SW + kx; }
  __device__ __forceinline__ conv_wptr wptr() const { return (conv_wptr)w; }
  __device__ __forceinline__ void next() {
    w += pfp;
    if (++kx == k) {
      kx = 0;
      if (++ky == k) {
        ky = 0;
        ++c;
      }
    }
  }
};

// Transposed convolution of each row: out (ci, iy, ix) = sum over co and the
// taps with iy + p - ky = s oy, ix + p - kx = s ox of in (co, oy, ox) W (co, ci, ky, kx).
template <class Epi, int CB, int P>
__global__ __launch_bounds__(256) void k_convt(ConvDesc cd, ConvPlan pl, const double* __restrict__ in,
                                               Epi epi, double* __restrict__ part, int ntiles) {
  extern __shared__ double band[];
  __shared__ double sred[4 * NSUM_MAX];
  constexpr int NS = Epi::NSUM;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int r, slot, tile, g;
  conv_wg(pl, r, slot, tile, g);
  const int s = cd.s, k = cd.k;
  const int A0 = tile * pl.TA;
  // the wave's task: (class, chunk, block), blocks innermost
  const int task = g * 4 + wave;
  const bool has = task < pl.ntask;
  const int blk = has ? task % pl.nblk : 0;
  const int qc = has ? task / pl.nblk : 0;
  const int chunk = qc % pl.nch, cl = qc / pl.nch;
  const int cy = cl / s, cx = cl - (cl / s) * s;
  const int ky0 = (cy + cd.p) % s, kx0 = (cx + cd.p) % s;
  const int nty = ky0 < k ? (k - ky0 + s - 1) / s : 0;
  const int ntx = kx0 < k ? (k - kx0 + s - 1) / s : 0;
  const int dy = (cy + cd.p - ky0) / s, dx = (cx + cd.p - kx0) / s;
  const int ny = (cd.hi - cy + s - 1) / s, nx = (cd.wi - cx + s - 1) / s;
  bool live[P];
  int iy[P], ix[P], base[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int idx = chunk * 64 * P + 64 * p + lane;
    int al = nx > 0 ? idx / nx : 0;
    int b = idx - al * nx;
    live[p] = has && nx > 0 && al < pl.TA && A0 + al < ny;
    if (!live[p]) al = b = 0;
    iy[p] = s * (A0 + al) + cy;
    ix[p] = s * b + cx;
    base[p] = (al + dy - pl.dmin) * pl.SW + (b + dx - pl.dmin);
  }
  const int ci0 = blk * CB;
  const double* row = in + (size_t)r * cd.co * cd.ho * cd.wo;
  double acc[P][CB];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[p][q] = 0.0;
  const int wstep = k * k * cd.ptp;
  for (int c0 = 0; c0 < cd.co; c0 += pl.CC) {
    const int nc = min(pl.CC, cd.co - c0);
    if (c0 > 0) __syncthreads();
    conv_band(band, row, c0, nc, cd.co, cd.ho, cd.wo, A0 + pl.dmin, pl.dmin, pl.SH, pl.SW, pl.plane,
              pl.inv_sh);
    __syncthreads();
    if (!has) continue;
    ConvtPairs it{cd.Wb + (size_t)c0 * wstep + ci0, 0, 0, 0, nty, ntx, pl.SW, pl.plane, k, s,
                  ky0, kx0, cd.ptp, wstep};
    conv_pairs<CB, P>(acc, band, base, it, nc * nty * ntx);
  }
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
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
  conv_row_sums<NS>(sums, sred, part, r, ntiles, slot, pl.nT * pl.wgt);
}

// Forward convolution of each row (the adjoint): out (co, oy, ox) = sum over
// ci and taps of in (ci, oy s - p + ky, ox s - p + kx) W (co, ci, ky, kx).
template <class Epi, int CB, int P>
__global__ __launch_bounds__(256) void k_convf(ConvDesc cd, ConvPlan pl, const double* __restrict__ in,
                                               Epi epi, double* __restrict__ part, int ntiles) {
  extern __shared__ double band[];
  __shared__ double sred[4 * NSUM_MAX];
  constexpr int NS = Epi::NSUM;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int r, slot, tile, g;
  conv_wg(pl, r, slot, tile, g);
  const int s = cd.s, k = cd.k;
  const int Y0 = tile * pl.TA;
  const int task = g * 4 + wave;
  const bool has = task < pl.ntask;
  const int blk = has ? task % pl.nblk : 0;
  const int chunk = has ? task / pl.nblk : 0;
  bool live[P];
  int oy[P], ox[P], base[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int idx = chunk * 64 * P + 64 * p + lane;
    int yl = idx / cd.wo;
    int x = idx - yl * cd.wo;
    live[p] = has && yl < pl.TA && Y0 + yl < cd.ho;
    if (!live[p]) yl = x = 0;
    oy[p] = Y0 + yl;
    ox[p] = x;
    base[p] = yl * s * pl.SW + x * s;
  }
  const int co0 = blk * CB;
  const double* row = in + (size_t)r * cd.ci * cd.hi * cd.wi;
  double acc[P][CB];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[p][q] = 0.0;
  const int wstep = k * k * cd.pfp;
  for (int c0 = 0; c0 < cd.ci; c0 += pl.CC) {
    const int nc = min(pl.CC, cd.ci - c0);
    if (c0 > 0) __syncthreads();
    conv_band(band, row, c0, nc, cd.ci, cd.hi, cd.wi, Y0 * s - cd.p, -cd.p, pl.SH, pl.SW, pl.plane,
              pl.inv_sh);
    __syncthreads();
    if (!has) continue;
    ConvfPairs it{cd.Wf + (size_t)c0 * wstep + co0, 0, 0, 0, k, pl.SW, pl.plane, cd.pfp};
    conv_pairs<CB, P>(acc, band, base, it, nc * k * k);
  }
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
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
  conv_row_sums<NS>(sums, sred, part, r, ntiles, slot, pl.nT * pl.wgt);
}

// Matrix-core steps over one staged chunk: n steps of (group of four input
// channels, tap), each MT x NQ MFMAs; the A and B fragments of step j+1 are
// requested before the MFMAs of step j (A by vector loads, B from LDS: two
// wait counters, so each wait covers only its own loads).  `it` walks the
// steps in order: xoff() is the step's band offset (added to each lane's
// column offset boff), woff() its offset in the lane's weight stream wl.
template <int MT, int NQ, class It>
__device__ __forceinline__ void conv_mfma_steps(d4_t (&acc)[MT][NQ], const double* __restrict__ band,
                                                const int (&boff)[NQ], const double* __restrict__ wl,
                                                It& it, int n) {
  if (n <= 0) return;
  double a0[MT], b0[NQ], a1[MT], b1[NQ];
  auto ld = [&](double (&a)[MT], double (&b)[NQ]) {
    const int xo = it.xoff();
    const double* w = wl + it.woff();
#pragma unroll
    for (int m = 0; m < MT; ++m) a[m] = w[16 * m];
#pragma unroll
    for (int q = 0; q < NQ; ++q) b[q] = band[boff[q] + xo];
    it.next();
  };
  auto mm = [&](const double (&a)[MT], const double (&b)[NQ]) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
  };
  ld(a0, b0);
  for (int j = 0;;) {
    if (j + 1 < n) ld(a1, b1);
    mm(a0, b0);
    if (++j == n) break;
    if (j + 1 < n) ld(a0, b0);
    mm(a1, b1);
    if (++j == n) break;
  }
}

// Steps of the transposed convolution: channel group g, then the class's
// taps (t, u); band offset 4 g plane - (t SW + u), weights of input channel
// 4 g + (lane / 16) at tap (ky0 + s t, kx0 + s u).
struct ConvtSteps {
  int g, t, u, nty, ntx, SW, plane, k, s, ky0, kx0, ptp;
  __device__ __forceinline__ int xoff() const { return 4 * g * plane - (t * SW + u); }
  __device__ __forceinline__ int woff() const {
    return (4 * g * k * k + (ky0 + s * t) * k + kx0 + s * u) * ptp;
  }
  __device__ __forceinline__ void next() {
    if (++u == ntx) {
      u = 0;
      if (++t == nty) {
        t = 0;
        ++g;
      }
    }
  }
};

// Steps of the forward convolution: channel group g, then taps (ky, kx).
struct ConvfSteps {
  int g, ky, kx, k, SW, plane, pfp;
  __device__ __forceinline__ int xoff() const { return 4 * g * plane + ky * SW + kx; }
  __device__ __forceinline__ int woff() const { return (4 * g * k * k + ky * k + kx) * pfp; }
  __device__ __forceinline__ void next() {
    if (++kx == k) {
      kx = 0;
      if (++ky == k) {
        ky = 0;
        ++g;
      }
    }
  }
};

// Matrix-core transposed convolution (>= 16 output channels).  A task covers
// 16 MT output channels (ci) and 16 NQ positions of one class; lane L feeds
// B[L/16][L%16] = band value of input channel 4g + L/16 for position L%16 of
// a column tile and receives D[L/16 + 4v][L%16].
template <class Epi, int MT, int NQ>
__global__ __launch_bounds__(256) void k_convt_mf(ConvDesc cd, ConvPlan pl, const double* __restrict__ in,
                                                  Epi epi, double* __restrict__ part, int ntiles) {
  extern __shared__ double band[];
  __shared__ double sred[4 * NSUM_MAX];
  constexpr int NS = Epi::NSUM;
  const int lane = threadIdx.x & 63;
  const int lk = lane >> 4, lc = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int r, slot, tile, g;
  conv_wg(pl, r, slot, tile, g);
  const int s = cd.s, k = cd.k;
  const int A0 = tile * pl.TA;
  const int task = g * 4 + wave;
  const bool has = task < pl.ntask;
  const int blk = has ? task % pl.nblk : 0;
  const int qc = has ? task / pl.nblk : 0;
  const int grp = qc % pl.nch, cl = qc / pl.nch;
  const int cy = cl / s, cx = cl - (cl / s) * s;
  const int ky0 = (cy + cd.p) % s, kx0 = (cx + cd.p) % s;
  const int nty = ky0 < k ? (k - ky0 + s - 1) / s : 0;
  const int ntx = kx0 < k ? (k - kx0 + s - 1) / s : 0;
  const int dy = (cy + cd.p - ky0) / s, dx = (cx + cd.p - kx0) / s;
  const int ny = (cd.hi - cy + s - 1) / s, nx = (cd.wi - cx + s - 1) / s;
  bool live[NQ];
  int iy[NQ], ix[NQ], boff[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = (grp * NQ + q) * 16 + lc;
    int al = nx > 0 ? idx / nx : 0;
    int b = idx - al * nx;
    live[q] = has && nx > 0 && al < pl.TA && A0 + al < ny;
    if (!live[q]) al = b = 0;
    iy[q] = s * (A0 + al) + cy;
    ix[q] = s * b + cx;
    boff[q] = lk * pl.plane + (al + dy - pl.dmin) * pl.SW + (b + dx - pl.dmin);
  }
  const int ch0 = blk * 16 * MT;
  const double* row = in + (size_t)r * cd.co * cd.ho * cd.wo;
  d4_t acc[MT][NQ];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[m][q] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < cd.co; c0 += pl.CC) {
    const int nc4 = (min(pl.CC, cd.co - c0) + 3) & ~3;
    if (c0 > 0) __syncthreads();
    conv_band(band, row, c0, nc4, cd.co, cd.ho, cd.wo, A0 + pl.dmin, pl.dmin, pl.SH, pl.SW, pl.plane,
              pl.inv_sh);
    __syncthreads();
    if (!has) continue;
    ConvtSteps it{0, 0, 0, nty, ntx, pl.SW, pl.plane, k, s, ky0, kx0, cd.ptp};
    const double* wl = cd.Wb + ((size_t)(c0 + lk) * k * k) * cd.ptp + ch0 + lc;
    conv_mfma_steps<MT, NQ>(acc, band, boff, wl, it, (nc4 / 4) * nty * ntx);
  }
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (live[q]) {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ci = ch0 + 16 * m + lk + 4 * v;
          if (ci < cd.ci) {
            const int c = (ci * cd.hi + iy[q]) * cd.wi + ix[q];
            const auto pre = epi.load(w, r, c);
            epi.apply(w, pre, r, c, acc[m][q][v], sums);
          }
        }
      }
    }
  }
  conv_row_sums<NS>(sums, sred, part, r, ntiles, slot, pl.nT * pl.wgt);
}

// Matrix-core forward convolution (>= 16 output channels): a task covers
// 16 MT output channels (co) and 16 NQ output positions of the tile.
template <class Epi, int MT, int NQ>
__global__ __launch_bounds__(256) void k_convf_mf(ConvDesc cd, ConvPlan pl, const double* __restrict__ in,
                                                  Epi epi, double* __restrict__ part, int ntiles) {
  extern __shared__ double band[];
  __shared__ double sred[4 * NSUM_MAX];
  constexpr int NS = Epi::NSUM;
  const int lane = threadIdx.x & 63;
  const int lk = lane >> 4, lc = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int r, slot, tile, g;
  conv_wg(pl, r, slot, tile, g);
  const int s = cd.s, k = cd.k;
  const int Y0 = tile * pl.TA;
  const int task = g * 4 + wave;
  const bool has = task < pl.ntask;
  const int blk = has ? task % pl.nblk : 0;
  const int grp = has ? task / pl.nblk : 0;
  bool live[NQ];
  int oy[NQ], ox[NQ], boff[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = (grp * NQ + q) * 16 + lc;
    int yl = idx / cd.wo;
    int x = idx - yl * cd.wo;
    live[q] = has && yl < pl.TA && Y0 + yl < cd.ho;
    if (!live[q]) yl = x = 0;
    oy[q] = Y0 + yl;
    ox[q] = x;
    boff[q] = lk * pl.plane + yl * s * pl.SW + x * s;
  }
  const int ch0 = blk * 16 * MT;
  const double* row = in + (size_t)r * cd.ci * cd.hi * cd.wi;
  d4_t acc[MT][NQ];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[m][q] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < cd.ci; c0 += pl.CC) {
    const int nc4 = (min(pl.CC, cd.ci - c0) + 3) & ~3;
    if (c0 > 0) __syncthreads();
    conv_band(band, row, c0, nc4, cd.ci, cd.hi, cd.wi, Y0 * s - cd.p, -cd.p, pl.SH, pl.SW, pl.plane,
              pl.inv_sh);
    __syncthreads();
    if (!has) continue;
    ConvfSteps it{0, 0, 0, k, pl.SW, pl.plane, cd.pfp};
    const double* wl = cd.Wf + ((size_t)(c0 + lk) * k * k) * cd.pfp + ch0 + lc;
    conv_mfma_steps<MT, NQ>(acc, band, boff, wl, it, (nc4 / 4) * k * k);
  }
  const auto w = epi.row(r);
  double sums[NSUM_MAX] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (live[q]) {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int co = ch0 + 16 * m + lk + 4 * v;
          if (co < cd.co) {
            const int c = (co * cd.ho + oy[q]) * cd.wo + ox[q];
            const auto pre = epi.load(w, r, c);
            epi.apply(w, pre, r, c, acc[m][q][v], sums);
          }
        }
      }
    }
  }
  conv_row_sums<NS>(sums, sred, part, r, ntiles, slot, pl.nT * pl.wgt);
}

// Whole-row convolutions, for rows whose input fits LDS (up to 64 KiB):
// one workgroup per row stages the whole input row once (no halo, no
// tiles) and its four waves take tasks = (channel block of 4/8/16, chunk
// of 64 P output positions); weights come by scalar loads; each output sums
// over its taps in order and, within a tap, over input channels in order.
// In the transposed convolution the lanes of a task share one stride-parity
// class, so a tap's divisibility by the stride is uniform; borders are
// masked per lane.  Longer rows take the tiled kernels above.
constexpr int CONV_STAGE_MAX = 8192;

// Copy one row into LDS with many loads in flight per thread.
__device__ __forceinline__ void conv_stage_row(double* __restrict__ dst, const double* __restrict__ src,
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
template <class Epi, int CB, int P>
__global__ __launch_bounds__(256) void k_convt_row(int R, ConvDesc cd, const double* __restrict__ in,
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
  conv_stage_row(srow, row, (int)(cd.co * cin));
  const double* src = srow;
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
  conv_row_sums<NS>(sums, sred, part, r, ntiles, 0, 1);
}

// Forward convolution of each row (adjoint): out (co, oy, ox) =
// sum over ci and taps of in (ci, oy*s - p + ky, ox*s - p + kx) * W (co, ci, ky, kx).
template <class Epi, int CB, int P>
__global__ __launch_bounds__(256) void k_convf_row(int R, ConvDesc cd, const double* __restrict__ in,
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
  conv_stage_row(srow, row, (int)(cd.ci * cin));
  const double* src = srow;
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
  conv_row_sums<NS>(sums, sred, part, r, ntiles, 0, 1);
}

// Channel block of a convolution: the largest of 16, 8, 4 that still gives
// every wave of a row a task (fewer channels: the smallest block covering them).
inline int conv_block_row(int ch, int tasks_per_block) {
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
inline int conv_positions_row(int cb, int nblk, int npos_min, int per_blk64) {
  if (cb * 2 <= 32 && npos_min >= 128 && nblk * ((per_blk64 + 1) / 2) >= 4) return 2;
  return 1;
}

template <class Epi, int CB, int P>
void launch_convt_row_p(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                    hipStream_t s) {
  const int n = cd.co * cd.ho * cd.wo;
  hipLaunchKernelGGL((k_convt_row<Epi, CB, P>), dim3(R), dim3(256), (size_t)n * 8, s, R, cd, in, epi,
                     part, ntiles);
}

// variant 0: positions per lane by conv_positions_row; 1, 2, 3: one, two, four.
template <class Epi, int CB>
void launch_convt_row_cb(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
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
                                  : conv_positions_row(CB, (cd.ci + CB - 1) / CB, cls_min, per_blk);
  if (P == 4)
    launch_convt_row_p<Epi, CB, 4>(R, cd, in, epi, part, ntiles, s);
  else if (P == 2)
    launch_convt_row_p<Epi, CB, 2>(R, cd, in, epi, part, ntiles, s);
  else
    launch_convt_row_p<Epi, CB, 1>(R, cd, in, epi, part, ntiles, s);
}

template <class Epi, int CB, int P>
void launch_convf_row_p(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                    hipStream_t s) {
  const int n = cd.ci * cd.hi * cd.wi;
  hipLaunchKernelGGL((k_convf_row<Epi, CB, P>), dim3(R), dim3(256), (size_t)n * 8, s, R, cd, in, epi,
                     part, ntiles);
}

template <class Epi, int CB>
void launch_convf_row_cb(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int P = 0) {
  const int npos = cd.ho * cd.wo;
  if (P == 0) P = conv_positions_row(CB, (cd.co + CB - 1) / CB, npos, (npos + 63) / 64);
  if (P == 4)
    launch_convf_row_p<Epi, CB, 4>(R, cd, in, epi, part, ntiles, s);
  else if (P == 2)
    launch_convf_row_p<Epi, CB, 2>(R, cd, in, epi, part, ntiles, s);
  else
    launch_convf_row_p<Epi, CB, 1>(R, cd, in, epi, part, ntiles, s);
}

// Transposed convolution; variant (autotuner) 0: positions per lane by the
// shape heuristic, 1/2/3: one, two or four positions per lane.  Every variant
// accumulates each output in the same order.
template <class Epi>
hipError_t run_convt_row(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant = 0) {
  if (R <= 0) return hipSuccess;
  int per_blk = 0;
  for (int cy = 0; cy < cd.s; ++cy)
    for (int cx = 0; cx < cd.s; ++cx)
      per_blk += (((cd.hi - cy + cd.s - 1) / cd.s) * ((cd.wi - cx + cd.s - 1) / cd.s) + 63) / 64;
  switch (conv_block_row(cd.ci, per_blk)) {
    case 4: launch_convt_row_cb<Epi, 4>(R, cd, in, epi, part, ntiles, s, variant); break;
    case 8: launch_convt_row_cb<Epi, 8>(R, cd, in, epi, part, ntiles, s, variant); break;
    default: launch_convt_row_cb<Epi, 16>(R, cd, in, epi, part, ntiles, s, variant); break;
  }
  return hipGetLastError();
}

// variant: 0 the block size of conv_block_row, 1/2/3 blocks of 4/8/16
// channels (positions per lane by shape), 4/5 blocks of 8/16 channels with
// four positions per lane.  The forward convolution has no row sums and
// every variant accumulates each output in the same order, so the choice
// changes no result.
template <class Epi>
hipError_t run_convf_row(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant = 0) {
  if (R <= 0) return hipSuccess;
  const int cb = variant == 1 ? 4 : (variant == 2 || variant == 4) ? 8
                                  : (variant == 3 || variant == 5) ? 16
                                                                   : conv_block_row(cd.co, (cd.ho * cd.wo + 63) / 64);
  const int P = variant >= 4 ? 4 : 0;
  switch (cb) {
    case 4: launch_convf_row_cb<Epi, 4>(R, cd, in, epi, part, ntiles, s, P); break;
    case 8: launch_convf_row_cb<Epi, 8>(R, cd, in, epi, part, ntiles, s, P); break;
    default: launch_convf_row_cb<Epi, 16>(R, cd, in, epi, part, ntiles, s, P); break;
  }
  return hipGetLastError();
}

// Channel block of the vector kernels: 4, 8 or 16 channels, the smallest
// that covers a layer of up to 8 channels, else 16.
inline int conv_block(int ch) { return ch <= 4 ? 4 : ch <= 8 ? 8 : 16; }

// Positions per lane (vector kernels): two where the (class, block) pairs of
// a row times its full chunks of 128 positions per class still give every
// wave a task, else one (each weight then feeds fewer FMAs, but no wave
// idles).
inline int conv_positions(int pairs, int npos_class) { return pairs * (npos_class / 128) >= 4 ? 2 : 1; }

// Band plane: SH x SW doubles, rounded up (matrix-core kernels) to 16 mod
// 32 doubles so that the four lane groups of a B fragment, which read four
// consecutive channels, fall on disjoint LDS banks.
inline int conv_plane(int SH, int SW, bool mf) {
  const int n = SH * SW;
  return mf ? n + ((16 - n % 32) + 32) % 32 : n;
}

// Channels staged per chunk: `cc` if given, else the most of 16, 8, 4
// (matrix cores; the vector kernels also 2, 1) whose band fits 32 KiB;
// always within the band budget, and at most the layer's channels (rounded
// up to 4 on the matrix cores).
inline int conv_depth(int cc, int plane, int nin, bool mf) {
  const int lo = mf ? 4 : 1;
  if (cc <= 0) {
    cc = 16;
    while (cc > lo && (size_t)cc * plane * 8 > 32768) cc >>= 1;
  }
  while (cc > lo && (size_t)cc * plane > CONV_BAND_MAX) cc >>= 1;
  const int cap = mf ? (nin + 3) & ~3 : nin;
  return std::max(lo, std::min(cc, cap));
}

// Tiles: class rows TA so that a tile's class holds about `target`
// positions (at least one row), groups of `per` positions per class.
inline void conv_tiles(ConvPlan& pl, int ncls, int nymax, int nxmax, int per, int target) {
  pl.TA = std::max(1, std::min(nymax, (target + nxmax - 1) / std::max(1, nxmax)));
  pl.nch = (pl.TA * nxmax + per - 1) / per;
  pl.nT = (nymax + pl.TA - 1) / pl.TA;
  pl.ntask = ncls * pl.nch * pl.nblk;
  pl.wgt = (pl.ntask + 3) / 4;
}

// Shape of a task: the matrix cores for 16 or more output channels (up to
// 64 per task; NQ = 2 column tiles unless that leaves waves idle), else the
// vector kernel's channel block and positions per lane; then the tiles.
inline void conv_shape(ConvPlan& pl, int nout, int ncls, int nymax, int nxmax) {
  pl.mf = nout >= 16;
  if (pl.mf) {
    pl.MT = std::min(4, (nout + 15) / 16);
    pl.nblk = (nout + 16 * pl.MT - 1) / (16 * pl.MT);
    pl.NQ = ncls * pl.nblk * ((nymax * nxmax) / 32) >= 4 ? 2 : 1;
    const int per = 16 * pl.NQ;
    const int want = std::max(1, (4 + ncls * pl.nblk - 1) / (ncls * pl.nblk));
    conv_tiles(pl, ncls, nymax, nxmax, per, std::max(64, want * per));
  } else {
    pl.CB = conv_block(nout);
    pl.nblk = (nout + pl.CB - 1) / pl.CB;
    pl.P = conv_positions(ncls * pl.nblk, nymax * nxmax);
    const int per = 64 * pl.P;
    const int want = std::max(1, (4 + ncls * pl.nblk - 1) / (ncls * pl.nblk));
    conv_tiles(pl, ncls, nymax, nxmax, per, want * per);
  }
}

// Plan of a transposed convolution (output: ci x hi x wi; input: co x ho x wo).
inline ConvPlan plan_convt(const ConvDesc& cd, int cc) {
  ConvPlan pl{};
  const int s = cd.s, k = cd.k;
  const int nymax = (cd.hi + s - 1) / s, nxmax = (cd.wi + s - 1) / s;
  conv_shape(pl, cd.ci, s * s, nymax, nxmax);
  // band: input rows a + dy - t over the classes that have taps
  int dmin = 1 << 30, dmax = -(1 << 30);
  for (int c = 0; c < s; ++c) {
    const int k0 = (c + cd.p) % s;
    if (k0 >= k) continue;
    const int nt = (k - k0 + s - 1) / s, d = (c + cd.p - k0) / s;
    dmin = std::min(dmin, d - nt + 1);
    dmax = std::max(dmax, d);
  }
  pl.dmin = dmin;
  pl.SH = pl.TA + dmax - dmin;
  pl.SW = nxmax + dmax - dmin;
  pl.plane = conv_plane(pl.SH, pl.SW, pl.mf);
  pl.CC = conv_depth(cc, pl.plane, cd.co, pl.mf);
  pl.inv_sh = 1.0f / (float)pl.SH;
  return pl;
}

// Plan of a forward convolution (input ci x hi x wi, output co x ho x wo);
// nq > 0 fixes the matrix-core kernel's column tiles per task.
inline ConvPlan plan_convf(const ConvDesc& cd, int nq, int cc) {
  ConvPlan pl{};
  conv_shape(pl, cd.co, 1, cd.ho, cd.wo);
  if (pl.mf && nq > 0 && nq != pl.NQ) {
    pl.NQ = nq;
    const int per = 16 * nq;
    const int want = std::max(1, (4 + pl.nblk - 1) / pl.nblk);
    conv_tiles(pl, 1, cd.ho, cd.wo, per, std::max(64, want * per));
  }
  pl.SH = (pl.TA - 1) * cd.s + cd.k;
  pl.SW = (cd.wo - 1) * cd.s + cd.k;
  pl.plane = conv_plane(pl.SH, pl.SW, pl.mf);
  pl.CC = conv_depth(cc, pl.plane, cd.ci, pl.mf);
  pl.inv_sh = 1.0f / (float)pl.SH;
  return pl;
}

template <class Epi, int CB, int P>
void launch_convt(int R, const ConvDesc& cd, const ConvPlan& pl, const double* in, Epi epi,
                  double* part, int ntiles, hipStream_t s) {
  const long long nwg = (long long)R * pl.nT * pl.wgt;
  hipLaunchKernelGGL((k_convt<Epi, CB, P>), dim3((unsigned)nwg), dim3(256),
                     (size_t)pl.CC * pl.plane * 8, s, cd, pl, in, epi, part, ntiles);
}

template <class Epi, int CB, int P>
void launch_convf(int R, const ConvDesc& cd, const ConvPlan& pl, const double* in, Epi epi,
                  double* part, int ntiles, hipStream_t s) {
  const long long nwg = (long long)R * pl.nT * pl.wgt;
  hipLaunchKernelGGL((k_convf<Epi, CB, P>), dim3((unsigned)nwg), dim3(256),
                     (size_t)pl.CC * pl.plane * 8, s, cd, pl, in, epi, part, ntiles);
}

template <class Epi, int MT, int NQ>
void launch_convt_mf(int R, const ConvDesc& cd, const ConvPlan& pl, const double* in, Epi epi,
                     double* part, int ntiles, hipStream_t s) {
  const long long nwg = (long long)R * pl.nT * pl.wgt;
  hipLaunchKernelGGL((k_convt_mf<Epi, MT, NQ>), dim3((unsigned)nwg), dim3(256),
                     (size_t)pl.CC * pl.plane * 8, s, cd, pl, in, epi, part, ntiles);
}

template <class Epi, int MT, int NQ>
void launch_convf_mf(int R, const ConvDesc& cd, const ConvPlan& pl, const double* in, Epi epi,
                     double* part, int ntiles, hipStream_t s) {
  const long long nwg = (long long)R * pl.nT * pl.wgt;
  hipLaunchKernelGGL((k_convf_mf<Epi, MT, NQ>), dim3((unsigned)nwg), dim3(256),
                     (size_t)pl.CC * pl.plane * 8, s, cd, pl, in, epi, part, ntiles);
}

// A plan the kernels can run: a band that fits LDS and the staging loop
// (SW <= 256), at most `ntiles` row-sum slots per row, a grid within range.
inline bool conv_plan_ok(const ConvPlan& pl, int R, int ntiles) {
  return pl.plane * pl.CC <= CONV_BAND_MAX && pl.SW <= 256 && pl.nT * pl.wgt <= ntiles &&
         (long long)R * pl.nT * pl.wgt < (1ll << 31);
}

// The whole-row kernels take a layer whose input row (transposed: co x ho x
// wo, forward: ci x hi x wi) fits their LDS staging, unless it has 32 or
// more channels on both sides (a contraction the matrix cores of the tiled
// kernels run faster, measured at the 3x32x32 CNNs) or the net was made to
// run the tiled kernels everywhere.
inline bool conv_whole_row(const ConvDesc& cd, bool transposed) {
  const bool wide = cd.ci >= 32 && cd.co >= 32;
  return !cd.tiled && !wide &&
         (transposed ? cd.co * cd.ho * cd.wo : cd.ci * cd.hi * cd.wi) <= CONV_STAGE_MAX;
}

// Transposed convolution: the whole-row kernels where the input row fits
// LDS (variants as run_convt_row), else the tiled ones, variant (autotuner)
// 0: staging depth by the band budget, 1/2/3: 4, 8 or 16 channels per
// chunk.  No variant changes a result.
template <class Epi>
hipError_t run_convt(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant = 0) {
  if (R <= 0) return hipSuccess;
  if (conv_whole_row(cd, true)) return run_convt_row(R, cd, in, epi, part, ntiles, s, variant);
  const int cc = variant == 1 ? 4 : variant == 2 ? 8 : variant == 3 ? 16 : 0;
  const ConvPlan pl = plan_convt(cd, cc);
  if (!conv_plan_ok(pl, R, Epi::NSUM > 0 ? ntiles : 1 << 30)) return hipErrorInvalidValue;
  if (pl.mf) {
    switch (pl.MT * 10 + pl.NQ) {
      case 11: launch_convt_mf<Epi, 1, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 12: launch_convt_mf<Epi, 1, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 21: launch_convt_mf<Epi, 2, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 22: launch_convt_mf<Epi, 2, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 31: launch_convt_mf<Epi, 3, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 32: launch_convt_mf<Epi, 3, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 41: launch_convt_mf<Epi, 4, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      default: launch_convt_mf<Epi, 4, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
    }
    return hipGetLastError();
  }
  switch (pl.CB * 10 + pl.P) {
    case 41: launch_convt<Epi, 4, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
    case 42: launch_convt<Epi, 4, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
    case 81: launch_convt<Epi, 8, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
    default: launch_convt<Epi, 8, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
  }
  return hipGetLastError();
}

// Forward convolution: the whole-row kernels where the input row fits LDS
// (variants as run_convf_row), else the tiled ones, variant 0: tiles and
// staging depth by shape, 1/2/3: 4, 8 or 16 channels per chunk, 4: the
// other column-tile count (matrix cores; the vector kernel keeps its shape).  The forward convolution has no
// row sums and accumulates each output in the same order under every
// variant, so the choice changes no result.
template <class Epi>
hipError_t run_convf(int R, const ConvDesc& cd, const double* in, Epi epi, double* part, int ntiles,
                     hipStream_t s, int variant = 0) {
  if (R <= 0) return hipSuccess;
  if (conv_whole_row(cd, false)) return run_convf_row(R, cd, in, epi, part, ntiles, s, variant);
  const int cc = variant == 1 ? 4 : variant == 2 ? 8 : variant == 3 ? 16 : 0;
  ConvPlan pl = plan_convf(cd, 0, cc);
  if (variant == 4 && pl.mf) pl = plan_convf(cd, 3 - pl.NQ, 0);
  if (!conv_plan_ok(pl, R, Epi::NSUM > 0 ? ntiles : 1 << 30)) return hipErrorInvalidValue;
  if (pl.mf) {
    switch (pl.MT * 10 + pl.NQ) {
      case 11: launch_convf_mf<Epi, 1, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 12: launch_convf_mf<Epi, 1, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 21: launch_convf_mf<Epi, 2, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 22: launch_convf_mf<Epi, 2, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 31: launch_convf_mf<Epi, 3, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 32: launch_convf_mf<Epi, 3, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
      case 41: launch_convf_mf<Epi, 4, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
      default: launch_convf_mf<Epi, 4, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
    }
    return hipGetLastError();
  }
  switch (pl.CB * 10 + pl.P) {
    case 41: launch_convf<Epi, 4, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
    case 42: launch_convf<Epi, 4, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
    case 81: launch_convf<Epi, 8, 1>(R, cd, pl, in, epi, part, ntiles, s); break;
    default: launch_convf<Epi, 8, 2>(R, cd, pl, in, epi, part, ntiles, s); break;
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

bool conv_whole_row_layer(const ConvDesc& cd, bool transposed) { return conv_whole_row(cd, transposed); }

int gemm_ntiles(int N) { return (N + TileDefault::BN - 1) / TileDefault::BN; }

hipError_t launch_gemm_relax(int R, int K, int N, const double* Om, const float* W,
                             const ConvDesc* conv, int M, int Nh,
                             int off, const float* lz, const float* uz, const float* alpha,
                             double alpha_def, const float* bprev, CvProps props, int layer,
                             double* Om_out, float* trace, double* part, int variant,
                             hipStream_t s) {
  const bool full = alpha && trace;
  if (props.host) {  // one property: its error weight for every row
    EpiRelax<false> e{M, Nh, off, lz, uz, alpha, alpha_def, bprev, props.host->wrel[layer], props,
                      layer, Om_out, N, trace};
    if (conv) return run_convt(R, *conv, Om, e, part, gemm_ntiles(N), s, variant);
    if (full) {
      EpiRelax<false, true> f{M, Nh, off, lz, uz, alpha, alpha_def, bprev, props.host->wrel[layer],
                              props, layer, Om_out, N, trace};
      return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, f, part, s);
    }
    return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, e, part, s);
  }
  EpiRelax<true> e{M, Nh, off, lz, uz, alpha, alpha_def, bprev, nullptr, props, layer, Om_out, N,
                   trace};
  if (conv) return run_convt(R, *conv, Om, e, part, gemm_ntiles(N), s, variant);
  if (full) {
    EpiRelax<true, true> f{M, Nh, off, lz, uz, alpha, alpha_def, bprev, nullptr, props, layer,
                           Om_out, N, trace};
    return run_gemm_v(variant, R, K, N, LoadF64{Om, K}, W, N, f, part, s);
  }
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
  const bool full = alpha_in && alpha && lr > 0.0 && !fresh && adam_m && adam_v;
  if (full) {
    EpiAdjT<true> f{M, Nh, off, b, lz, uz, alpha, alpha_def, trace, infeasible, grad, adam_m, adam_v,
                    lr, b1, b2, eps, bc1, bc2, Psibar_out, N, alpha_in, fresh};
    // the whole-row forward convolutions gain from the fixed form (config 3's
    // layers 1.765 -> 1.690 ms); the tiled ones lost (4.14 -> 4.23 ms)
    if (conv && conv_whole_row(*conv, false)) return run_convf_row(R, *conv, Abar, f, nullptr, 1, s, variant);
    if (!conv) return run_gemm_v(variant, R, K, N, LoadF64{Abar, K}, Wt, N, f, nullptr, s);
  }
  if (conv) return run_convf(R, *conv, Abar, e, nullptr, 1, s, variant);
  return run_gemm_v(variant, R, K, N, LoadF64{Abar, K}, Wt, N, e, nullptr, s);
}
