// Host-side internals of libclipverify: handle layouts and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>

#define CV_MAX_LAYERS 32

// A convolution layer (cross-correlation, zero padding; activations
// flattened channel-major): input (ci, hi, wi) -> output (co, ho, wo).
struct ConvDesc {
  int ci, hi, wi, co, ho, wo, k, s, p;
  int ptp, pfp;      // ci and co rounded up to a multiple of 16 (of 64 past 64 channels)
  double* Wb;        // device [co rounded up to 4][k][k][ptp]: transposed convolution (blocks of ci)
  double* Wf;        // device [ci rounded up to 4][k][k][pfp]: forward convolution (blocks of co)
  bool tiled;        // the tiled kernels also where the whole-row ones would run
};

struct cv_net_s {
  int L = 0;                  // number of affine layers
  int n[CV_MAX_LAYERS + 1];   // n[0] input dim, n[i] output dim of layer i (1-based)
  float* W[CV_MAX_LAYERS];    // device, layer i at index i-1: [n_i, n_{i-1}]
  float* Wt[CV_MAX_LAYERS];   // device transposes [n_{i-1}, n_i]
  float* b[CV_MAX_LAYERS];    // device [n_i] (conv: the bias repeated over positions)
  ConvDesc conv[CV_MAX_LAYERS];  // conv layers: kernels of the direct convolutions
  bool is_conv[CV_MAX_LAYERS];
  // kernel variants per layer (index i-1 for W_i) chosen by cv_net_autotune:
  // tile of the backward (relax, final) and adjoint GEMMs, channel block of
  // the forward convolution; 0 = the built-in choice
  int8_t tune[3][CV_MAX_LAYERS];
  int off[CV_MAX_LAYERS];     // global offset of hidden layer i (index i-1)
  int n_hidden = 0;
  int nmax_hidden = 0;
  // host copies for the root set-up: hW the matrix of a linear layer (empty
  // for a conv layer), hK the kernel of a conv layer [co][ci][k][k] (empty
  // for a linear layer), hb the bias (conv: repeated over positions)
  std::vector<std::vector<float>> hW, hK, hb;
  // working memory of the root pass, kept between cv_root_create calls on
  // this net (grown as needed, freed with the net)
  void* root_ws = nullptr;
  size_t root_ws_bytes = 0;
};

// Device view of one property's root state: pointers into its cv_root_s.
struct RootDev {
  const float* A_lo;      // cached planes (float32 coefficients): row prow[j] of neuron j,
  const float* A_hi;      // [N, n0] (prow null: row j) or [U, n0] (root-unstable neurons only)
  const int32_t* prow;    // [N] plane row of each neuron, -1: none kept; null: row j
  const double* c_lo;     // [N] float64 intercepts
  const double* c_hi;
  const float* l0;        // [N] root bounds
  const float* u0;
  const double* X0;       // [n0] max(|lo0|, |hi0|)
  const int32_t* uidx;    // [U] root-unstable neurons
  const int32_t* sidx;    // [N - U] root-stable neurons
  const float* P;         // [2 n0, 2U] packed planes
  const double* cP;       // [2U]
  const double* eP;       // [2U]
  int U;
  const double* wrel[CV_MAX_LAYERS];   // hidden layer i at index i-1
  const double* vgemm[CV_MAX_LAYERS];  // layer i at index i-1
};

// Property of each subdomain: subdomain b reads tab[pid[b]] (pid clamped to
// [0, P)); pid null: every subdomain belongs to property 0.
struct CvProps {
  const RootDev* tab;
  const int32_t* pid;
  int P;
  const RootDev* host;  // host copy of the entry when the call has one property (P == 1), else null
};

__device__ __forceinline__ int prop_index(const CvProps& p, int b) {
  if (!p.pid) return 0;
  const int q = p.pid[b];
  return q < 0 ? 0 : (q >= p.P ? p.P - 1 : q);
}

__device__ __forceinline__ const RootDev& prop_of(const CvProps& p, int b) {
  return p.tab[prop_index(p, b)];
}

struct cv_root_s {
  cv_net_s* net = nullptr;
  // A set of properties (cv_rootset_create) has P > 1 members sharing one
  // network; it borrows their state and owns only its table.  A single
  // root is the set of itself (P = 1).
  int P = 1;
  std::vector<cv_root_s*> members;
  RootDev* dtab = nullptr;                    // device [P]
  RootDev htab{};                             // host copy of dtab[0] (single roots)
  int Umax = 0;                               // max U over the members
  int n0 = 0, N = 0, U = 0;
  float alpha0 = 0.5f;
  float *A_lo = nullptr, *A_hi = nullptr;    // [N, n0] or [U, n0] float32 plane coefficients
  int32_t* prow = nullptr;                   // [N] plane row of each neuron (null: all kept)
  double *c_lo = nullptr, *c_hi = nullptr;   // [N] intercepts (float64, see k_root_store)
  double* xc0 = nullptr;                     // [n0] centre of the root box
  double* rad0 = nullptr;                    // [n0] half-width of the root box
  float *l0 = nullptr, *u0 = nullptr;                                        // [N]
  float *lo0 = nullptr, *hi0 = nullptr;                                      // [n0]
  double* X0 = nullptr;                       // [n0] max(|lo0|, |hi0|)
  double* vgemm[CV_MAX_LAYERS];               // layer i: |W_i| H_{i-1} + |b_i|  [n_i]
  double* wrel[CV_MAX_LAYERS];                // hidden layer i: max(|l0|,|u0|) + vgemm_i  [n_i]
  double gamma_big = 0.0;                     // error factor of one backward pass
  // re-concretization of cached planes: unstable neurons, packed plane matrix P [2 n0, 2U]
  int32_t* uidx = nullptr;                    // [U] global index of each root-unstable neuron
  int32_t* sidx = nullptr;                    // [N - U] root-stable neurons
  float* P_planes = nullptr;                  // [2 n0, 2U]
  double* cP = nullptr;                       // [2U] intercepts (lower | upper)
  double* eP = nullptr;                       // [2U] rigorous error bound per column
};

// ----------------------------------------------------------- launchers
// All return hipError_t of the launch.

// Per (subdomain, constraint position) statistics of a constraint over the
// box, shared by every objective row of the subdomain (launch_cons_stats):
// m = min over the box of g.x (h not included), em = sum_j |g_j| max(|lo_j|,
// |hi_j|) and tmax = max_j |g_j| max(|lo_j|,|hi_j|) (rounded up to float32:
// it only scales a tolerance).
struct __align__(8) CvKStat {
  double m, em;
  float tmax, unused;
};

struct CvCons {  // device view of cv_constraints (resolved)
  int kmax;
  const int32_t* count;
  const int32_t* neuron;
  const int8_t* sign;
  const float* G;
  const float* h;
  CvProps props;  // split form: the planes of each subdomain's property (eqs. 9-10)
  int nplanes;    // rows of the plane table; split slots with other indices are ignored
  const int32_t* order;  // [B, kmax] position -> slot, or null (list order)
  // [B, kmax] per position, or null: the constraint's box statistics
  const CvKStat* kstats;
};

// Number of used slots of subdomain b, clamped to [0, kmax].
__device__ __forceinline__ int cons_count(const CvCons& c, int b) {
  int k = c.count ? c.count[b] : c.kmax;
  return k < 0 ? 0 : (k > c.kmax ? c.kmax : k);
}

// Slot processed at position `pos` of subdomain b (the constraint order, if
// any; an index outside [0, kmax) yields -1, an ignored slot).
__device__ __forceinline__ int cons_slot(const CvCons& c, int b, int pos) {
  if (!c.order) return pos;
  const int k = c.order[(size_t)b * c.kmax + pos];
  return (k >= 0 && k < c.kmax) ? k : -1;
}

// Row, sign and offset of slot k of subdomain b as  scale * row . x + h <= 0
// (row == null: the slot is ignored).  Split form: branch z <= 0 gives
// A_lo x + c_lo <= 0, branch z >= 0 gives -A_hi x - c_hi <= 0 (eqs. 9-10).
__device__ __forceinline__ void cons_row_slot(const CvCons& c, int b, int k, int n,
                                              const float*& row, float& scale, double& h) {
  row = nullptr;
  scale = 0.0f;
  h = 0.0;
  if (k < 0) return;
  const size_t s = (size_t)b * c.kmax + k;
  if (c.neuron) {
    const int j = c.neuron[s];
    if (j < 0 || j >= c.nplanes) return;  // not a hidden neuron: slot ignored
    const RootDev& rd = prop_of(c.props, b);
    // a root where only unstable neurons keep planes ignores splits of the
    // others (a dropped constraint only loosens the bounds)
    const int q = rd.prow ? rd.prow[j] : j;
    if (q < 0) return;
    if (c.sign[s] < 0) {
      row = rd.A_lo + (size_t)q * n;
      scale = 1.0f;
      h = rd.c_lo[j];
    } else {
      row = rd.A_hi + (size_t)q * n;
      scale = -1.0f;
      h = -rd.c_hi[j];
    }
  } else {
    row = c.G + s * n;
    scale = 1.0f;
    h = (double)c.h[s];
  }
}

// The constraint at position pos (in the constraint order).
__device__ __forceinline__ void cons_row(const CvCons& c, int b, int pos, int n, const float*& row,
                                         float& scale, double& h) {
  cons_row_slot(c, b, cons_slot(c, b, pos), n, row, scale, h);
}

hipError_t launch_cons_order(int B, int n, const CvCons& cons, const float* lo, const float* hi,
                             int32_t* order, hipStream_t s);
hipError_t launch_clip(int B, int n, const CvCons& cons, float* lo, float* hi, uint8_t* infeasible,
                       int mode, hipStream_t s);

// backward pass building blocks
hipError_t launch_top(int P, int M, int nT, int nP, const float* C, const float* t,
                      const float* W, const float* b, CvProps props, int layer, double* psiT,
                      double* c0, double* e0, double* cabs0, hipStream_t s);
hipError_t launch_top_eye(int P, int M, int nP, double eye, const float* W, const ConvDesc* conv,
                          const float* b, CvProps props, int layer, double* psiT, double* c0,
                          double* e0, double* cabs0, hipStream_t s);
// Rows [0, rows) of the dense matrix of a convolution layer (float32).
// Debug-build input scan: clear the device flag of non-finite values, flag
// those of p[0, n), read the flag back (synchronises s).
hipError_t launch_nonfinite_reset(hipStream_t s);
hipError_t launch_nonfinite_scan(const float* p, size_t n, hipStream_t s);
hipError_t nonfinite_result(unsigned* found, hipStream_t s);
// Whether a conv layer's transposed (or forward) convolution runs the
// whole-row kernels (its input row fits LDS) rather than the tiled ones.
bool conv_whole_row_layer(const ConvDesc& cd, bool transposed);
hipError_t launch_conv_dense(const ConvDesc& cd, int rows, float* out, hipStream_t s);
// dst[q, :] = src[idx[q], :], rows of n floats.
hipError_t launch_gather_rows(int rows, int n, const int32_t* idx, const float* src, float* dst,
                              hipStream_t s);
hipError_t launch_relax_top(int R, int M, int nP, int Nh, int off, const double* psiT,
                            const double* c0, const double* e0, const double* cabs0,
                            const float* lz, const float* uz, const float* alpha,
                            double alpha_def, const float* bprev, CvProps props, int layer,
                            double* Om,
                            float* trace, double* rowc, double* rowerr, double* rowcabs,
                            hipStream_t s);
hipError_t launch_gemm_relax(int R, int K, int N, const double* Om, const float* W,
                             const ConvDesc* conv, int M, int Nh,
                             int off, const float* lz, const float* uz, const float* alpha,
                             double alpha_def, const float* bprev, CvProps props, int layer,
                             double* Om_out, float* trace, double* part, int variant,
                             hipStream_t s);
hipError_t launch_rowacc(int R, int ntiles, const double* part, double* rowc, double* rowerr,
                         double* rowcabs, hipStream_t s);
hipError_t launch_gemm_final(int R, int K, int N, const double* Om, const float* W,
                             const ConvDesc* conv, int M,
                             const float* lo, const float* hi, CvProps props, double* Ax,
                             float* A_out, double* part, int variant, hipStream_t s);
int gemm_ntiles(int N);
hipError_t launch_finalize(int R, int M, int ntiles, const double* part, const double* rowc,
                           double* rowerr, const double* rowcabs, double gamma_big,
                           const uint8_t* infeasible, float* lb, float* c_out, hipStream_t s);
hipError_t launch_gemm_adjoint(int R, int K, int N, const double* Abar, const float* Wt,
                               const ConvDesc* conv,
                               const float* b, int M, int Nh, int off, const float* lz,
                               const float* uz,
                               float* alpha, const float* alpha_in, double alpha_def,
                               const float* trace, const uint8_t* infeasible, float* grad,
                               float* adam_m, float* adam_v, double lr, double b1, double b2,
                               double eps, int step, bool fresh, double* Psibar_out, int variant,
                               hipStream_t s);

// peak probes (benchmark instrumentation)
hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_probe_mfma(int blocks, int iters, double* out, hipStream_t s);

// re-concretization of the cached planes
hipError_t launch_fill_stable(int B, int Nh, int nSmax, CvProps props, float* l, float* u,
                              hipStream_t s);
hipError_t launch_gemm_planes(int B, int n0, int Umax, const float* lo, const float* hi,
                              CvProps props, int Nh, float* l, float* u, hipStream_t s);
hipError_t launch_split_fix(int B, int Nh, const CvCons& splits, float* l, float* u,
                            uint8_t* infeasible, hipStream_t s);

// complete clipping (coordinate ascent over the 1-D duals)
hipError_t launch_cons_stats(int B, int n, const CvCons& cons, const float* lo, const float* hi,
                             CvKStat* stats, hipStream_t s);
hipError_t launch_ca_rows(int R, int M, int n, const CvCons& cons, int passes, double* Ax,
                          const double* rowc, const double* rowerr, const float* lo,
                          const float* hi, uint8_t* infeasible, float* lb, float* beta_out,
                          int write_xstar, float* best, int best_init, hipStream_t s);
hipError_t launch_ca_generic(int B, int P, int n, const float* A, int A_shared, const float* c,
                             const float* lo, const float* hi, const CvCons* cons, int passes,
                             float* lb, float* ub, float* beta_out, uint8_t* infeasible,
                             hipStream_t s);
hipError_t launch_ca_neurons(int B, int Umax, int n, CvProps props,
                             const CvCons& cons, int passes, const float* lo, const float* hi,
                             const float* l, const float* u, int Nh, const uint8_t* infeasible,
                             const uint8_t* select, float* Ltmp, hipStream_t s);
hipError_t launch_branch_relu(int B, int Nh, const float* l, const float* u, const float* weight,
                              CvProps props, int kin, const int32_t* neuron, const int8_t* sign,
                              const int32_t* count, int n0, const float* lo, const float* hi,
                              int kout, int32_t* chosen, int32_t* neuron2, int8_t* sign2,
                              int32_t* count2, float* lo2, float* hi2, hipStream_t s);
hipError_t launch_branch_input(int B, int M, int n0, const float* lo, const float* hi,
                               const float* A, int32_t* dim, float* lo2, float* hi2,
                               hipStream_t s);
hipError_t launch_fill_pattern(double* p, size_t n, double lo, double hi, uint32_t seed,
                               hipStream_t s);
hipError_t launch_fill_pattern(float* p, size_t n, double lo, double hi, uint32_t seed,
                               hipStream_t s);
hipError_t launch_merge_layer(int B, int n, int Nh, int off, const float* lbl, const float* lbn,
                              float* l, float* u, uint8_t* infeasible, hipStream_t s);
hipError_t launch_babsr_weight(int M, int Nh, const float* trace, float* weight, hipStream_t s);
hipError_t launch_select_topk(int B, int Nh, int nlayers, const int* off, const int* size,
                              const float* l, const float* u, const float* weight, CvProps props,
                              int k, uint8_t* select, hipStream_t s);
hipError_t launch_merge_neurons(int B, int Umax, CvProps props, int Nh, const float* Ltmp,
                                float* l, float* u, uint8_t* infeasible, hipStream_t s);

// root set-up helpers
hipError_t launch_root_store_planes(int rows, int n0, const double* Ax, const double* rowc,
                                    const double* rowerr, const double* xc0, const double* rad0,
                                    int negate, float* A_dst, double* c_dst, hipStream_t s);
hipError_t launch_concretize_rows(int rows, int n0, const float* A, const double* c,
                                  const float* lo, const float* hi, int upper, float* out,
                                  hipStream_t s);
hipError_t launch_build_P(int n0, int U, const int32_t* uidx, const float* A_lo, const float* A_hi,
                          const double* c_lo, const double* c_hi, const double* X0, float* P,
                          double* cP, double* eP, hipStream_t s);
hipError_t launch_round_intercepts(int N, const double* c, int upper, float* out, hipStream_t s);
