// Small kernels of the backward pass and of the root set-up: the shared top
// layer, the first relaxation, row-state accumulation, final rounding,
// split fixes, and the packing of the cached planes.
#include "cv_common.h"
#include "cv_internal.h"

namespace {

// Psi_T = C W_T (shared by the subdomains of a property), c0 = t + C b_T and
// the error weight e0 = |C| vT, one workgroup per (objective row m, property p);
// C is [P, M, nT], t [P, M], outputs [P, M, .].
__global__ __launch_bounds__(256) void k_top(int M, int nT, int nP, const float* __restrict__ C,
                                             const float* __restrict__ t,
                                             const float* __restrict__ W,
                                             const float* __restrict__ b, CvProps props,
                                             int layer, double* psiT, double* c0, double* e0,
                                             double* cabs0) {
  const int m = blockIdx.y * M + blockIdx.x;  // row of the stacked objective
  const double* __restrict__ vT = props.tab[blockIdx.y].vgemm[layer];
  const float* crow = C + (size_t)m * nT;
  for (int j = threadIdx.x; j < nP; j += blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < nT; ++k) acc += (double)crow[k] * (double)W[(size_t)k * nP + j];
    psiT[(size_t)m * nP + j] = acc;
  }
  if (threadIdx.x < 64) {
    double cb = 0.0, ea = 0.0;
    for (int k = threadIdx.x; k < nT; k += 64) {
      cb += (double)crow[k] * (double)b[k];
      ea += fabs((double)crow[k]) * vT[k];
    }
    cb = wave_sum(cb);
    ea = wave_sum(ea);
    if (threadIdx.x == 0) {
      c0[m] = (double)t[m] + cb;
      e0[m] = ea;
      cabs0[m] = fabs((double)t[m]) + fabs(cb);
    }
  }
}

// Entry (m, j) of the dense matrix of convolution layer cd: output m =
// (co, oy, ox) reads input j = (ci, iy, ix) through the kernel tap (ky, kx) =
// (iy - oy*s + p, ix - ox*s + p) when that tap exists, else 0 (kernel from the
// transposed-convolution layout Wb [co][k][k][ptp], which holds the float32
// weights exactly).
__device__ __forceinline__ double conv_entry(const ConvDesc& cd, size_t m, size_t j) {
  const int hw = cd.ho * cd.wo, ihw = cd.hi * cd.wi;
  const int co = (int)(m / hw), oy = (int)((m % hw) / cd.wo), ox = (int)(m % cd.wo);
  const int ci = (int)(j / ihw), iy = (int)((j % ihw) / cd.wi), ix = (int)(j % cd.wi);
  const int ky = iy - oy * cd.s + cd.p, kx = ix - ox * cd.s + cd.p;
  if (ky < 0 || ky >= cd.k || kx < 0 || kx >= cd.k) return 0.0;
  return cd.Wb[(((size_t)co * cd.k + ky) * cd.k + kx) * cd.ptp + ci];
}

// The same for the objective C = eye * I (eye = +-1), t = 0 (intermediate
// bounds of a layer): Psi_T is row m of W_T times eye, c0 = eye b_T[m], e0 =
// vT[m] -- what k_top computes for that C, exactly, without its dense loop.
// A conv layer T (conv = 1) gives its rows from the kernel.
__global__ void k_top_eye(int M, int nP, double eye, const float* __restrict__ W, ConvDesc cd,
                          int conv, const float* __restrict__ b, CvProps props, int layer,
                          double* psiT, double* c0, double* e0, double* cabs0) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = (size_t)props.P * M * nP;
  if (i >= tot) return;
  const int p = (int)(i / ((size_t)M * nP));
  const int m = (int)((i / nP) % M), j = (int)(i % nP);
  psiT[i] = eye * (conv ? conv_entry(cd, m, j) : (double)W[(size_t)m * nP + j]);
  if (j == 0) {
    const size_t row = (size_t)p * M + m;
    c0[row] = eye * (double)b[m];
    e0[row] = props.tab[p].vgemm[layer][m];
    cabs0[row] = fabs((double)b[m]);
  }
}

// Rows [0, rows) of the dense matrix of convolution layer cd, float32.
__global__ void k_conv_dense(ConvDesc cd, int rows, float* out) {
  const size_t ncol = (size_t)cd.ci * cd.hi * cd.wi;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)rows * ncol) return;
  out[i] = (float)conv_entry(cd, i / ncol, i % ncol);
}

// dst[q, :] = src[idx[q], :] for q < rows (rows of n floats).
__global__ void k_gather_rows(int rows, int n, const int32_t* __restrict__ idx,
                              const float* __restrict__ src, float* dst) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)rows * n) return;
  const size_t q = i / n, c = i % n;
  dst[i] = src[(size_t)idx[q] * n + c];
}

// One lane's share of a top row: elements j = lane, lane + 64, ... in
// chunks of four per lane, every load of a chunk issued before the first is
// used; the sums accumulate the elements in increasing j.  HAS_ALPHA is a
// template flag so no branch on it sits between the loads.
template <bool HAS_ALPHA>
__device__ __forceinline__ void relax_top_lane(int lane, int nP, const double* __restrict__ psirow,
                                               const float* __restrict__ lzb,
                                               const float* __restrict__ uzb,
                                               const float* __restrict__ alr, double alpha_def,
                                               const float* __restrict__ bprev,
                                               const double* __restrict__ wrel, double* omr,
                                               float* trr, double& s1, double& s2, double& s3) {
  constexpr int U = 4;
  for (int j0 = lane; j0 < nP; j0 += 64 * U) {
    double psi[U], wr[U];
    float lv[U], uv[U], av[U], bp[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      // past the end: a valid index whose values go unused (j0 < nP here)
      const int j = min(j0 + 64 * q, nP - 1);
      psi[q] = psirow[j];
      lv[q] = lzb[j];
      uv[q] = uzb[j];
      av[q] = HAS_ALPHA ? alr[j] : 0.0f;
      bp[q] = bprev[j];
      wr[q] = wrel[j];
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = j0 + 64 * q;
      if (j >= nP) break;
      const double al = HAS_ALPHA ? (double)av[q] : alpha_def;
      const Relax rl = relax_apply(psi[q], relax_line(lv[q], uv[q]), al);
      const double om = psi[q] * rl.s;
      omr[j] = om;
      if (trr) trr[j] = trace32(psi[q]);
      s1 += psi[q] * rl.t;
      s2 += om * (double)bp[q];
      s3 += fabs(psi[q]) * wr[q];
    }
  }
}

// First relaxation (ReLU of layer T-1) of every row r = (b, m): one wave
// per row.  Writes Omega_{T-1} and initialises the row state; the top rows
// are those of subdomain b's property.
__global__ __launch_bounds__(256) void k_relax_top(
    int R, int M, int nP, int Nh, int off, const double* __restrict__ psiT,
    const double* __restrict__ c0, const double* __restrict__ e0, const double* __restrict__ cabs0,
    const float* __restrict__ lz, const float* __restrict__ uz, const float* __restrict__ alpha,
    double alpha_def, const float* __restrict__ bprev, CvProps props, int layer,
    double* Om, float* trace, double* rowc, double* rowerr, double* rowcabs) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  const int b = r / M;
  const int p = prop_index(props, b);
  const int m = p * M + r % M;
  const double* __restrict__ wrel = props.tab[p].wrel[layer];
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const double* psirow = psiT + (size_t)m * nP;
  const size_t bbase = (size_t)b * Nh + off, rbase = (size_t)r * Nh + off;
  double* omr = Om + (size_t)r * nP;
  float* trr = trace ? trace + rbase : nullptr;
  if (alpha)
    relax_top_lane<true>(lane, nP, psirow, lz + bbase, uz + bbase, alpha + rbase, alpha_def, bprev,
                         wrel, omr, trr, s1, s2, s3);
  else
    relax_top_lane<false>(lane, nP, psirow, lz + bbase, uz + bbase, nullptr, alpha_def, bprev,
                          wrel, omr, trr, s1, s2, s3);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  s3 = wave_sum(s3);
  if (lane == 0) {
    rowc[r] = c0[m] + s1 + s2;
    rowerr[r] = e0[m] + s3;
    rowcabs[r] = cabs0[m] + fabs(s1) + fabs(s2);
  }
}

__global__ void k_rowacc(int R, int ntiles, const double* __restrict__ part, double* rowc,
                         double* rowerr, double* rowcabs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    const double* p = part + ((size_t)r * ntiles + t) * 3;
    s1 += p[0];
    s2 += p[1];
    s3 += p[2];
  }
  rowc[r] += s1 + s2;
  rowerr[r] += s3;
  rowcabs[r] += fabs(s1) + fabs(s2);
}

// lb = c + sum_j min(A_j lo_j, A_j hi_j), moved down by the rigorous error
// bound, rounded down to float32.  rowerr becomes the error bound of the
// plane (A, c) itself (used by complete clipping); c_out (optional) is c moved
// down by that bound and by the float32 rounding of A.
__global__ void k_finalize(int R, int M, int ntiles, const double* __restrict__ part,
                           const double* __restrict__ rowc, double* rowerr,
                           const double* __restrict__ rowcabs, double gamma_big,
                           const uint8_t* __restrict__ infeasible, float* lb, float* c_out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double slb = 0.0, sabs = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    const double* p = part + ((size_t)r * ntiles + t) * 2;
    slb += p[0];
    sabs += p[1];
  }
  const double c = rowc[r];
  const double eplane = (gamma_big * (rowerr[r] + sabs) + 4.0 * CV_U64 * 16.0 * rowcabs[r]) * CV_ERR_SLACK;
  const double v = c + slb;
  const double err = eplane + 8.0 * CV_U64 * (fabs(c) + fabs(slb));
  const bool dead = infeasible && infeasible[r / M];
  lb[r] = dead ? INFINITY : rd32(v - err);
  rowerr[r] = eplane;
  if (c_out) c_out[r] = rd32(c - eplane - 1.2e-7 * sabs);
}

// Root-stable neurons of each subdomain's property keep their root bounds.
__global__ void k_fill_stable(int B, int Nh, int nSmax, CvProps props, float* l, float* u) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * nSmax) return;
  const int b = (int)(i / nSmax), q = (int)(i % nSmax);
  const RootDev& rd = prop_of(props, b);
  if (q >= Nh - rd.U) return;
  const int j = rd.sidx[q];
  l[(size_t)b * Nh + j] = rd.l0[j];
  u[(size_t)b * Nh + j] = rd.u0[j];
}

// Split neurons are fixed to their branch; l > u marks the subdomain empty.
__global__ void k_split_fix(int B, int Nh, CvCons sp, float* l, float* u, uint8_t* infeasible) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * sp.kmax) return;
  const int b = i / sp.kmax, k = i % sp.kmax;
  if (k >= cons_count(sp, b)) return;
  const int j = sp.neuron[(size_t)b * sp.kmax + k];
  if (j < 0 || j >= Nh) return;
  const size_t bi = (size_t)b * Nh + j;
  if (sp.sign[(size_t)b * sp.kmax + k] > 0) l[bi] = fmaxf(l[bi], 0.0f);
  else u[bi] = fminf(u[bi], 0.0f);
  if (l[bi] > u[bi]) infeasible[b] = 1;
}

// Complete-clipping results of intermediate neurons: l <- max(l, L_lo),
// u <- min(u, -L_up); an empty result marks the subdomain.
__global__ void k_merge_neurons(int B, int Umax, CvProps props, int Nh,
                                const float* __restrict__ Ltmp, float* l, float* u,
                                uint8_t* infeasible) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * Umax) return;
  const int b = (int)(i / Umax), c = (int)(i % Umax);
  const RootDev& rd = prop_of(props, b);
  if (c >= rd.U) return;
  const int j = rd.uidx[c];
  const float Ll = Ltmp[i * 2], Lu = Ltmp[i * 2 + 1];
  const size_t bi = (size_t)b * Nh + j;
  if (Ll == INFINITY || Lu == INFINITY) { infeasible[b] = 1; return; }
  l[bi] = fmaxf(l[bi], Ll);
  u[bi] = fminf(u[bi], -Lu);
  if (l[bi] > u[bi]) infeasible[b] = 1;
}

// Root set-up: the float64 plane (A, c) of a row, valid up to its error bound
// e, becomes a plane with float32 coefficients A32 = nearest(A) that is still
// valid on the root box: A x + c and A32 x + c' differ by (A - A32).x, which
// is (A - A32).xc exactly at the box centre xc and varies by at most
// sum |A - A32| r over the box (r its half-width), so
//   c' = c - e + (A - A32).xc - sum |A - A32| r     (lower plane)
// stays below the exact plane everywhere on the box (A - A32 is exact in
// float64; the two sums get their own rounding bound).  The intercept is
// kept in float64.  negate != 0 stores the upper plane (-A, -c) from the
// objective -I, moved up instead.  Centring keeps the widening at
// 2^-24 sum |A| r instead of 2^-24 sum |A| max(|lo|, |hi|), which matters for
// narrow boxes far from the origin (images in [0, 1] with eps 2/255).
__global__ __launch_bounds__(64) void k_root_store(int rows, int n0, const double* __restrict__ Ax,
                                                   const double* __restrict__ rowc,
                                                   const double* __restrict__ rowerr,
                                                   const double* __restrict__ xc0,
                                                   const double* __restrict__ rad0, int negate,
                                                   float* A_dst, double* c_dst) {
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  double corr = 0.0, wid = 0.0, scale = 0.0;
  for (int j = lane; j < n0; j += 64) {
    const double a = negate ? -Ax[(size_t)r * n0 + j] : Ax[(size_t)r * n0 + j];
    const float f = (float)a;
    A_dst[(size_t)r * n0 + j] = f;
    const double d = a - (double)f;  // exact
    corr += d * xc0[j];
    wid += fabs(d) * rad0[j];
    scale += fabs(d) * (fabs(xc0[j]) + rad0[j]);
  }
  corr = wave_sum(corr);
  wid = wave_sum(wid);
  scale = wave_sum(scale);
  if (lane == 0) {
    const double e = rowerr[r] * CV_ERR_SLACK + cv_gamma(n0 + 2) * scale;
    const double c = negate ? -rowc[r] : rowc[r];
    c_dst[r] = negate ? c + corr + wid + e : c + corr - wid - e;
  }
}

// min (upper = 0) or max (upper = 1) of A[r].x + c[r] over one box, rounded
// outward after a rigorous float64 error bound.
__global__ __launch_bounds__(64) void k_concretize_rows(int rows, int n0, const float* __restrict__ A,
                                                        const double* __restrict__ c,
                                                        const float* __restrict__ lo,
                                                        const float* __restrict__ hi, int upper,
                                                        float* out) {
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0, e = 0.0;
  for (int j = lane; j < n0; j += 64) {
    const double a = (double)A[(size_t)r * n0 + j];
    const double x0 = (double)lo[j], x1 = (double)hi[j];
    s += upper ? fmax(a * x0, a * x1) : fmin(a * x0, a * x1);
    e += fabs(a) * fmax(fabs(x0), fabs(x1));
  }
  s = wave_sum(s);
  e = wave_sum(e);
  if (lane == 0) {
    const double cc = c[r];
    const double err = (cv_gamma(n0 + 1) * (e + fabs(cc))) * CV_ERR_SLACK;
    out[r] = upper ? ru32(s + cc + err) : rd32(s + cc - err);
  }
}

// float32 images of the intercepts, rounded outward (down for lower planes,
// up for upper planes), for callers that read the planes.
__global__ __launch_bounds__(256) void k_round_intercepts(int N, const double* __restrict__ c,
                                                          int upper, float* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < N) out[i] = upper ? ru32(c[i]) : rd32(c[i]);
}

// Packed plane matrix for the re-concretization GEMM.  Column q < U is the
// lower plane of neuron uidx[q]: rows [0, n0) hold A_lo^+ (multiplying lo),
// rows [n0, 2 n0) hold A_lo^- (multiplying hi).  Column U + q is the upper
// plane: A_hi^- against lo, A_hi^+ against hi.  eP is the rigorous error
// bound of the float64 evaluation (products of float32 values are exact).
__global__ __launch_bounds__(64) void k_build_P(int n0, int U, const int32_t* __restrict__ uidx,
                                                const float* __restrict__ A_lo,
                                                const float* __restrict__ A_hi,
                                                const double* __restrict__ c_lo,
                                                const double* __restrict__ c_hi,
                                                const double* __restrict__ X0, float* P, double* cP,
                                                double* eP) {
  const int q = blockIdx.x;  // 0 .. 2U-1
  const int lane = threadIdx.x;
  const bool up = q >= U;
  const int j = uidx[up ? q - U : q];
  const float* a = (up ? A_hi : A_lo) + (size_t)j * n0;
  const size_t ld = (size_t)2 * U;
  double e = 0.0;
  for (int k = lane; k < n0; k += 64) {
    const float v = a[k];
    const float pos = v > 0.0f ? v : 0.0f, neg = v < 0.0f ? v : 0.0f;
    P[(size_t)k * ld + q] = up ? neg : pos;
    P[(size_t)(k + n0) * ld + q] = up ? pos : neg;
    e += fabs((double)v) * X0[k];
  }
  e = wave_sum(e);
  if (lane == 0) {
    const double cc = up ? c_hi[j] : c_lo[j];
    cP[q] = cc;
    eP[q] = cv_gamma(2 * n0 + 2) * (e + fabs(cc)) * CV_ERR_SLACK;
  }
}

// Weights of the neuron-selection score: max(0, -mean over the objective rows
// of the backward coefficient Psi of each hidden neuron), from the trace of a
// backward pass over one box (rows m = 0..M-1).
__global__ __launch_bounds__(256) void k_babsr_weight(int M, int Nh, const float* __restrict__ trace,
                                                      float* weight) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= Nh) return;
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += (double)trace[(size_t)m * Nh + k];
  weight[k] = (float)fmax(0.0, -(s / (double)M));
}

// Top-k unstable neurons of one hidden layer of one subdomain by the BaBSR
// intercept score  max(0,-l) max(0,u) / (u - l) * weight  (float64), ties to
// the lower index.  One workgroup per (subdomain, layer); the layer's scores
// sit in LDS and every neuron counts the ones ranked above it.
struct LayerTable {
  int count;
  int off[CV_MAX_LAYERS];
  int size[CV_MAX_LAYERS];
};
constexpr int TOPK_NMAX = 4096;
__global__ __launch_bounds__(256) void k_select_topk(int Nh, LayerTable lt, const float* __restrict__ l,
                                                     const float* __restrict__ u,
                                                     const float* __restrict__ wall, CvProps props,
                                                     int k, uint8_t* select) {
  __shared__ double ssc[TOPK_NMAX];
  const int b = blockIdx.x, layer = blockIdx.y;
  const float* __restrict__ weight = wall + (size_t)prop_index(props, b) * Nh;  // [P, Nh]
  const int off = lt.off[layer], n = lt.size[layer];
  const float* lb = l + (size_t)b * Nh + off;
  const float* ub = u + (size_t)b * Nh + off;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double lj = (double)lb[j], uj = (double)ub[j];
    ssc[j] = (lj < 0.0 && uj > 0.0) ? (-lj) * uj / (uj - lj) * (double)weight[off + j] : -1.0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += 256) {
    const double sj = ssc[j];
    int rank = 0;
    if (sj >= 0.0)
      for (int i = 0; i < n && rank < k; ++i) {
        const double si = ssc[i];
        rank += (si > sj || (si == sj && i < j)) ? 1 : 0;
      }
    select[(size_t)b * Nh + off + j] = (sj >= 0.0 && rank < k) ? 1 : 0;
  }
}

// l[b, off + m] = max(l, lbl[b, m]) and u[b, off + m] = min(u, -lbn[b, m]):
// the CROWN bounds of one layer over each box (objective +I: lower bound,
// objective -I: minus the upper bound), intersected with the bounds at hand.
__global__ void k_merge_layer(int B, int n, int Nh, int off, const float* __restrict__ lbl,
                              const float* __restrict__ lbn, float* l, float* u,
                              uint8_t* infeasible) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)B * n) return;
  const size_t b = i / n, m = i % n;
  float* pl = l + b * Nh + off + m;
  float* pu = u + b * Nh + off + m;
  const float nl = fmaxf(*pl, lbl[i]), nu = fminf(*pu, -lbn[i]);
  *pl = nl;
  *pu = nu;
  if (nl > nu && infeasible) infeasible[b] = 1;  // both bounds valid: the box is empty
}

// Deterministic filler in [lo, hi) (a 32-bit integer hash of the index):
// synthetic operands for timing kernel variants.
template <class T>
__global__ void k_fill_pattern(T* p, size_t n, double lo, double hi, uint32_t seed) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t x = (uint32_t)i * 2654435761u ^ seed;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  p[i] = (T)(lo + (hi - lo) * (double)x * 2.3283064365386963e-10);
}

}  // namespace

hipError_t launch_top(int P, int M, int nT, int nP, const float* C, const float* t,
                      const float* W, const float* b, CvProps props, int layer, double* psiT,
                      double* c0, double* e0, double* cabs0, hipStream_t s) {
  hipLaunchKernelGGL(k_top, dim3(M, P), dim3(256), 0, s, M, nT, nP, C, t, W, b, props, layer,
                     psiT, c0, e0, cabs0);
  return hipGetLastError();
}

hipError_t launch_top_eye(int P, int M, int nP, double eye, const float* W, const ConvDesc* conv,
                          const float* b, CvProps props, int layer, double* psiT, double* c0,
                          double* e0, double* cabs0, hipStream_t s) {
  const size_t tot = (size_t)P * M * nP;
  if (tot == 0) return hipSuccess;
  if ((tot + 255) / 256 > 0x7fffffffu) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_top_eye, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, nP, eye, W,
                     conv ? *conv : ConvDesc{}, conv ? 1 : 0, b, props, layer, psiT, c0, e0,
                     cabs0);
  return hipGetLastError();
}

hipError_t launch_conv_dense(const ConvDesc& cd, int rows, float* out, hipStream_t s) {
  const size_t tot = (size_t)rows * cd.ci * cd.hi * cd.wi;
  if (tot == 0) return hipSuccess;
  if ((tot + 255) / 256 > 0x7fffffffu) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_conv_dense, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, cd, rows,
                     out);
  return hipGetLastError();
}

hipError_t launch_gather_rows(int rows, int n, const int32_t* idx, const float* src, float* dst,
                              hipStream_t s) {
  const size_t tot = (size_t)rows * n;
  if (tot == 0) return hipSuccess;
  if ((tot + 255) / 256 > 0x7fffffffu) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rows, n,
                     idx, src, dst);
  return hipGetLastError();
}

hipError_t launch_relax_top(int R, int M, int nP, int Nh, int off, const double* psiT,
                            const double* c0, const double* e0, const double* cabs0,
                            const float* lz, const float* uz, const float* alpha,
                            double alpha_def, const float* bprev, CvProps props, int layer,
                            double* Om, float* trace, double* rowc, double* rowerr,
                            double* rowcabs, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relax_top, dim3((R + 3) / 4), dim3(256), 0, s, R, M, nP, Nh, off, psiT, c0,
                     e0, cabs0, lz, uz, alpha, alpha_def, bprev, props, layer, Om, trace, rowc,
                     rowerr, rowcabs);
  return hipGetLastError();
}

hipError_t launch_rowacc(int R, int ntiles, const double* part, double* rowc, double* rowerr,
                         double* rowcabs, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rowacc, dim3((R + 255) / 256), dim3(256), 0, s, R, ntiles, part, rowc,
                     rowerr, rowcabs);
  return hipGetLastError();
}

hipError_t launch_finalize(int R, int M, int ntiles, const double* part, const double* rowc,
                           double* rowerr, const double* rowcabs, double gamma_big,
                           const uint8_t* infeasible, float* lb, float* c_out, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((R + 255) / 256), dim3(256), 0, s, R, M, ntiles, part, rowc,
                     rowerr, rowcabs, gamma_big, infeasible, lb, c_out);
  return hipGetLastError();
}

hipError_t launch_fill_stable(int B, int Nh, int nSmax, CvProps props, float* l, float* u,
                              hipStream_t s) {
  const size_t tot = (size_t)B * nSmax;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_stable, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B, Nh,
                     nSmax, props, l, u);
  return hipGetLastError();
}

hipError_t launch_split_fix(int B, int Nh, const CvCons& splits, float* l, float* u,
                            uint8_t* infeasible, hipStream_t s) {
  const int tot = B * splits.kmax;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_fix, dim3((tot + 255) / 256), dim3(256), 0, s, B, Nh, splits, l, u,
                     infeasible);
  return hipGetLastError();
}

hipError_t launch_merge_neurons(int B, int Umax, CvProps props, int Nh, const float* Ltmp,
                                float* l, float* u, uint8_t* infeasible, hipStream_t s) {
  const size_t tot = (size_t)B * Umax;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_neurons, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B, Umax,
                     props, Nh, Ltmp, l, u, infeasible);
  return hipGetLastError();
}

hipError_t launch_root_store_planes(int rows, int n0, const double* Ax, const double* rowc,
                                    const double* rowerr, const double* xc0, const double* rad0,
                                    int negate, float* A_dst, double* c_dst, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_root_store, dim3(rows), dim3(64), 0, s, rows, n0, Ax, rowc, rowerr, xc0,
                     rad0, negate, A_dst, c_dst);
  return hipGetLastError();
}

hipError_t launch_round_intercepts(int N, const double* c, int upper, float* out, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_round_intercepts, dim3((N + 255) / 256), dim3(256), 0, s, N, c, upper, out);
  return hipGetLastError();
}

hipError_t launch_concretize_rows(int rows, int n0, const float* A, const double* c,
                                  const float* lo, const float* hi, int upper, float* out,
                                  hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_concretize_rows, dim3(rows), dim3(64), 0, s, rows, n0, A, c, lo, hi, upper,
                     out);
  return hipGetLastError();
}

hipError_t launch_build_P(int n0, int U, const int32_t* uidx, const float* A_lo, const float* A_hi,
                          const double* c_lo, const double* c_hi, const double* X0, float* P,
                          double* cP, double* eP, hipStream_t s) {
  if (U <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_P, dim3(2 * U), dim3(64), 0, s, n0, U, uidx, A_lo, A_hi, c_lo, c_hi,
                     X0, P, cP, eP);
  return hipGetLastError();
}

hipError_t launch_babsr_weight(int M, int Nh, const float* trace, float* weight, hipStream_t s) {
  if (Nh <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_babsr_weight, dim3((Nh + 255) / 256), dim3(256), 0, s, M, Nh, trace, weight);
  return hipGetLastError();
}

hipError_t launch_select_topk(int B, int Nh, int nlayers, const int* off, const int* size,
                              const float* l, const float* u, const float* weight, CvProps props,
                              int k, uint8_t* select, hipStream_t s) {
  if (B <= 0 || nlayers <= 0) return hipSuccess;
  LayerTable lt{};
  lt.count = nlayers;
  for (int i = 0; i < nlayers; ++i) {
    if (size[i] > TOPK_NMAX) return hipErrorInvalidValue;
    lt.off[i] = off[i];
    lt.size[i] = size[i];
  }
  hipLaunchKernelGGL(k_select_topk, dim3(B, nlayers), dim3(256), 0, s, Nh, lt, l, u, weight, props,
                     k, select);
  return hipGetLastError();
}

hipError_t launch_fill_pattern(double* p, size_t n, double lo, double hi, uint32_t seed,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_pattern<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p,
                     n, lo, hi, seed);
  return hipGetLastError();
}

hipError_t launch_fill_pattern(float* p, size_t n, double lo, double hi, uint32_t seed,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_pattern<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p,
                     n, lo, hi, seed);
  return hipGetLastError();
}

hipError_t launch_merge_layer(int B, int n, int Nh, int off, const float* lbl, const float* lbn,
                              float* l, float* u, uint8_t* infeasible, hipStream_t s) {
  const size_t tot = (size_t)B * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_layer, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B, n, Nh,
                     off, lbl, lbn, l, u, infeasible);
  return hipGetLastError();
}

// ------------------------------------------------ debug-build input scan
// Flags non-finite values of float arrays in one device word (cleared,
// set by any wave that sees one -- every writer stores the same value --
// and read back on the stream).  Only the debug build's entry points call
// these.
namespace {
__device__ unsigned g_nonfinite;

__global__ void k_nonfinite_reset() { g_nonfinite = 0u; }

__global__ __launch_bounds__(256) void k_nonfinite_scan(const float* __restrict__ p, size_t n) {
  unsigned bad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    bad |= !isfinite(p[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) g_nonfinite = 1u;
}
}  // namespace

hipError_t launch_nonfinite_reset(hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite_reset, dim3(1), dim3(1), 0, s);
  return hipGetLastError();
}

hipError_t launch_nonfinite_scan(const float* p, size_t n, hipStream_t s) {
  const size_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_nonfinite_scan, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t nonfinite_result(unsigned* found, hipStream_t s) {
  hipError_t e = hipMemcpyFromSymbolAsync(found, HIP_SYMBOL(g_nonfinite), sizeof(unsigned), 0,
                                          hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

