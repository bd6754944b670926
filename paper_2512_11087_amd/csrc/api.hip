// C ABI of libclipverify: handles, argument validation, workspace layout
// and the host-side sequencing of the kernels (all work is enqueued on the
// caller's stream; only the create calls synchronise).
#include <math.h>
#include <string.h>
#include <algorithm>
#include <vector>

#include <functional>
#include <initializer_list>
#include <cstdlib>
#include <mutex>

#include "clipverify.h"
#include "cv_common.h"
#include "cv_internal.h"

#define CV_VERSION 10000

namespace {

thread_local int g_last_hip = 0;
thread_local const char* t_last_kernel = nullptr;
// Set while an allocation-free entry point runs on this thread: the timing
// instrumentation records no events then (creating one may allocate).
thread_local bool t_noalloc = false;

cv_status hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return CV_E_HIP;
}
#define CV_HIP(x)                                  \
  do {                                             \
    hipError_t e__ = (x);                          \
    if (e__ != hipSuccess) return hip_fail(e__);   \
  } while (0)

// ------------------------------------------------------ kernel timing
// Optional instrumentation: while enabled, every kernel the library enqueues
// is bracketed by two HIP events recorded on its own stream, together with
// the algorithmic work of that launch (flops, bytes).  Process-global, for
// single-threaded use (benchmarks and profiling runs).
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  double flops, bytes;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_pool;
size_t g_pool_used = 0;
struct ProfAgg {
  const char* name;
  int launches;
  double ms, flops, bytes;
};
std::vector<ProfAgg> g_agg;

hipEvent_t prof_event() {
  if (g_pool_used < g_pool.size()) return g_pool[g_pool_used++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  g_pool.push_back(e);
  ++g_pool_used;
  return e;
}

struct Prof {
  const char* name;
  double flops, bytes;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Prof(const char* n, double f, double by, hipStream_t st) : name(n), flops(f), bytes(by), s(st) {
    if (g_prof_on && !t_noalloc && (a = prof_event())) (void)hipEventRecord(a, s);
  }
  ~Prof() {
    if (!g_prof_on || t_noalloc || !a) return;
    hipEvent_t b = prof_event();
    if (b && hipEventRecord(b, s) == hipSuccess) g_prof.push_back({name, a, b, flops, bytes});
  }
};
// A kernel launch of the hot calls: named (cv_last_kernel) and timed when
// the instrumentation is on; a debug build synchronises the stream and
// checks for an error after every launch.
#ifdef CV_DEBUG
#define CV_DEBUG_SYNC()                            \
  do {                                             \
    CV_HIP(hipStreamSynchronize(s));               \
    CV_HIP(hipGetLastError());                     \
  } while (0)
#else
#define CV_DEBUG_SYNC() \
  do {                  \
  } while (0)
#endif
#define PLAUNCH(name, flops, bytes, call)          \
  do {                                             \
    t_last_kernel = name;                          \
    {                                              \
      Prof pf__(name, (double)(flops), (double)(bytes), s); \
      CV_HIP(call);                                \
    }                                              \
    CV_DEBUG_SYNC();                               \
  } while (0)

// Debug builds: CV_E_NONFINITE if any of the float arrays (pointer, count;
// null pointers skipped) holds a NaN or +-inf, scanned on the device on
// stream s (which is synchronised).  Release builds: CV_OK, nothing read.
struct FArr {
  const float* p;
  size_t n;
};
cv_status debug_finite(hipStream_t s, std::initializer_list<FArr> arrays) {
#ifdef CV_DEBUG
  t_last_kernel = "scan_nonfinite";
  CV_HIP(launch_nonfinite_reset(s));
  for (const FArr& a : arrays)
    if (a.p && a.n) CV_HIP(launch_nonfinite_scan(a.p, a.n, s));
  unsigned found = 0;
  CV_HIP(nonfinite_result(&found, s));
  return found ? CV_E_NONFINITE : CV_OK;
#else
  (void)s;
  (void)arrays;
  return CV_OK;
#endif
}

// Bump allocator over a caller workspace (256-byte aligned slices).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* p) : base((char*)p) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

template <class T>
cv_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return CV_OK;
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) return CV_E_NOMEM;
  return CV_OK;
}

// Layer i (1-based) computed as a direct convolution, or null for a GEMM.
const ConvDesc* conv_of(const cv_net_s* net, int i) {
  return net->is_conv[i - 1] ? &net->conv[i - 1] : nullptr;
}

// Algorithmic float64 flops of one pass of R rows through layer i: the
// multiply-adds of the convolution (every tap, borders included) or of the
// dense product.
double layer_flops(const cv_net_s* net, int i, long long R) {
  if (const ConvDesc* c = conv_of(net, i))
    return 2.0 * R * c->co * c->ho * c->wo * c->ci * c->k * c->k;
  return 2.0 * R * net->n[i] * net->n[i - 1];
}

// Weight bytes one pass reads from memory (float32 matrices, float64 kernels).
double layer_wbytes(const cv_net_s* net, int i) {
  if (const ConvDesc* c = conv_of(net, i)) return 8.0 * c->co * c->ci * c->k * c->k;
  return 4.0 * net->n[i] * net->n[i - 1];
}

// Workspace of one backward pass (rows R = B*M, objective rows M).
// Constraint slots of complete clipping (CV_TEAM_KMAX of the kernels).
constexpr int CA_SLOTS = 64;

struct Bwd {
  double *Om0, *Om1, *Ax, *part, *rowc, *rowerr, *rowcabs, *psiT, *c0, *e0, *cabs0;
  float* trace;
  CvKStat* kst;  // [B, CA_SLOTS] per-constraint box statistics for complete clipping
};

// Row counts a backward pass supports: every per-layer matrix of R rows
// (widest layer below T, and the [R, n_hidden] slope trace) stays under 2^31
// entries; larger batches are split by the caller.
bool rows_fit(const cv_net_s* net, int T, long long R) {
  long long nmax = net->n_hidden;
  for (int i = 0; i < T; ++i) nmax = std::max<long long>(nmax, net->n[i]);
  return R * nmax <= 0x7fffffffLL;
}

size_t bwd_layout(const cv_net_s* net, int T, long long R, int M, int P, bool keepAx, bool trace,
                  void* ws, Bwd* w) {
  const long long B = R / M;
  Carve cv(ws);
  int nmax = 1, ntmax = 1;
  for (int i = 1; i < T; ++i) nmax = std::max(nmax, net->n[i]);
  for (int i = 0; i < T; ++i) ntmax = std::max(ntmax, gemm_ntiles(net->n[i]));
  Bwd x{};
  x.Om0 = cv.take<double>((size_t)R * nmax);
  x.Om1 = cv.take<double>((size_t)R * nmax);
  x.Ax = keepAx ? cv.take<double>((size_t)R * net->n[0]) : nullptr;
  x.part = cv.take<double>((size_t)R * ntmax * 3);
  x.rowc = cv.take<double>(R);
  x.rowerr = cv.take<double>(R);
  x.rowcabs = cv.take<double>(R);
  x.psiT = cv.take<double>((size_t)P * M * net->n[T - 1]);
  x.c0 = cv.take<double>((size_t)P * M);
  x.e0 = cv.take<double>((size_t)P * M);
  x.cabs0 = cv.take<double>((size_t)P * M);
  x.trace = trace ? cv.take<float>((size_t)R * net->n_hidden) : nullptr;
  x.kst = cv.take<CvKStat>((size_t)B * CA_SLOTS);
  if (w) *w = x;
  return cv.off + 256;
}

// CROWN backward pass through layers T..1 of `net` for rows r = (b, m):
// objective C (M x n_T per property, [P, M, n_T]) on z_T, then concretization
// over each box; the root-derived error weights are those of each subdomain's
// property.  Leaves the intercept and the plane's error bound in w.rowc /
// w.rowerr and, when w.Ax is set, the input plane in w.Ax.
// eye = +-1: the objective is +-I with t = 0 (C and t are then not read).
cv_status backward_run(const cv_net_s* net, const cv_root_s* root, CvProps props, int T, int B,
                       int M,
                       const float* C, const float* t, const float* l, const float* u,
                       const float* alpha, double alpha_def, const float* lo, const float* hi,
                       const uint8_t* infeasible, const Bwd& w, float* lb, float* A_out,
                       float* c_out, hipStream_t s, int eye = 0) {
  const int R = B * M;
  const int Nh = net->n_hidden;
  const int nP = net->n[T - 1];
  if (!eye && conv_of(net, T)) return CV_E_UNSUPPORTED;  // a general objective needs a linear layer
  if (eye)
    PLAUNCH("top", 0, 8.0 * props.P * M * nP, launch_top_eye(props.P, M, nP, (double)eye, net->W[T - 1], conv_of(net, T), net->b[T - 1], props, T - 1,
                          w.psiT, w.c0, w.e0, w.cabs0, s));
  else
    PLAUNCH("top", 2.0 * props.P * M * net->n[T] * nP, 8.0 * props.P * M * nP, launch_top(props.P, M, net->n[T], nP, C, t, net->W[T - 1], net->b[T - 1], props, T - 1,
                      w.psiT, w.c0, w.e0, w.cabs0, s));
  // ReLU of hidden layer T-1 (array index T-2)
  PLAUNCH("relax_top", 0, 8.0 * R * nP, launch_relax_top(R, M, nP, Nh, net->off[T - 2], w.psiT, w.c0, w.e0, w.cabs0, l, u, alpha,
                          alpha_def, net->b[T - 2], props, T - 2, w.Om0, w.trace, w.rowc,
                          w.rowerr, w.rowcabs, s));
  double* cur = w.Om0;
  double* nxt = w.Om1;
  for (int i = T - 1; i >= 2; --i) {
    const int K = net->n[i], N = net->n[i - 1];
    const ConvDesc* cd = conv_of(net, i);
    PLAUNCH(cd ? "conv_relax" : "gemm_relax", layer_flops(net, i, R), 8.0 * R * (K + N) + layer_wbytes(net, i), launch_gemm_relax(R, K, N, cur, net->W[i - 1], cd, M, Nh, net->off[i - 2], l, u, alpha,
                             alpha_def, net->b[i - 2], props, i - 2, nxt, w.trace, w.part, net->tune[CV_TUNE_RELAX][i - 1], s));
    PLAUNCH("rowacc", 0, 8.0 * R * (3 * gemm_ntiles(N) + 6), launch_rowacc(R, gemm_ntiles(N), w.part, w.rowc, w.rowerr, w.rowcabs, s));
    std::swap(cur, nxt);
  }
  const int n0 = net->n[0];
  PLAUNCH(conv_of(net, 1) ? "conv_final" : "gemm_final", layer_flops(net, 1, R), 8.0 * R * net->n[1] + (w.Ax ? 8.0 * R * n0 : 0.0) + layer_wbytes(net, 1), launch_gemm_final(R, net->n[1], n0, cur, net->W[0], conv_of(net, 1), M, lo, hi, props, w.Ax, A_out,
                           w.part, net->tune[CV_TUNE_FINAL][0], s));
  PLAUNCH("finalize", 0, 8.0 * R * (2 * gemm_ntiles(n0) + 3), launch_finalize(R, M, gemm_ntiles(n0), w.part, w.rowc, w.rowerr, w.rowcabs,
                         root->gamma_big, infeasible, lb, c_out, s));
  return CV_OK;
}

// The property table of `root` with each subdomain's property index.
CvProps props_of(const cv_root_s* root, const int32_t* pid) {
  const bool single = root && root->P == 1;
  return CvProps{root ? root->dtab : nullptr, pid, root ? root->P : 1,
                 single ? &root->htab : nullptr};
}

cv_status resolve_cons(const cv_root_s* root, const int32_t* pid, const cv_constraints* c,
                       CvCons* out) {
  memset(out, 0, sizeof(*out));
  if (!c) return CV_OK;
  if (c->kmax < 0) return CV_E_SHAPE;
  out->kmax = c->kmax;
  out->count = c->count;
  if (c->kmax == 0) return CV_OK;
  if (c->neuron) {
    if (!root) return CV_E_INVALID;
    if (!c->sign) return CV_E_INVALID;
    out->neuron = c->neuron;
    out->sign = c->sign;
    out->props = props_of(root, pid);
    out->nplanes = root->N;
  } else {
    if (!c->G || !c->h) return CV_E_INVALID;
    out->G = c->G;
    out->h = c->h;
  }
  out->order = c->order;
  return CV_OK;
}

bool finite01(float a) { return a >= 0.0f && a <= 1.0f; }

RootDev root_dev(const cv_root_s* r) {
  RootDev d{};
  d.A_lo = r->A_lo;
  d.A_hi = r->A_hi;
  d.prow = r->prow;
  d.c_lo = r->c_lo;
  d.c_hi = r->c_hi;
  d.l0 = r->l0;
  d.u0 = r->u0;
  d.X0 = r->X0;
  d.uidx = r->uidx;
  d.sidx = r->sidx;
  d.P = r->P_planes;
  d.cP = r->cP;
  d.eP = r->eP;
  d.U = r->U;
  for (int i = 0; i < CV_MAX_LAYERS; ++i) {
    d.wrel[i] = r->wrel[i];
    d.vgemm[i] = r->vgemm[i];
  }
  return d;
}

// (Re)writes the one-entry property table of a single root.
cv_status root_sync_tab(cv_root_s* r) {
  if (!r->dtab) {
    if (hipMalloc((void**)&r->dtab, sizeof(RootDev)) != hipSuccess) {
      r->dtab = nullptr;
      return CV_E_NOMEM;
    }
  }
  r->htab = root_dev(r);
  if (hipMemcpy(r->dtab, &r->htab, sizeof(RootDev), hipMemcpyHostToDevice) != hipSuccess)
    return hip_fail(hipGetLastError());
  r->Umax = r->U;
  return CV_OK;
}

// ---------------------------------------------- allocation-free variant
// Scratch of cv_concretize_planes_static: a file-scope device array, one copy
// on every device the library runs on, held until the process ends.  Host
// code never passes the array's name as an address (in host code it is a
// host-side stand-in); hipGetSymbolAddress, called once per device with that
// device current, gives the device copy's address, which is what the kernels
// receive.
constexpr size_t kStaticScratchBytes = (size_t)CV_CONCRETIZE_PLANES_STATIC_BYTES;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on
// that device).
cv_status static_scratch(void** out) {
  int dev = -1;
  CV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CV_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return CV_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CV_OK;
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char* cv_status_string(cv_status s) {
  switch (s) {
    case CV_OK: return "ok";
    case CV_E_INVALID: return "invalid argument";
    case CV_E_SHAPE: return "inconsistent shape";
    case CV_E_UNSUPPORTED: return "unsupported";
    case CV_E_WORKSPACE: return "workspace too small";
    case CV_E_HIP: return "HIP runtime error";
    case CV_E_NOMEM: return "device allocation failed";
    case CV_E_NONFINITE: return "non-finite input (debug build)";
  }
  return "unknown status";
}

int cv_last_hip_error(void) { return g_last_hip; }
int cv_version(void) { return CV_VERSION; }
#ifdef CV_DEBUG
int cv_debug_build(void) { return 1; }
#else
int cv_debug_build(void) { return 0; }
#endif
const char* cv_last_kernel(void) { return t_last_kernel; }

cv_status cv_net_create(const cv_layer_desc* layers, int n_layers, cv_net* out) {
  if (!layers || !out) return CV_E_INVALID;
  *out = nullptr;
  if (n_layers < 2) return CV_E_UNSUPPORTED;  // at least one hidden ReLU layer
  if (n_layers > CV_MAX_LAYERS) return CV_E_UNSUPPORTED;
  for (int i = 0; i < n_layers; ++i) {
    const cv_layer_desc& d = layers[i];
    if (d.kind != CV_LINEAR && d.kind != CV_CONV2D) return CV_E_INVALID;
    if (!d.W || !d.b) return CV_E_INVALID;
    if (d.kind == CV_CONV2D) {
      if (d.in_c <= 0 || d.in_h <= 0 || d.in_w <= 0 || d.out_c <= 0 || d.kernel <= 0 ||
          d.stride <= 0 || d.pad < 0)
        return CV_E_INVALID;
      const long long oh = (d.in_h + 2LL * d.pad - d.kernel) / d.stride + 1;
      const long long ow = (d.in_w + 2LL * d.pad - d.kernel) / d.stride + 1;
      if (d.in_h + 2LL * d.pad < d.kernel || d.in_w + 2LL * d.pad < d.kernel) return CV_E_SHAPE;
      if (oh != d.out_h || ow != d.out_w) return CV_E_SHAPE;
      if ((long long)d.in_c * d.in_h * d.in_w != d.in_features ||
          (long long)d.out_c * d.out_h * d.out_w != d.out_features)
        return CV_E_SHAPE;
    }
    if (d.in_features <= 0 || d.out_features <= 0) return CV_E_INVALID;
    if (d.kind == CV_LINEAR) {  // kept as a dense matrix and its transpose
      if ((long long)d.in_features * d.out_features > (1LL << 28)) return CV_E_UNSUPPORTED;
    } else {  // kept as its kernel; the objective layer must be linear
      if (i == n_layers - 1) return CV_E_UNSUPPORTED;
      if (d.in_features > (1 << 26) || d.out_features > (1 << 26)) return CV_E_UNSUPPORTED;
    }
    if (i > 0 && d.in_features != layers[i - 1].out_features) return CV_E_SHAPE;
  }
  cv_net_s* net = new cv_net_s();
  net->L = n_layers;
  net->n[0] = layers[0].in_features;
  int acc = 0;
  for (int i = 0; i < n_layers; ++i) {
    const cv_layer_desc& d = layers[i];
    const int no = d.out_features, ni = d.in_features;
    net->n[i + 1] = no;
    net->W[i] = net->Wt[i] = net->b[i] = nullptr;
    net->is_conv[i] = false;
    net->conv[i] = ConvDesc{};
    for (int k = 0; k < 3; ++k) net->tune[k][i] = 0;
    std::vector<float> W, Wt, K, bb;
    if (d.kind == CV_LINEAR) {
      W.assign(d.W, d.W + (size_t)no * ni);
      bb.assign(d.b, d.b + no);
      Wt.resize((size_t)no * ni);
      for (int r = 0; r < no; ++r)
        for (int c = 0; c < ni; ++c) Wt[(size_t)c * no + r] = W[(size_t)r * ni + c];
      if (dev_alloc(&net->W[i], W.size()) || dev_alloc(&net->Wt[i], Wt.size())) {
        cv_net_destroy(net);
        return CV_E_NOMEM;
      }
      if (hipMemcpy(net->W[i], W.data(), W.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(net->Wt[i], Wt.data(), Wt.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        cv_net_destroy(net);
        return hip_fail(hipGetLastError());
      }
    } else {
      // the bias repeats over the output positions (maps flattened channel-major)
      K.assign(d.W, d.W + (size_t)d.out_c * d.in_c * d.kernel * d.kernel);
      bb.resize(no);
      for (int r = 0; r < no; ++r) bb[r] = d.b[r / (d.out_h * d.out_w)];
    }
    if (dev_alloc(&net->b[i], bb.size())) {
      cv_net_destroy(net);
      return CV_E_NOMEM;
    }
    if (hipMemcpy(net->b[i], bb.data(), bb.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      cv_net_destroy(net);
      return hip_fail(hipGetLastError());
    }
    if (d.kind == CV_CONV2D) {
      // Kernels of the direct convolutions: Wb [co][k][k][ci padded] (the
      // transposed convolution's; blocks of its output channels ci are
      // contiguous) and Wf [ci][k][k][co padded] (the forward one's).  The
      // contiguous dimension is padded to 16 (to 64 past 64 channels: the
      // matrix-core tasks take up to 64 output channels), the outer one to a
      // multiple of 4 (the matrix cores contract four channels per step);
      // padding is zero.
      ConvDesc& c = net->conv[i];
      auto pad_out = [](int n) { return n <= 64 ? (n + 15) / 16 * 16 : (n + 63) / 64 * 64; };
      const char* tiled = std::getenv("CV_CONV_TILED");
      c = ConvDesc{d.in_c, d.in_h, d.in_w, d.out_c, d.out_h, d.out_w, d.kernel, d.stride, d.pad,
                   pad_out(d.in_c), pad_out(d.out_c), nullptr, nullptr,
                   tiled != nullptr && tiled[0] == '1'};
      net->is_conv[i] = true;
      const int K = c.k;
      const int pt = c.ptp, pf = c.pfp;
      const int co4 = (c.co + 3) / 4 * 4, ci4 = (c.ci + 3) / 4 * 4;
      std::vector<double> Wb((size_t)co4 * K * K * pt, 0.0), Wf((size_t)ci4 * K * K * pf, 0.0);
      for (int co = 0; co < c.co; ++co)
        for (int ci = 0; ci < c.ci; ++ci)
          for (int ky = 0; ky < K; ++ky)
            for (int kx = 0; kx < K; ++kx) {
              const double v = d.W[(((size_t)co * c.ci + ci) * K + ky) * K + kx];
              Wb[(((size_t)co * K + ky) * K + kx) * pt + ci] = v;
              Wf[(((size_t)ci * K + ky) * K + kx) * pf + co] = v;
            }
      if (dev_alloc(&c.Wb, Wb.size()) || dev_alloc(&c.Wf, Wf.size())) {
        cv_net_destroy(net);
        return CV_E_NOMEM;
      }
      if (hipMemcpy(c.Wb, Wb.data(), Wb.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c.Wf, Wf.data(), Wf.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        cv_net_destroy(net);
        return hip_fail(hipGetLastError());
      }
    }
    net->hW.push_back(std::move(W));
    net->hK.push_back(std::move(K));
    net->hb.push_back(std::move(bb));
    if (i < n_layers - 1) {
      net->off[i] = acc;
      acc += no;
      net->nmax_hidden = std::max(net->nmax_hidden, no);
    }
  }
  net->n_hidden = acc;
  *out = net;
  return CV_OK;
}

cv_status cv_net_destroy(cv_net net) {
  if (!net) return CV_OK;
  for (int i = 0; i < net->L; ++i) {
    if (net->W[i]) (void)hipFree(net->W[i]);
    if (net->Wt[i]) (void)hipFree(net->Wt[i]);
    if (net->b[i]) (void)hipFree(net->b[i]);
    if (net->is_conv[i]) {
      if (net->conv[i].Wb) (void)hipFree(net->conv[i].Wb);
      if (net->conv[i].Wf) (void)hipFree(net->conv[i].Wf);
    }
  }
  if (net->root_ws) (void)hipFree(net->root_ws);
  delete net;
  return CV_OK;
}

// Variants a layer offers: GEMM tiles 32/64/128 x 128 (the adjoint also
// 32 x 256).  A conv layer whose input row fits LDS runs the whole-row
// convolutions: positions per lane of the transposed one (built-in, 1, 2,
// 4), channel block and positions per lane of the forward one (6); a longer
// row the tiled convolutions: the depth of the input staging (built-in, 4,
// 8, 16 channels), the forward one also the other column-tile count.
static int tune_variants(const cv_net_s* net, int kind, int layer) {
  if (net->is_conv[layer - 1]) {
    const ConvDesc& c = net->conv[layer - 1];
    if (kind == CV_TUNE_ADJOINT) return conv_whole_row_layer(c, false) ? 6 : 5;
    return 4;
  }
  return kind == CV_TUNE_ADJOINT ? 4 : 3;
}

static bool tune_layer_valid(const cv_net_s* net, int kind, int layer) {
  if (kind == CV_TUNE_RELAX) return layer >= 2 && layer <= net->L - 1;
  if (kind == CV_TUNE_FINAL) return layer == 1;
  if (kind == CV_TUNE_ADJOINT) return layer >= 1 && layer <= net->L - 1;
  return false;
}

cv_status cv_net_tuning(cv_net net, int kind, int layer, int* variant, int* count) {
  if (!net || !tune_layer_valid(net, kind, layer)) return CV_E_INVALID;
  if (variant) *variant = net->tune[kind][layer - 1];
  if (count) *count = tune_variants(net, kind, layer);
  return CV_OK;
}

cv_status cv_net_set_tuning(cv_net net, int kind, int layer, int variant) {
  if (!net || !tune_layer_valid(net, kind, layer)) return CV_E_INVALID;
  if (variant < 0 || variant >= tune_variants(net, kind, layer)) return CV_E_INVALID;
  net->tune[kind][layer - 1] = (int8_t)variant;
  return CV_OK;
}

cv_status cv_net_autotune(cv_net net, int B, int M, hipStream_t s) {
  if (!net || B <= 0 || M <= 0) return CV_E_INVALID;
  const long long R = (long long)B * M;
  const int L = net->L, Nh = net->n_hidden, n0 = net->n[0];
  int nmax = n0;
  for (int i = 1; i <= L; ++i) nmax = std::max(nmax, net->n[i]);
  int ntmax = 1;
  for (int i = 0; i <= L; ++i) ntmax = std::max(ntmax, gemm_ntiles(net->n[i]));
  double *A0 = nullptr, *A1 = nullptr, *part = nullptr, *wr = nullptr, *X0 = nullptr;
  float *l = nullptr, *u = nullptr, *trace = nullptr, *lo = nullptr, *hi = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    double* ds[] = {A0, A1, part, wr, X0};
    for (double* p : ds)
      if (p) (void)hipFree(p);
    float* fs[] = {l, u, trace, lo, hi};
    for (float* p : fs)
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (dev_alloc(&A0, (size_t)R * nmax) || dev_alloc(&A1, (size_t)R * nmax) ||
      dev_alloc(&part, (size_t)R * ntmax * 3) || dev_alloc(&wr, nmax) || dev_alloc(&X0, n0) ||
      dev_alloc(&l, (size_t)B * Nh) || dev_alloc(&u, (size_t)B * Nh) ||
      dev_alloc(&trace, (size_t)R * Nh) || dev_alloc(&lo, (size_t)B * n0) ||
      dev_alloc(&hi, (size_t)B * n0)) {
    cleanup();
    return CV_E_NOMEM;
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return hip_fail(hipGetLastError());
  }
  // synthetic operands: coefficients in [-1, 1), bounds with unstable neurons
  if (launch_fill_pattern(A0, (size_t)R * nmax, -1.0, 1.0, 1u, s) ||
      launch_fill_pattern(wr, nmax, 0.5, 1.5, 2u, s) || launch_fill_pattern(X0, n0, 0.0, 1.0, 3u, s) ||
      launch_fill_pattern(l, (size_t)B * Nh, -1.0, 0.2, 4u, s) ||
      launch_fill_pattern(u, (size_t)B * Nh, 0.3, 1.5, 5u, s) ||
      launch_fill_pattern(trace, (size_t)R * Nh, -1.0, 1.0, 6u, s) ||
      launch_fill_pattern(lo, (size_t)B * n0, 0.0, 0.4, 7u, s) ||
      launch_fill_pattern(hi, (size_t)B * n0, 0.5, 1.0, 8u, s)) {
    cleanup();
    return hip_fail(hipGetLastError());
  }
  RootDev tmp{};
  tmp.X0 = X0;
  for (int i = 0; i < CV_MAX_LAYERS; ++i) tmp.wrel[i] = wr;
  const CvProps props{nullptr, nullptr, 1, &tmp};
  // average time of 3 launches after a warm-up one
  auto timed = [&](const std::function<hipError_t()>& launch, float* ms) -> hipError_t {
    hipError_t e = launch();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
    for (int rep = 0; rep < 3; ++rep)
      if ((e = launch()) != hipSuccess) return e;
    if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
    return hipEventElapsedTime(ms, e0, e1);
  };
  for (int kind = 0; kind < 3; ++kind) {
    for (int layer = 1; layer <= L; ++layer) {
      if (!tune_layer_valid(net, kind, layer)) continue;
      const int nv = tune_variants(net, kind, layer);
      if (nv < 2) continue;
      const ConvDesc* cd = conv_of(net, layer);
      float best = 0.0f;
      int bestv = 0;
      for (int v = 0; v < nv; ++v) {
        std::function<hipError_t()> launch;
        if (kind == CV_TUNE_RELAX) {
          const int K = net->n[layer], N = net->n[layer - 1];
          launch = [=]() {
            return launch_gemm_relax((int)R, K, N, A0, net->W[layer - 1], cd, M, Nh,
                                     net->off[layer - 2], l, u, nullptr, 0.5, net->b[layer - 2],
                                     props, layer - 2, A1, nullptr, part, v, s);
          };
        } else if (kind == CV_TUNE_FINAL) {
          launch = [=]() {
            return launch_gemm_final((int)R, net->n[1], n0, A0, net->W[0], cd, M, lo, hi, props,
                                     A1, nullptr, part, v, s);
          };
        } else {
          const int K = net->n[layer - 1], N = net->n[layer];
          double* out = layer < L - 1 ? A1 : nullptr;
          launch = [=]() {
            return launch_gemm_adjoint((int)R, K, N, A0, net->Wt[layer - 1], cd, net->b[layer - 1],
                                       M, Nh, net->off[layer - 1], l, u, nullptr, nullptr, 0.5,
                                       trace, nullptr, nullptr, nullptr, nullptr, 0.0, 0.9, 0.999,
                                       1e-8, 1, false, out, v, s);
          };
        }
        float ms = 0.0f;
        const hipError_t e = timed(launch, &ms);
        if (e != hipSuccess) {
          cleanup();
          return hip_fail(e);
        }
        if (v == 0 || ms < best) {
          best = ms;
          bestv = v;
        }
      }
      net->tune[kind][layer - 1] = (int8_t)bestv;
    }
  }
  cleanup();
  return CV_OK;
}

cv_status cv_net_info(cv_net net, int* n_in, int* n_out, int* n_hidden, int* n_layers) {
  if (!net) return CV_E_INVALID;
  if (n_in) *n_in = net->n[0];
  if (n_out) *n_out = net->n[net->L];
  if (n_hidden) *n_hidden = net->n_hidden;
  if (n_layers) *n_layers = net->L;
  return CV_OK;
}

cv_status cv_root_destroy(cv_root r) {
  if (!r) return CV_OK;
  if (r->dtab) (void)hipFree(r->dtab);
  if (!r->members.empty()) {  // a set owns only its table
    delete r;
    return CV_OK;
  }
  float* fs[] = {r->A_lo, r->A_hi, r->l0, r->u0, r->lo0, r->hi0, r->P_planes};
  for (float* p : fs)
    if (p) (void)hipFree(p);
  double* ds[] = {r->c_lo, r->c_hi, r->cP, r->xc0, r->rad0};
  for (double* p : ds)
    if (p) (void)hipFree(p);
  if (r->X0) (void)hipFree(r->X0);
  if (r->eP) (void)hipFree(r->eP);
  if (r->uidx) (void)hipFree(r->uidx);
  if (r->sidx) (void)hipFree(r->sidx);
  if (r->prow) (void)hipFree(r->prow);
  for (int i = 0; i < CV_MAX_LAYERS; ++i) {
    if (r->vgemm[i]) (void)hipFree(r->vgemm[i]);
    if (r->wrel[i]) (void)hipFree(r->wrel[i]);
  }
  delete r;
  return CV_OK;
}

cv_status cv_root_create(cv_net net, const float* lo0, const float* hi0, float alpha0,
                         hipStream_t s, cv_root* out) {
  return cv_root_create_ex(net, lo0, hi0, alpha0, CV_ROOT_PLANES_AUTO, s, out);
}

cv_status cv_root_create_ex(cv_net net, const float* lo0, const float* hi0, float alpha0,
                            int planes, hipStream_t s, cv_root* out) {
  if (!net || !lo0 || !hi0 || !out) return CV_E_INVALID;
  if (!finite01(alpha0)) return CV_E_INVALID;
  if (planes != CV_ROOT_PLANES_AUTO && planes != CV_ROOT_PLANES_ALL &&
      planes != CV_ROOT_PLANES_UNSTABLE)
    return CV_E_INVALID;
  *out = nullptr;
  const int n0 = net->n[0], N = net->n_hidden, L = net->L;
  cv_root_s* r = new cv_root_s();
  for (int i = 0; i < CV_MAX_LAYERS; ++i) r->vgemm[i] = r->wrel[i] = nullptr;
  r->net = net;
  r->n0 = n0;
  r->N = N;
  r->alpha0 = alpha0;
  cv_status st = CV_OK;
  auto fail = [&](cv_status e) {
    cv_root_destroy(r);
    return e;
  };
  if ((st = dev_alloc(&r->A_lo, (size_t)N * n0)) || (st = dev_alloc(&r->A_hi, (size_t)N * n0)) ||
      (st = dev_alloc(&r->c_lo, N)) || (st = dev_alloc(&r->c_hi, N)) ||
      (st = dev_alloc(&r->l0, N)) || (st = dev_alloc(&r->u0, N)) ||
      (st = dev_alloc(&r->lo0, n0)) || (st = dev_alloc(&r->hi0, n0)) ||
      (st = dev_alloc(&r->X0, n0)) || (st = dev_alloc(&r->xc0, n0)) ||
      (st = dev_alloc(&r->rad0, n0)))
    return fail(st);
  // root box and |x| bound
  std::vector<float> hlo(n0), hhi(n0);
  if (hipMemcpyAsync(hlo.data(), lo0, n0 * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hhi.data(), hi0, n0 * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(hip_fail(hipGetLastError()));
  for (int j = 0; j < n0; ++j)
    if (!(hlo[j] <= hhi[j])) return fail(CV_E_INVALID);
  std::vector<double> hX0(n0), hxc(n0), hrad(n0);
  for (int j = 0; j < n0; ++j) {
    hX0[j] = std::max(fabs((double)hlo[j]), fabs((double)hhi[j]));
    hxc[j] = 0.5 * ((double)hlo[j] + (double)hhi[j]);   // exact
    hrad[j] = 0.5 * ((double)hhi[j] - (double)hlo[j]);  // exact
  }
  if (hipMemcpy(r->lo0, hlo.data(), n0 * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->hi0, hhi.data(), n0 * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->X0, hX0.data(), n0 * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->xc0, hxc.data(), n0 * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->rad0, hrad.data(), n0 * 8, hipMemcpyHostToDevice) != hipSuccess)
    return fail(hip_fail(hipGetLastError()));
  int kmax_dot = 2 * n0 + 2;
  for (int i = 0; i <= L; ++i) kmax_dot = std::max(kmax_dot, net->n[i] + 2);
  r->gamma_big = cv_gamma(kmax_dot);

  std::vector<float> hl0(N), hu0(N);
  std::vector<double> H(hX0);  // bound on |input| of the current layer
  auto upload_vec = [&](double** dst, const std::vector<double>& v) -> cv_status {
    cv_status e = dev_alloc(dst, v.size());
    if (e) return e;
    if (hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return hip_fail(hipGetLastError());
    return CV_OK;
  };
  // vgemm of layer i (1-based) from the bound H on its input
  auto make_vgemm = [&](int i) -> cv_status {
    const int no = net->n[i], ni = net->n[i - 1];
    std::vector<double> v(no);
    const std::vector<float>& b = net->hb[i - 1];
    if (const ConvDesc* c = conv_of(net, i)) {  // the taps of each output position
      const std::vector<float>& Kw = net->hK[i - 1];
      const int K = c->k;
      for (int co = 0; co < c->co; ++co)
        for (int oy = 0; oy < c->ho; ++oy)
          for (int ox = 0; ox < c->wo; ++ox) {
            const int k = (co * c->ho + oy) * c->wo + ox;
            double s_ = fabs((double)b[k]);
            for (int ci = 0; ci < c->ci; ++ci)
              for (int ky = 0; ky < K; ++ky) {
                const int iy = oy * c->s - c->p + ky;
                if (iy < 0 || iy >= c->hi) continue;
                for (int kx = 0; kx < K; ++kx) {
                  const int ix = ox * c->s - c->p + kx;
                  if (ix < 0 || ix >= c->wi) continue;
                  s_ += fabs((double)Kw[(((size_t)co * c->ci + ci) * K + ky) * K + kx]) *
                        H[((size_t)ci * c->hi + iy) * c->wi + ix];
                }
              }
            v[k] = s_ * (1.0 + 1e-12);
          }
    } else {
      const std::vector<float>& W = net->hW[i - 1];
      for (int k = 0; k < no; ++k) {
        double s_ = fabs((double)b[k]);
        for (int j = 0; j < ni; ++j) s_ += fabs((double)W[(size_t)k * ni + j]) * H[j];
        v[k] = s_ * (1.0 + 1e-12);
      }
    }
    return upload_vec(&r->vgemm[i - 1], v);
  };
  // after hidden layer i's root bounds are known: wrel_i and the next H
  auto finish_layer = [&](int i) -> cv_status {
    const int no = net->n[i], off = net->off[i - 1];
    if (hipMemcpy(hl0.data() + off, r->l0 + off, no * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hu0.data() + off, r->u0 + off, no * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return hip_fail(hipGetLastError());
    std::vector<double> vg(no), wr(no);
    if (hipMemcpy(vg.data(), r->vgemm[i - 1], no * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return hip_fail(hipGetLastError());
    H.assign(no, 0.0);
    for (int k = 0; k < no; ++k) {
      const double lz = hl0[off + k], uz = hu0[off + k];
      wr[k] = std::max(fabs(lz), fabs(uz)) + vg[k];
      H[k] = std::max(uz, 0.0);
    }
    return upload_vec(&r->wrel[i - 1], wr);
  };

  // hidden layer 1: planes are W1, b1 exactly
  const int n1 = net->n[1];
  if ((st = make_vgemm(1))) return fail(st);
  std::vector<double> hb1(net->hb[0].begin(), net->hb[0].end());
  if ((conv_of(net, 1) ? launch_conv_dense(*conv_of(net, 1), n1, r->A_lo, s)
                       : hipMemcpyAsync(r->A_lo, net->W[0], (size_t)n1 * n0 * 4,
                                        hipMemcpyDeviceToDevice, s)) ||
      hipMemcpyAsync(r->A_hi, r->A_lo, (size_t)n1 * n0 * 4, hipMemcpyDeviceToDevice, s) ||
      hipMemcpy(r->c_lo, hb1.data(), n1 * 8, hipMemcpyHostToDevice) ||
      hipMemcpy(r->c_hi, hb1.data(), n1 * 8, hipMemcpyHostToDevice))
    return fail(hip_fail(hipGetLastError()));
  if (launch_concretize_rows(n1, n0, r->A_lo, r->c_lo, r->lo0, r->hi0, 0, r->l0, s) ||
      launch_concretize_rows(n1, n0, r->A_hi, r->c_hi, r->lo0, r->hi0, 1, r->u0, s) ||
      hipStreamSynchronize(s))
    return fail(hip_fail(hipGetLastError()));
  if ((st = finish_layer(1))) return fail(st);

  // deeper hidden layers: CROWN with objectives +I (lower) and -I (upper),
  // in the net's cached working memory (sized for the largest layer once,
  // then reused by every root of the net)
  size_t need = 0;
  for (int i = 2; i <= L - 1; ++i) {
    if (!rows_fit(net, i, net->n[i])) return fail(CV_E_UNSUPPORTED);
    need = std::max(need, bwd_layout(net, i, net->n[i], net->n[i], 1, true, false, nullptr,
                                     nullptr) + (size_t)net->n[i] * 4 + 256);
  }
  if (need > net->root_ws_bytes) {
    if (net->root_ws) (void)hipFree(net->root_ws);
    net->root_ws = nullptr;
    net->root_ws_bytes = 0;
    if (hipMalloc(&net->root_ws, need) != hipSuccess) {
      net->root_ws = nullptr;
      return fail(CV_E_NOMEM);
    }
    net->root_ws_bytes = need;
  }
  for (int i = 2; i <= L - 1; ++i) {
    const int ni = net->n[i], off = net->off[i - 1];
    if ((st = make_vgemm(i))) return fail(st);
    Bwd w;
    const size_t used = bwd_layout(net, i, ni, ni, 1, true, false, net->root_ws, &w);
    Carve cv((char*)net->root_ws + used);
    float* lbtmp = cv.take<float>(ni);
    for (int side = 0; side < 2; ++side) {
      if ((st = root_sync_tab(r))) return fail(st);
      st = backward_run(net, r, props_of(r, nullptr), i, 1, ni, nullptr, nullptr, r->l0, r->u0,
                        nullptr, alpha0, r->lo0, r->hi0, nullptr, w, lbtmp, nullptr, nullptr, s,
                        side ? -1 : 1);
      if (st) return fail(st);
      float* Adst = (side ? r->A_hi : r->A_lo) + (size_t)off * n0;
      double* cdst = (side ? r->c_hi : r->c_lo) + off;
      if (launch_root_store_planes(ni, n0, w.Ax, w.rowc, w.rowerr, r->xc0, r->rad0, side, Adst,
                                   cdst, s))
        return fail(hip_fail(hipGetLastError()));
    }
    if (launch_concretize_rows(ni, n0, r->A_lo + (size_t)off * n0, r->c_lo + off, r->lo0, r->hi0,
                               0, r->l0 + off, s) ||
        launch_concretize_rows(ni, n0, r->A_hi + (size_t)off * n0, r->c_hi + off, r->lo0, r->hi0,
                               1, r->u0 + off, s) ||
        hipStreamSynchronize(s))
      return fail(hip_fail(hipGetLastError()));
    if ((st = finish_layer(i))) return fail(st);
  }
  if ((st = make_vgemm(L))) return fail(st);

  // unstable / stable lists and the packed plane matrix
  std::vector<int32_t> us, ss;
  for (int j = 0; j < N; ++j) (hl0[j] < 0.0f && hu0[j] > 0.0f ? us : ss).push_back(j);
  r->U = (int)us.size();
  if ((st = dev_alloc(&r->uidx, us.size())) || (st = dev_alloc(&r->sidx, ss.size())) ||
      (st = dev_alloc(&r->P_planes, (size_t)2 * n0 * 2 * r->U)) || (st = dev_alloc(&r->cP, 2 * r->U)) ||
      (st = dev_alloc(&r->eP, 2 * r->U)))
    return fail(st);
  if ((!us.empty() && hipMemcpy(r->uidx, us.data(), us.size() * 4, hipMemcpyHostToDevice)) ||
      (!ss.empty() && hipMemcpy(r->sidx, ss.data(), ss.size() * 4, hipMemcpyHostToDevice)))
    return fail(hip_fail(hipGetLastError()));
  if (launch_build_P(n0, r->U, r->uidx, r->A_lo, r->A_hi, r->c_lo, r->c_hi, r->X0, r->P_planes,
                     r->cP, r->eP, s) ||
      hipStreamSynchronize(s))
    return fail(hip_fail(hipGetLastError()));
  // keep the planes of the root-unstable neurons only (row q: neuron uidx[q])
  // when asked, or by default when all planes would pass 2^28 coefficients
  // per side
  const bool compact = planes == CV_ROOT_PLANES_UNSTABLE ||
                       (planes == CV_ROOT_PLANES_AUTO && (long long)N * n0 > (1LL << 28));
  if (compact) {
    std::vector<int32_t> prow(N, -1);
    for (int q = 0; q < r->U; ++q) prow[us[q]] = q;
    float *clo = nullptr, *chi = nullptr;
    if ((st = dev_alloc(&r->prow, N)) || (st = dev_alloc(&clo, (size_t)r->U * n0)) ||
        (st = dev_alloc(&chi, (size_t)r->U * n0))) {
      if (clo) (void)hipFree(clo);
      return fail(st);
    }
    if (hipMemcpy(r->prow, prow.data(), (size_t)N * 4, hipMemcpyHostToDevice) != hipSuccess ||
        launch_gather_rows(r->U, n0, r->uidx, r->A_lo, clo, s) != hipSuccess ||
        launch_gather_rows(r->U, n0, r->uidx, r->A_hi, chi, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      if (clo) (void)hipFree(clo);
      if (chi) (void)hipFree(chi);
      return fail(hip_fail(hipGetLastError()));
    }
    (void)hipFree(r->A_lo);
    (void)hipFree(r->A_hi);
    r->A_lo = clo;
    r->A_hi = chi;
  }
  if ((st = root_sync_tab(r))) return fail(st);
  *out = r;
  return CV_OK;
}

cv_status cv_rootset_create(const cv_root* roots, int P, cv_root* out) {
  if (!roots || !out || P < 1) return CV_E_INVALID;
  *out = nullptr;
  std::vector<RootDev> tab(P);
  for (int p = 0; p < P; ++p) {
    const cv_root_s* m = roots[p];
    if (!m || !m->members.empty()) return CV_E_INVALID;  // members are single roots
    if (m->net != roots[0]->net) return CV_E_INVALID;
    tab[p] = root_dev(m);
  }
  cv_root_s* r = new cv_root_s();
  for (int i = 0; i < CV_MAX_LAYERS; ++i) r->vgemm[i] = r->wrel[i] = nullptr;
  const cv_root_s* r0 = roots[0];
  r->net = r0->net;
  r->n0 = r0->n0;
  r->N = r0->N;
  r->alpha0 = r0->alpha0;
  r->gamma_big = r0->gamma_big;  // depends on the layer widths only
  r->P = P;
  r->U = -1;
  // a set of one property takes the single-property launch paths, which
  // read the host copy of its table entry
  r->htab = tab[0];
  for (int p = 0; p < P; ++p) {
    r->members.push_back(roots[p]);
    r->Umax = std::max(r->Umax, roots[p]->U);
  }
  if (hipMalloc((void**)&r->dtab, sizeof(RootDev) * P) != hipSuccess) {
    r->dtab = nullptr;
    cv_root_destroy(r);
    return CV_E_NOMEM;
  }
  if (hipMemcpy(r->dtab, tab.data(), sizeof(RootDev) * P, hipMemcpyHostToDevice) != hipSuccess) {
    cv_root_destroy(r);
    return hip_fail(hipGetLastError());
  }
  *out = r;
  return CV_OK;
}

cv_status cv_root_count(cv_root r, int* P) {
  if (!r || !P) return CV_E_INVALID;
  *P = r->P;
  return CV_OK;
}

cv_status cv_root_bounds(cv_root r, float* l0, float* u0, hipStream_t s) {
  if (!r || !l0 || !u0 || !r->members.empty()) return CV_E_INVALID;
  CV_HIP(hipMemcpyAsync(l0, r->l0, (size_t)r->N * 4, hipMemcpyDeviceToDevice, s));
  CV_HIP(hipMemcpyAsync(u0, r->u0, (size_t)r->N * 4, hipMemcpyDeviceToDevice, s));
  return CV_OK;
}

cv_status cv_root_planes(cv_root r, float* A_lo, float* c_lo, float* A_hi, float* c_hi,
                         hipStream_t s) {
  if (!r || !A_lo || !c_lo || !A_hi || !c_hi || !r->members.empty()) return CV_E_INVALID;
  if (r->prow) return CV_E_UNSUPPORTED;  // only the unstable neurons' planes are kept
  const size_t na = (size_t)r->N * r->n0 * 4;
  CV_HIP(hipMemcpyAsync(A_lo, r->A_lo, na, hipMemcpyDeviceToDevice, s));
  CV_HIP(hipMemcpyAsync(A_hi, r->A_hi, na, hipMemcpyDeviceToDevice, s));
  CV_HIP(launch_round_intercepts(r->N, r->c_lo, 0, c_lo, s));
  CV_HIP(launch_round_intercepts(r->N, r->c_hi, 1, c_hi, s));
  return CV_OK;
}

cv_status cv_root_unstable_count(cv_root r, int* count) {
  if (!r || !count || !r->members.empty()) return CV_E_INVALID;
  *count = r->U;
  return CV_OK;
}

cv_status cv_clip_domains(cv_root root, const int32_t* pid, int B, int n,
                          const cv_constraints* cons, float* lo, float* hi, uint8_t* infeasible,
                          int mode, hipStream_t s) {
  if (B < 0 || n <= 0) return CV_E_SHAPE;
  if (mode != CV_CLIP_PARALLEL && mode != CV_CLIP_SEQUENTIAL) return CV_E_INVALID;
  if (B == 0) return CV_OK;
  if (!cons || !lo || !hi || !infeasible) return CV_E_INVALID;
  if (n > 4096) return CV_E_UNSUPPORTED;
  if (cons->neuron && root && root->n0 != n) return CV_E_SHAPE;
  CvCons c;
  cv_status st = resolve_cons(root, pid, cons, &c);
  if (st) return st;
  if ((st = debug_finite(s, {{lo, (size_t)B * n}, {hi, (size_t)B * n}}))) return st;
  PLAUNCH("clip", 0, 16.0 * B * n + 4.0 * B * c.kmax * n, launch_clip(B, n, c, lo, hi, infeasible, mode, s));
  return CV_OK;
}

cv_status cv_constraint_order(cv_root root, const int32_t* pid, int B, int n,
                              const cv_constraints* cons, const float* lo, const float* hi,
                              int32_t* order, hipStream_t s) {
  if (B < 0 || n <= 0) return CV_E_SHAPE;
  if (!cons) return CV_E_INVALID;
  if (B == 0 || cons->kmax == 0) return CV_OK;
  if (!lo || !hi || !order) return CV_E_INVALID;
  if (cons->kmax > 64) return CV_E_UNSUPPORTED;
  if (cons->neuron && root && root->n0 != n) return CV_E_SHAPE;
  CvCons c;
  cv_status st = resolve_cons(root, pid, cons, &c);
  if (st) return st;
  c.order = nullptr;
  PLAUNCH("cons_order", 0, 8.0 * B * n + 4.0 * B * c.kmax * n, launch_cons_order(B, n, c, lo, hi, order, s));
  return CV_OK;
}

cv_status cv_concretize_planes_workspace(cv_root root, int B, int complete, size_t* bytes) {
  if (!root || !bytes || B < 0) return CV_E_INVALID;
  *bytes = complete ? (size_t)B * root->Umax * 2 * sizeof(float) + (size_t)B * root->N +
                         (size_t)B * CA_SLOTS * sizeof(CvKStat) + 1024
                   : 0;
  return CV_OK;
}

cv_status cv_concretize_planes(cv_root root, const int32_t* pid, int B, const float* lo,
                               const float* hi, const cv_constraints* splits, int complete,
                               int passes, int topk,
                               const float* weight, float* l, float* u, uint8_t* infeasible,
                               uint8_t* select, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!root || B < 0) return CV_E_INVALID;
  if (B == 0) return CV_OK;
  if (!lo || !hi || !l || !u || !infeasible) return CV_E_INVALID;
  if (splits && splits->kmax > 0 && splits->neuron && !splits->sign) return CV_E_INVALID;
  if (splits && splits->kmax > 0 && !splits->neuron && (!splits->G || !splits->h))
    return CV_E_INVALID;
  if (complete && passes < 1) return CV_E_INVALID;
  if (complete && topk >= 0 && !weight) return CV_E_INVALID;
  size_t need = 0;
  cv_concretize_planes_workspace(root, B, complete, &need);
  if (complete && ws_bytes < need) return CV_E_WORKSPACE;
  if (complete && root->n0 > 4096) return CV_E_UNSUPPORTED;
  CvCons sp;
  cv_status st = resolve_cons(root, pid, splits, &sp);
  if (st) return st;
  if ((st = debug_finite(s, {{lo, (size_t)B * root->n0}, {hi, (size_t)B * root->n0}}))) return st;
  const CvProps props = props_of(root, pid);
  const int Nh = root->N, U = root->Umax;
  int Umin = U;
  for (const cv_root_s* m : root->members) Umin = std::min(Umin, m->U);
  // algorithmic work at the widest property (exact for a single root)
  PLAUNCH("fill_stable", 0, 8.0 * B * (Nh - U), launch_fill_stable(B, Nh, Nh - Umin, props, l, u, s));
  PLAUNCH("gemm_planes", 2.0 * B * (2.0 * root->n0) * (2.0 * U), 8.0 * B * root->n0 + 8.0 * B * U + 16.0 * root->n0 * U, launch_gemm_planes(B, root->n0, U, lo, hi, props, Nh, l, u, s));
  if (splits && splits->kmax > 0 && splits->neuron) PLAUNCH("split_fix", 0, 8.0 * B * splits->kmax, launch_split_fix(B, Nh, sp, l, u, infeasible, s));
  if (complete && splits && splits->kmax > 0 && U > 0) {
    Carve cv(ws);
    float* Ltmp = cv.take<float>((size_t)B * U * 2);
    uint8_t* sel = nullptr;
    if (topk >= 0) {
      // top-k unstable neurons per layer by the BaBSR intercept score
      sel = select ? select : cv.take<uint8_t>((size_t)B * Nh);
      const cv_net_s* net = root->net;
      const int nl = net->L - 1;
      PLAUNCH("select_topk", 0, 8.0 * B * Nh + 1.0 * B * Nh, launch_select_topk(B, Nh, nl, net->off, net->n + 1, l, u, weight, props, topk, sel, s));
    }
    if (sp.kmax <= CA_SLOTS) {  // statistics of each (subdomain, constraint), shared by its neurons
      CvKStat* kst = cv.take<CvKStat>((size_t)B * CA_SLOTS);
      PLAUNCH("cons_stats", 0, 8.0 * B * root->n0 + 4.0 * B * sp.kmax * root->n0, launch_cons_stats(B, root->n0, sp, lo, hi, kst, s));
      sp.kstats = kst;
    }
    PLAUNCH("ca_neurons", 0, 8.0 * B * U * root->n0, launch_ca_neurons(B, U, root->n0, props, sp, passes, lo, hi, l, u, Nh, infeasible, sel, Ltmp, s));
    PLAUNCH("merge_neurons", 0, 16.0 * B * U, launch_merge_neurons(B, U, props, Nh, Ltmp, l, u, infeasible, s));
  }
  return CV_OK;
}

cv_status cv_concretize_planes_static(cv_root root, const int32_t* pid, int B, const float* lo,
                                      const float* hi, const cv_constraints* splits, int complete,
                                      int passes, int topk, const float* weight, float* l,
                                      float* u, uint8_t* infeasible, uint8_t* select,
                                      hipStream_t s) {
  if (!root || B < 0) return CV_E_INVALID;
  size_t need = 0;
  cv_status st = cv_concretize_planes_workspace(root, B, complete, &need);
  if (st) return st;
  if (need > kStaticScratchBytes) return CV_E_WORKSPACE;
  void* ws = nullptr;
  if (need > 0 && (st = static_scratch(&ws))) return st;
  t_noalloc = true;
  st = cv_concretize_planes(root, pid, B, lo, hi, splits, complete, passes, topk, weight, l, u,
                            infeasible, select, ws, need > 0 ? kStaticScratchBytes : 0, s);
  t_noalloc = false;
  return st;
}

cv_status cv_babsr_weights_workspace(cv_net net, int M, size_t* bytes) {
  if (!net || !bytes || M <= 0) return CV_E_INVALID;
  *bytes = bwd_layout(net, net->L, M, M, 1, false, true, nullptr, nullptr) + (size_t)M * 4 + 256;
  return CV_OK;
}

cv_status cv_babsr_weights(cv_net net, cv_root root, int M, const float* C, const float* t,
                           float* weight, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!net || !root || M <= 0 || !C || !t || !weight) return CV_E_INVALID;
  if (root->net != net) return CV_E_INVALID;
  size_t need = 0;
  cv_babsr_weights_workspace(net, M, &need);
  if (!ws || ws_bytes < need) return CV_E_WORKSPACE;
  Bwd w;
  const size_t used = bwd_layout(net, net->L, M, M, 1, false, true, ws, &w);
  float* lbtmp = Carve((char*)ws + used).take<float>(M);
  // per property: one backward pass over its root box with its root bounds and slope
  const int nL = net->n[net->L], Nh = net->n_hidden;
  for (int p = 0; p < root->P; ++p) {
    const cv_root_s* m = root->members.empty() ? root : root->members[p];
    cv_status st = backward_run(net, m, props_of(m, nullptr), net->L, 1, M, C + (size_t)p * M * nL,
                                t + (size_t)p * M, m->l0, m->u0, nullptr, m->alpha0, m->lo0,
                                m->hi0, nullptr, w, lbtmp, nullptr, nullptr, s);
    if (st) return st;
    PLAUNCH("babsr_weight", 0, 4.0 * M * Nh, launch_babsr_weight(M, Nh, w.trace, weight + (size_t)p * Nh, s));
  }
  return CV_OK;
}

cv_status cv_intermediate_bounds_workspace(cv_net net, int B, size_t* bytes) {
  if (!net || !bytes || B < 0) return CV_E_INVALID;
  size_t best = 0;
  int nmax = 1;
  for (int i = 2; i <= net->L - 1; ++i) {
    const int ni = net->n[i];
    if (!rows_fit(net, i, (long long)B * ni)) return CV_E_UNSUPPORTED;
    nmax = std::max(nmax, ni);
    best = std::max(best, bwd_layout(net, i, (long long)B * ni, ni, 1, false, false, nullptr, nullptr));
  }
  *bytes = best + 2 * (size_t)B * nmax * 4 + 1024;
  return CV_OK;
}

cv_status cv_intermediate_bounds(cv_net net, cv_root root, int B, const float* lo, const float* hi,
                                 float* l, float* u, uint8_t* infeasible, void* ws,
                                 size_t ws_bytes, hipStream_t s) {
  if (!net || !root || B < 0) return CV_E_INVALID;
  if (root->net != net) return CV_E_INVALID;
  if (!root->members.empty()) return CV_E_UNSUPPORTED;
  if (B == 0) return CV_OK;
  if (!lo || !hi || !l || !u) return CV_E_INVALID;
  size_t need = 0;
  if (cv_status e = cv_intermediate_bounds_workspace(net, B, &need)) return e;
  if (!ws || ws_bytes < need) return CV_E_WORKSPACE;
  const int Nh = net->n_hidden;
  for (int i = 2; i <= net->L - 1; ++i) {
    const int ni = net->n[i];
    Bwd w;
    const size_t used = bwd_layout(net, i, (long long)B * ni, ni, 1, false, false, ws, &w);
    Carve cv((char*)ws + used);
    float* lbl = cv.take<float>((size_t)B * ni);
    float* lbn = cv.take<float>((size_t)B * ni);
    for (int side = 0; side < 2; ++side) {  // objectives +I, then -I
      cv_status st = backward_run(net, root, props_of(root, nullptr), i, B, ni, nullptr, nullptr, l, u,
                                  nullptr, root->alpha0, lo, hi, infeasible, w,
                                  side ? lbn : lbl, nullptr, nullptr, s, side ? -1 : 1);
      if (st) return st;
    }
    PLAUNCH("merge_layer", 0, 16.0 * B * ni, launch_merge_layer(B, ni, Nh, net->off[i - 1], lbl, lbn, l, u, infeasible, s));
  }
  return CV_OK;
}

cv_status cv_branch_relu(cv_root root, const int32_t* pid, int B, const float* l, const float* u,
                         const float* weight,
                         const cv_constraints* splits, const float* lo, const float* hi,
                         int kmax_out, int32_t* chosen, int32_t* neuron2, int8_t* sign2,
                         int32_t* count2, float* lo2, float* hi2, hipStream_t s) {
  if (!root || B < 0) return CV_E_INVALID;
  if (B == 0) return CV_OK;
  if (!l || !u || !weight || !splits || !lo || !hi || !chosen || !neuron2 || !sign2 || !count2 ||
      !lo2 || !hi2)
    return CV_E_INVALID;
  if (splits->kmax > 0 && (!splits->neuron || !splits->sign)) return CV_E_INVALID;
  if (kmax_out < splits->kmax || kmax_out < 1) return CV_E_SHAPE;
  PLAUNCH("branch_relu", 0, 8.0 * B * root->N + 16.0 * B * root->n0, launch_branch_relu(B, root->N, l, u, weight, props_of(root, pid), splits->kmax, splits->neuron, splits->sign,
                             splits->count, root->n0, lo, hi, kmax_out, chosen, neuron2, sign2,
                             count2, lo2, hi2, s));
  return CV_OK;
}

cv_status cv_branch_input(int B, int M, int n, const float* lo, const float* hi, const float* A,
                          int32_t* dim, float* lo2, float* hi2, hipStream_t s) {
  if (B < 0 || M <= 0 || n <= 0) return CV_E_SHAPE;
  if (B == 0) return CV_OK;
  if (!lo || !hi || !A || !dim || !lo2 || !hi2) return CV_E_INVALID;
  PLAUNCH("branch_input", 0, 4.0 * B * M * n + 24.0 * B * n, launch_branch_input(B, M, n, lo, hi, A, dim, lo2, hi2, s));
  return CV_OK;
}

cv_status cv_concretize(cv_root root, const int32_t* pid, int B, int P, int n, const float* A,
                        int A_shared,
                        const float* c, const float* lo, const float* hi,
                        const cv_constraints* cons, int passes, float* lb, float* ub, float* beta,
                        uint8_t* infeasible, hipStream_t s) {
  if (B < 0 || P < 0 || n <= 0) return CV_E_SHAPE;
  if ((long long)B * P == 0) return CV_OK;
  if (!A || !c || !lo || !hi || !lb) return CV_E_INVALID;
  if (n > 4096) return CV_E_UNSUPPORTED;
  if (cons && passes < 1) return CV_E_INVALID;
  if (cons && cons->neuron && root && root->n0 != n) return CV_E_SHAPE;
  if (beta && !cons) return CV_E_INVALID;
  CvCons cc;
  cv_status st = resolve_cons(root, pid, cons, &cc);
  if (st) return st;
  const size_t na = (A_shared ? (size_t)P : (size_t)B * P);
  if ((st = debug_finite(s, {{A, na * n}, {c, na}, {lo, (size_t)B * n}, {hi, (size_t)B * n}})))
    return st;
  PLAUNCH("ca_generic", 0, 4.0 * B * P * n + 8.0 * B * n, launch_ca_generic(B, P, n, A, A_shared, c, lo, hi, cons ? &cc : nullptr, passes, lb, ub,
                           beta, infeasible, s));
  return CV_OK;
}

// Debug scan of the inputs of a bound propagation or slope step (alpha only
// where it is read).
cv_status debug_prop_inputs(const cv_net_s* net, const cv_root_s* root, int B, int M, const float* C,
                            const float* t, const float* l, const float* u, const float* alpha,
                            const float* lo, const float* hi, hipStream_t s) {
  const size_t PM = (size_t)root->P * M, BH = (size_t)B * net->n_hidden, B0 = (size_t)B * net->n[0];
  return debug_finite(s, {{C, PM * net->n[net->L]}, {t, PM}, {l, BH}, {u, BH},
                          {alpha, BH * M}, {lo, B0}, {hi, B0}});
}

static cv_status check_prop(cv_net net, cv_root root, int B, int M, const float* C, const float* t,
                            const float* l, const float* u, const float* lo, const float* hi,
                            const float* lb) {
  if (!net || !root || B < 0 || M <= 0) return CV_E_INVALID;
  if (root->net != net) return CV_E_INVALID;
  if (B == 0) return CV_OK;
  if (!C || !t || !l || !u || !lo || !hi || !lb) return CV_E_INVALID;
  if (net->n[0] > 4096) return CV_E_UNSUPPORTED;
  return CV_OK;
}

cv_status cv_bound_propagate_workspace(cv_net net, int P, int B, int M, size_t* bytes) {
  if (!net || !bytes || B < 0 || M <= 0 || P < 1) return CV_E_INVALID;
  if (!rows_fit(net, net->L, (long long)B * M)) return CV_E_UNSUPPORTED;
  *bytes = bwd_layout(net, net->L, (long long)B * M, M, P, true, false, nullptr, nullptr);
  return CV_OK;
}

cv_status cv_bound_propagate(cv_net net, int B, int M, const float* C, const float* t,
                             const float* l, const float* u, const float* alpha,
                             float alpha_default, const float* lo, const float* hi,
                             uint8_t* infeasible, cv_root root, const int32_t* pid,
                             const cv_constraints* cons, int passes, float* lb, float* A_out,
                             float* c_out, void* ws, size_t ws_bytes, hipStream_t s) {
  cv_status st = check_prop(net, root, B, M, C, t, l, u, lo, hi, lb);
  if (st || B == 0) return st;
  if (!alpha && !finite01(alpha_default)) return CV_E_INVALID;
  if (cons && passes < 1) return CV_E_INVALID;
  if ((A_out == nullptr) != (c_out == nullptr)) return CV_E_INVALID;
  size_t need = 0;
  if ((st = cv_bound_propagate_workspace(net, root->P, B, M, &need))) return st;
  if (!ws || ws_bytes < need) return CV_E_WORKSPACE;
  CvCons cc;
  if ((st = resolve_cons(root, pid, cons, &cc))) return st;
  if ((st = debug_prop_inputs(net, root, B, M, C, t, l, u, alpha, lo, hi, s))) return st;
  Bwd w;
  bwd_layout(net, net->L, (long long)B * M, M, root->P, true, false, ws, &w);
  st = backward_run(net, root, props_of(root, pid), net->L, B, M, C, t, l, u, alpha,
                    alpha_default, lo, hi, infeasible, w, lb, A_out, c_out, s);
  if (st) return st;
  if (cons && cons->kmax > 0 && cc.kmax <= CA_SLOTS) {
    PLAUNCH("cons_stats", 0, 8.0 * B * net->n[0] + 4.0 * B * cc.kmax * net->n[0], launch_cons_stats(B, net->n[0], cc, lo, hi, w.kst, s));
    cc.kstats = w.kst;
  }
  if (cons && cons->kmax > 0)
    PLAUNCH("ca_rows", 0, 8.0 * B * M * net->n[0] + 8.0 * B * net->n[0], launch_ca_rows(B * M, M, net->n[0], cc, passes, w.Ax, w.rowc, w.rowerr, lo, hi,
                          infeasible, lb, nullptr, 0, nullptr, 0, s));
  return CV_OK;
}

cv_status cv_alpha_step_workspace(cv_net net, int P, int B, int M, size_t* bytes) {
  if (!net || !bytes || B < 0 || M <= 0 || P < 1) return CV_E_INVALID;
  if (!rows_fit(net, net->L, (long long)B * M)) return CV_E_UNSUPPORTED;
  *bytes = bwd_layout(net, net->L, (long long)B * M, M, P, true, true, nullptr, nullptr);
  return CV_OK;
}

cv_status cv_alpha_step(cv_net net, int B, int M, const float* C, const float* t, const float* l,
                        const float* u, float* alpha, float alpha_init, const float* lo,
                        const float* hi, uint8_t* infeasible, cv_root root, const int32_t* pid,
                        const cv_constraints* cons, int passes,
                        float* adam_m, float* adam_v, int step, float lr, float beta1, float beta2,
                        float eps, float* lb, float* best, float* grad, void* ws, size_t ws_bytes,
                        hipStream_t s) {
  cv_status st = check_prop(net, root, B, M, C, t, l, u, lo, hi, lb);
  if (st || B == 0) return st;
  if (!alpha) return CV_E_INVALID;
  if (cons && passes < 1) return CV_E_INVALID;
  if (lr < 0.0f || !(lr == lr)) return CV_E_INVALID;
  if (step < 1) return CV_E_INVALID;
  if (lr > 0.0f) {
    if (!adam_m || !adam_v) return CV_E_INVALID;
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
      return CV_E_INVALID;
  }
  // step 1 starts an optimisation: the slopes are alpha_init when it is in
  // [0, 1] (alpha is then only written) and Adam's moments are zero
  const bool init = step == 1 && finite01(alpha_init);
  if (!init && !(alpha_init < 0.0f)) return CV_E_INVALID;
  size_t need = 0;
  if ((st = cv_alpha_step_workspace(net, root->P, B, M, &need))) return st;
  if (!ws || ws_bytes < need) return CV_E_WORKSPACE;
  CvCons cc;
  if ((st = resolve_cons(root, pid, cons, &cc))) return st;
  if ((st = debug_prop_inputs(net, root, B, M, C, t, l, u, init ? nullptr : alpha, lo, hi, s)))
    return st;
  Bwd w;
  const int R = B * M;
  bwd_layout(net, net->L, R, M, root->P, true, true, ws, &w);
  st = backward_run(net, root, props_of(root, pid), net->L, B, M, C, t, l, u,
                    init ? nullptr : alpha, init ? (double)alpha_init : 0.0, lo, hi, infeasible,
                    w, lb, nullptr, nullptr, s);
  if (st) return st;
  // complete clipping (or plain concretization) leaves the minimising corner
  // x* of the final dual in w.Ax: the adjoint of the bound w.r.t. the plane;
  // it also folds the bound into the running best
  CvCons none{};
  if (cons && cons->kmax > 0 && cc.kmax <= CA_SLOTS) {
    PLAUNCH("cons_stats", 0, 8.0 * B * net->n[0] + 4.0 * B * cc.kmax * net->n[0], launch_cons_stats(B, net->n[0], cc, lo, hi, w.kst, s));
    cc.kstats = w.kst;
  }
  PLAUNCH("ca_rows", 0, 16.0 * R * net->n[0] + 8.0 * B * net->n[0], launch_ca_rows(R, M, net->n[0], (cons && cons->kmax > 0) ? cc : none, passes,
                        w.Ax, w.rowc, w.rowerr, lo, hi, infeasible, lb, nullptr, 1, best,
                        step == 1 ? 1 : 0, s));
  const double dlr = lr;
  double* cur = w.Ax;
  double* bufs[2] = {w.Om0, w.Om1};
  for (int k = 1; k <= net->L - 1; ++k) {
    const int K = net->n[k - 1], N = net->n[k];
    double* out = (k < net->L - 1) ? bufs[(k - 1) & 1] : nullptr;
    const ConvDesc* cd = conv_of(net, k);
    PLAUNCH(cd ? "conv_adjoint" : "gemm_adjoint", layer_flops(net, k, R), 8.0 * R * (K + (out ? N : 0)) + 28.0 * R * N + layer_wbytes(net, k), launch_gemm_adjoint(R, K, N, cur, net->Wt[k - 1], cd, net->b[k - 1], M, net->n_hidden,
                               net->off[k - 1], l, u, alpha, init ? nullptr : alpha,
                               init ? (double)alpha_init : 0.0, w.trace, infeasible, grad,
                               adam_m, adam_v, dlr, beta1, beta2, eps, step, step == 1, out,
                               net->tune[CV_TUNE_ADJOINT][k - 1], s));
    cur = out;
  }
  return CV_OK;
}

cv_status cv_measure_peaks(double* hbm_gbs, double* f64_mfma_tflops, hipStream_t s) {
  if (!hbm_gbs || !f64_mfma_tflops) return CV_E_INVALID;
  const size_t bytes = (size_t)1 << 30;
  const int blocks = 2048, iters = 20000;
  void *src = nullptr, *dst = nullptr;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  cv_status st = CV_OK;
  auto fail = [&](hipError_t e) {
    if (e != hipSuccess && st == CV_OK) st = hip_fail(e);
    return e != hipSuccess;
  };
  if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, bytes) != hipSuccess ||
      hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(double)) != hipSuccess) {
    st = CV_E_NOMEM;
  }
  if (st == CV_OK && !fail(hipEventCreate(&e0)) && !fail(hipEventCreate(&e1)) &&
      !fail(hipMemsetAsync(src, 0, bytes, s))) {
    float best = 0.0f;
    for (int rep = 0; rep < 6 && st == CV_OK; ++rep) {  // first run warms up
      float ms = 0.0f;
      if (fail(hipEventRecord(e0, s)) || fail(launch_probe_copy(src, dst, bytes, s)) ||
          fail(hipEventRecord(e1, s)) || fail(hipEventSynchronize(e1)) ||
          fail(hipEventElapsedTime(&ms, e0, e1)))
        break;
      if (rep > 0 && (best == 0.0f || ms < best)) best = ms;
    }
    if (st == CV_OK) *hbm_gbs = 2.0 * (double)bytes / (best * 1e-3) / 1e9;
    best = 0.0f;
    for (int rep = 0; rep < 6 && st == CV_OK; ++rep) {
      float ms = 0.0f;
      if (fail(hipEventRecord(e0, s)) || fail(launch_probe_mfma(blocks, iters, out, s)) ||
          fail(hipEventRecord(e1, s)) || fail(hipEventSynchronize(e1)) ||
          fail(hipEventElapsedTime(&ms, e0, e1)))
        break;
      if (rep > 0 && (best == 0.0f || ms < best)) best = ms;
    }
    const double flops = (double)blocks * 4.0 * iters * 4.0 * 2048.0;
    if (st == CV_OK) *f64_mfma_tflops = flops / (best * 1e-3) / 1e12;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  if (out) (void)hipFree(out);
  return st;
}

cv_status cv_profile_enable(int on) {
  g_prof_on = on != 0;
  return CV_OK;
}

cv_status cv_profile_reset(void) {
  g_prof.clear();
  g_agg.clear();
  g_pool_used = 0;
  return CV_OK;
}

cv_status cv_profile_collect(int* entries) {
  if (!entries) return CV_E_INVALID;
  g_agg.clear();
  for (const ProfRec& r : g_prof) {
    float ms = 0.0f;
    CV_HIP(hipEventSynchronize(r.b));
    CV_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    ProfAgg* a = nullptr;
    for (ProfAgg& x : g_agg)
      if (strcmp(x.name, r.name) == 0) a = &x;
    if (!a) {
      g_agg.push_back({r.name, 0, 0.0, 0.0, 0.0});
      a = &g_agg.back();
    }
    a->launches += 1;
    a->ms += ms;
    a->flops += r.flops;
    a->bytes += r.bytes;
  }
  *entries = (int)g_agg.size();
  return CV_OK;
}

cv_status cv_profile_entry(int i, const char** name, int* launches, double* ms, double* flops,
                           double* bytes) {
  if (i < 0 || i >= (int)g_agg.size()) return CV_E_INVALID;
  const ProfAgg& a = g_agg[i];
  if (name) *name = a.name;
  if (launches) *launches = a.launches;
  if (ms) *ms = a.ms;
  if (flops) *flops = a.flops;
  if (bytes) *bytes = a.bytes;
  return CV_OK;
}

}  // extern "C"

