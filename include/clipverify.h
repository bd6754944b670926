/*
 * clipverify.h - C ABI of the MI355X (gfx950) clip-and-verify hot path.
 *
 * Batched evaluation, over many branch-and-bound subdomains at once, of
 * CROWN-style linear bound propagation together with linear-constraint
 * driven domain clipping (Clip-and-Verify, arXiv 2512.11087).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Floating-point data crossing the ABI is IEEE float32, row-major and
 *   contiguous.  Internally every sum and product is evaluated in float64
 *   and every bound written back as float32 is rounded outward (lower
 *   bounds down, upper bounds up) after subtracting a rigorous bound on the
 *   float64 rounding error, so a float32 result is never tighter than the
 *   exact real-arithmetic value it stands for.
 * - A "box" is a pair lo[n], hi[n] (lo <= x <= hi).  Constraints are
 *   G x + h <= 0 (the form of Thm 3.1 / Thm 3.2 / Alg. 1).
 * - Pointers named in "device" are device (HBM) pointers owned by the
 *   caller; the library never frees them.  Pointers named "host" are read
 *   during the call only.  Handles (cv_net, cv_root) own their device
 *   memory until destroyed.
 * - Every call that takes a hipStream_t enqueues its kernels on that
 *   stream and returns without synchronising.  Argument and shape checks
 *   happen before anything is enqueued; a failed check returns an error
 *   and enqueues nothing.  A HIP error from an enqueue returns CV_E_HIP and
 *   is kept for cv_last_hip_error().
 * - Calls that need scratch memory take a caller-provided device workspace
 *   (ws, ws_bytes) whose minimum size is reported by the matching
 *   *_workspace function; hot calls never allocate.
 * - Infeasibility is not an error: an infeasible subdomain gets flag 1 and
 *   +inf lower bounds (case 1 of the proof of Thm 3.1).
 * - Handles are immutable after creation: concurrent calls on different
 *   streams may share them; calls sharing one workspace must not overlap.
 * - Limits of this library: input dimension n <= 4096 and, for complete
 *   clipping and the constraint order, kmax <= 64 (CV_E_UNSUPPORTED beyond).
 */
#ifndef CLIPVERIFY_H
#define CLIPVERIFY_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CV_OK = 0,
  CV_E_INVALID = -1,     /* null pointer / invalid value (e.g. alpha outside [0,1]) */
  CV_E_SHAPE = -2,       /* sizes inconsistent with the handle or each other */
  CV_E_UNSUPPORTED = -3, /* valid request this library does not implement */
  CV_E_WORKSPACE = -4,   /* ws_bytes smaller than the reported requirement */
  CV_E_HIP = -5,         /* a HIP runtime call failed (see cv_last_hip_error) */
  CV_E_NOMEM = -6,       /* device allocation inside a create call failed */
  CV_E_NONFINITE = -7    /* debug build: a floating-point input holds NaN or +-inf */
} cv_status;

const char* cv_status_string(cv_status s);
/* Last HIP error code recorded by this thread (hipSuccess = 0). */
int cv_last_hip_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int cv_version(void);

/* Debug build (libclipverify_debug.so, compiled with CV_DEBUG): 1, else 0.
 * A debug build also checks what a release build takes on trust, at the
 * cost of synchronising the stream:
 * - the floating-point inputs of cv_clip_domains, cv_concretize,
 *   cv_concretize_planes, cv_bound_propagate and cv_alpha_step (boxes,
 *   planes and intercepts, objectives, intermediate bounds, slopes read)
 *   are scanned on the device before any kernel is enqueued; a NaN or
 *   +-inf returns CV_E_NONFINITE and enqueues nothing;
 * - every kernel launch is followed by a synchronisation of its stream and
 *   an error check, so a failing kernel returns CV_E_HIP from the call that
 *   launched it, and cv_last_kernel names it. */
int cv_debug_build(void);
/* Name of the kernel this thread's library calls launched last (NULL
 * before the first launch).  Host-owned static string. */
const char* cv_last_kernel(void);

/* ------------------------------------------------------------- network */

enum { CV_LINEAR = 0, CV_CONV2D = 1 };

/* One affine layer; a ReLU follows every layer except the last.
 * Linear: W host [out_features, in_features], b host [out_features].
 * Conv2d: W host [out_c, in_c, kernel, kernel], b host [out_c], cross-
 * correlation with zero padding; activations are flattened (c, h, w). */
typedef struct {
  int kind;
  int in_features, out_features;
  int in_c, in_h, in_w, out_c, out_h, out_w, kernel, stride, pad;
  const float* W;
  const float* b;
} cv_layer_desc;

typedef struct cv_net_s* cv_net;

/* Copies the weights to the current device.  n_layers >= 2 (one hidden ReLU
 * layer at least).  A conv layer (in_features = in_c*in_h*in_w, out_features
 * = out_c*out_h*out_w, out_h = (in_h + 2 pad - kernel)/stride + 1, likewise
 * out_w, activations flattened channel-major) is kept as its kernel only:
 * the backward passes and the adjoint run it as a direct (transposed)
 * convolution, and the root pass takes the rows of its matrix from the
 * kernel.  The last (objective) layer must be linear.  CV_E_UNSUPPORTED for
 * a conv as the last layer, a linear layer of more than 2^28 entries or a
 * conv layer of more than 2^26 inputs or outputs; CV_E_SHAPE for
 * inconsistent sizes.  A conv layer whose input row fits 64 KiB runs
 * whole-row convolution kernels (unless it has 32 or more channels on both
 * sides), the others tiled kernels; with
 * CV_CONV_TILED=1 in the environment when the net is made, every conv layer
 * runs the tiled kernels (a testing aid: it changes the summation order, not
 * the bounds' soundness). */
cv_status cv_net_create(const cv_layer_desc* layers, int n_layers, cv_net* out);
cv_status cv_net_destroy(cv_net net);
/* Host outputs: input dim, output dim, total hidden neurons, layer count. */
cv_status cv_net_info(cv_net net, int* n_in, int* n_out, int* n_hidden, int* n_layers);

/* Kernel variants of each layer, kind CV_TUNE_RELAX (backward step through
 * W_layer, 2 <= layer <= n_layers-1), CV_TUNE_FINAL (layer 1) or
 * CV_TUNE_ADJOINT (1 <= layer <= n_layers-1): the output tile of the GEMM
 * (0: 32 x 128, 1: 64 x 128, 2: 128 x 128 rows x columns; the adjoint also
 * 3: 32 x 256).  A conv layer runs as a direct convolution: where it runs
 * the whole-row kernels (see cv_net_create), the transposed
 * convolution (CV_TUNE_RELAX / CV_TUNE_FINAL) takes 0: positions per lane
 * by shape, 1/2/3: one, two or four, and the adjoint's forward convolution
 * 0: built-in, 1/2/3: channel blocks of 4/8/16, 4/5: blocks of 8/16 with
 * four positions per lane; where it runs the tiled kernels, their
 * transposed convolution takes the staging depth (0 built-in, 1/2/3: 4/8/16
 * channels per chunk) and whose forward convolution takes 0: built-in,
 * 1/2/3: 4/8/16 channels per chunk, 4: the other tile width.  Every variant
 * gives the same results (the same accumulation order per element).
 * cv_net_autotune times each variant of every layer once on synthetic
 * operands of B subdomains x M objective rows (allocating its own scratch,
 * synchronising `stream`) and keeps the fastest; the choice then applies to
 * every call with this net.  It changes the net: do not call it while the
 * net is in use on another stream.  cv_net_tuning reads a layer's variant
 * and variant count (host outputs, either may be NULL); cv_net_set_tuning
 * sets it (CV_E_INVALID for a kind, layer or variant out of range). */
enum { CV_TUNE_RELAX = 0, CV_TUNE_FINAL = 1, CV_TUNE_ADJOINT = 2 };
cv_status cv_net_autotune(cv_net net, int B, int M, hipStream_t stream);
cv_status cv_net_tuning(cv_net net, int kind, int layer, int* variant, int* count);
cv_status cv_net_set_tuning(cv_net net, int kind, int layer, int variant);

/* ---------------------------------------------------------- root state */

typedef struct cv_root_s* cv_root;

/* Root pass (once per property): CROWN bounds and planes of every hidden
 * neuron over the root box, cached for reuse by every subdomain (the
 * initial bounding pass of the activation-BaB section / Alg. 5,
 * Get_Constraints).  Layer-1 planes are W1, b1; for a deeper neuron the
 * lower plane is CROWN with objective +e_j on the cut network and the
 * upper plane the negation of CROWN with objective -e_j (Lemma A.3 and the
 * plane recursion of appendix A.3), with the fixed slope alpha0 in [0,1]
 * for unstable neurons.  Plane coefficients are stored float32 and the
 * intercepts float64, corrected at the root box centre and moved outward by
 * the rounding of the coefficients over the box radius, so the stored planes
 * are valid on the whole root box.
 * lo0, hi0: device [n_in].  Synchronises `stream` before returning.  The
 * pass's working memory (the backward-pass workspace of its widest layer,
 * one row per neuron of that layer) stays on the net for the next root and
 * is freed by cv_net_destroy, so roots of one net are created one at a time
 * (not concurrently from several threads). */
cv_status cv_root_create(cv_net net, const float* lo0, const float* hi0, float alpha0,
                         hipStream_t stream, cv_root* out);
/* The same with a choice of which planes stay cached (the root pass computes
 * them all; the bounds are the same either way):
 *   CV_ROOT_PLANES_ALL: every hidden neuron's planes, [n_hidden, n_in] per
 *     side;
 *   CV_ROOT_PLANES_UNSTABLE: only those of the root-unstable neurons
 *     (l0 < 0 < u0), [U, n_in] per side -- the memory answer for large
 *     networks, where the others cannot be split by a branch-and-bound
 *     anyway.  A split constraint on a neuron without a kept plane is then
 *     ignored (dropping a constraint can only loosen a bound, so results stay
 *     sound); cv_root_planes returns CV_E_UNSUPPORTED;
 *   CV_ROOT_PLANES_AUTO (what cv_root_create does): ALL unless n_hidden *
 *     n_in exceeds 2^28, then UNSTABLE.
 * Other values: CV_E_INVALID. */
enum { CV_ROOT_PLANES_AUTO = 0, CV_ROOT_PLANES_ALL = 1, CV_ROOT_PLANES_UNSTABLE = 2 };
cv_status cv_root_create_ex(cv_net net, const float* lo0, const float* hi0, float alpha0,
                            int planes, hipStream_t stream, cv_root* out);
cv_status cv_root_destroy(cv_root root);
/* Device outputs [n_hidden]: root pre-activation bounds (global neuron
 * order = layer by layer). */
cv_status cv_root_bounds(cv_root root, float* l0, float* u0, hipStream_t stream);
/* Device outputs: A_lo, A_hi [n_hidden, n_in], c_lo, c_hi [n_hidden]:
 * z_j >= A_lo[j].x + c_lo[j] and z_j <= A_hi[j].x + c_hi[j] on the root box
 * (intercepts rounded outward to float32).  CV_E_UNSUPPORTED for a root that
 * keeps the unstable neurons' planes only. */
cv_status cv_root_planes(cv_root root, float* A_lo, float* c_lo, float* A_hi, float* c_hi,
                         hipStream_t stream);
/* Host output: number of root-unstable neurons (l0 < 0 < u0). */
cv_status cv_root_unstable_count(cv_root root, int* count);

/* A set of P properties over one network (batching: many properties, each
 * with its own root box, root state and objective, bounded in the same
 * launches).  roots: host array of P single roots of the same net; the set
 * borrows their state (they must outlive it) and owns only a device table
 * of it.  Every call that takes a root accepts a set together with
 * pid: device [B] int32, the property of each subdomain (subdomains of one
 * property need not be contiguous, but grouping them is faster for
 * cv_concretize_planes; values outside [0, P) are clamped).  pid == NULL
 * means property 0 for every subdomain.  The objective of a set is
 * per property: C [P, M, n_out], t [P, M].  cv_root_bounds, cv_root_planes,
 * cv_root_unstable_count and cv_intermediate_bounds take single roots only
 * (CV_E_INVALID / CV_E_UNSUPPORTED for a set).  Destroy with cv_root_destroy. */
cv_status cv_rootset_create(const cv_root* roots, int P, cv_root* out);
/* Host output: number of properties (1 for a single root). */
cv_status cv_root_count(cv_root root, int* P);

/* --------------------------------------------------------- constraints */

/* The linear constraints of each subdomain, in one of two forms.
 * Split form (neuron != NULL; needs a cv_root): slot k of subdomain b is the
 * activation split (neuron[b,k], sign[b,k]) on a hidden neuron, turned into
 * an input halfspace with the cached root planes (eqs. 9-10): sign -1
 * (branch z <= 0) gives A_lo[j].x + c_lo[j] <= 0, sign +1 (branch z >= 0)
 * gives -A_hi[j].x - c_hi[j] <= 0.
 * Dense form (neuron == NULL): slot k of subdomain b is G[b,k,:].x + h[b,k] <= 0.
 * Slots k < count[b] are used (count == NULL: all kmax).  All device.
 * order (optional): [B, kmax] permutation, position -> slot, whose first
 * count[b] entries are the used slots; sequential relaxed clipping and
 * complete clipping take the constraints in that order (NULL: slot order).
 * Entries outside [0, kmax) are ignored slots; a non-permutation gives
 * unspecified bounds but no out-of-range access.  cv_constraint_order
 * computes the importance order of the heuristics appendix. */
typedef struct {
  int kmax;
  const int32_t* count;  /* [B] or NULL */
  const int32_t* neuron; /* [B, kmax] global hidden-neuron index */
  const int8_t* sign;    /* [B, kmax] +1 / -1 */
  const float* G;        /* [B, kmax, n] */
  const float* h;        /* [B, kmax] */
  const int32_t* order;  /* [B, kmax] or NULL */
} cv_constraints;

/* Constraint importance order (heuristics appendix): for each subdomain,
 * the used slots sorted by the Euclidean distance |g.xc + h| / ||g||_2 of
 * their hyperplane from the centre xc = (lo + hi)/2 of its box, closest
 * first; ties keep slot order, slots with g = 0 go last, unused slots keep
 * their place.  cons->order is not read.  Computed in float64.
 * lo, hi: device [B, n]; order: device output [B, kmax] (see cv_constraints).
 * Errors: CV_E_UNSUPPORTED if kmax > 64; CV_E_SHAPE if the split form's
 * root has another input size. */
cv_status cv_constraint_order(cv_root root, const int32_t* pid, int B, int n,
                              const cv_constraints* cons,
                              const float* lo, const float* hi, int32_t* order,
                              hipStream_t stream);

enum { CV_CLIP_PARALLEL = 0, CV_CLIP_SEQUENTIAL = 1 };

/* Relaxed clipping of each subdomain's box.  For each subdomain b and each used
 * constraint k, m = min over the box of G_k x + h_k; if m > 0 the box is
 * empty.  Otherwise coordinate i is tightened to lo_i - m/G_ki (upper bound,
 * G_ki > 0) or hi_i - m/G_ki (lower bound, G_ki < 0): the closed form of
 * Thm 3.2.  CV_CLIP_PARALLEL applies every constraint to the original box
 * and keeps the tightest value (Alg. 2); CV_CLIP_SEQUENTIAL applies them in
 * the constraint order (cons->order, else slot order) to the box left by the
 * previous one (Alg. 3).
 * root: required for the split form, else may be NULL.
 * lo, hi: device [B, n] in/out.  infeasible: device [B] uint8 out, 1 when
 * some constraint is certainly empty over the box or lo > hi afterwards.
 * B == 0 is a no-op. */
cv_status cv_clip_domains(cv_root root, const int32_t* pid, int B, int n,
                          const cv_constraints* cons,
                          float* lo, float* hi, uint8_t* infeasible, int mode,
                          hipStream_t stream);

/* Re-concretization of the cached planes over each subdomain's box (the
 * relaxed-clipping section: all intermediate bounds are re-concretized
 * over the clipped box without a new bound-propagation pass):
 *   l_j = min over box of A_lo[j].x + c_lo[j],  u_j = max of A_hi[j].x + c_hi[j]
 * for every root-unstable neuron j, intersected with the root bounds;
 * root-stable neurons keep their root bounds.  Split neurons are then fixed
 * to their branch (l_j = max(l_j, 0) for +1, u_j = min(u_j, 0) for -1).
 * splits: split form, dense form (complete clipping only; no split fix) or
 * NULL.  l, u: device [B, n_hidden] out.
 * infeasible: device [B] in/out (OR-ed with "some neuron has l > u").
 * With complete != 0 the bounds of the neurons still unstable are then
 * tightened by complete clipping (Alg. 1, `passes` passes) of their lower and
 * negated upper planes against the subdomain's split halfspaces: all of them
 * when topk < 0, else per hidden layer the topk neurons with the largest
 * BaBSR intercept score max(0,-l) max(0,u) / (u-l) * weight[j] (heuristics
 * appendix; ties to the lower index; weight from cv_babsr_weights or the
 * caller, device [P, n_hidden]).  select (optional) device [B, n_hidden]
 * receives the selection mask (1 = clipped). */
cv_status cv_concretize_planes(cv_root root, const int32_t* pid, int B, const float* lo,
                               const float* hi,
                               const cv_constraints* splits, int complete, int passes,
                               int topk, const float* weight,
                               float* l, float* u, uint8_t* infeasible, uint8_t* select,
                               void* ws, size_t ws_bytes, hipStream_t stream);
/* Workspace bytes of cv_concretize_planes (0 unless complete != 0). */
cv_status cv_concretize_planes_workspace(cv_root root, int B, int complete, size_t* bytes);

/* cv_concretize_planes for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, with the scratch taken from
 * a static device array of CV_CONCRETIZE_PLANES_STATIC_BYTES (64 MiB) instead
 * of a caller workspace.  The library holds one such array on every device
 * it runs on until the process ends; the first call on a device looks up
 * that device's copy (the current device: the one of `stream` and of every
 * pointer).  The call itself allocates nothing, and records no timing events
 * while the kernel-timing instrumentation is on.  Limit: the scratch
 * cv_concretize_planes_workspace reports for (root, B, complete) must fit in
 * the array, else CV_E_WORKSPACE and nothing is enqueued (with complete != 0
 * about B * (8 U + n_hidden + 1536) bytes, U the root-unstable neurons).
 * Calls on one device share its array and keep no state across calls, but
 * two calls that overlap in time on one device (other streams, other
 * threads) race on it: serialise them.  Other arguments, results and errors
 * as cv_concretize_planes. */
#define CV_CONCRETIZE_PLANES_STATIC_BYTES (64u << 20)
cv_status cv_concretize_planes_static(cv_root root, const int32_t* pid, int B, const float* lo,
                                      const float* hi, const cv_constraints* splits, int complete,
                                      int passes, int topk, const float* weight, float* l,
                                      float* u, uint8_t* infeasible, uint8_t* select,
                                      hipStream_t stream);

/* Weights of the neuron-selection score (heuristics appendix): weight[j] =
 * max(0, -mean over the M objective rows of Psi_mj), the coefficient with
 * which the ReLU output of hidden neuron j enters the CROWN lower bound of
 * row m, from one backward pass over the root box with the root bounds and
 * slope (once per property).  C, t: device [P, M, n_out], [P, M]; weight:
 * device [P, n_hidden] out (P = 1 for a single root).
 * ws: cv_babsr_weights_workspace(...) bytes. */
cv_status cv_babsr_weights(cv_net net, cv_root root, int M, const float* C, const float* t,
                           float* weight, void* ws, size_t ws_bytes, hipStream_t stream);
cv_status cv_babsr_weights_workspace(cv_net net, int M, size_t* bytes);

/* Concretization of linear functions over boxes (Lemma A.2), optionally
 * with complete clipping.  Row p of subdomain b is A[b,p,:].x + c[b,p]
 * (A_shared != 0: A[p,:], c[p] for every b).  Without constraints
 * (cons == NULL) lb[b,p] = min over the box.  With constraints, lb[b,p] is
 * max(that, D(beta)) where beta comes from `passes` passes of coordinate
 * ascent over the multipliers (Alg. 1): each step maximises the 1-D dual of
 * Thm 3.1 exactly by locating, among the breakpoints -a_j/g_j, the one where
 * the supergradient changes sign.  An empty constraint gives lb = +inf and
 * infeasible[b] = 1.  ub (optional) gets the maximum without constraints.
 * beta (optional) device [B, P, kmax] gets the multipliers.
 * lo, hi: device [B, n].  lb, ub: device [B, P].  infeasible: [B] or NULL. */
cv_status cv_concretize(cv_root root, const int32_t* pid, int B, int P, int n, const float* A,
                        int A_shared,
                        const float* c, const float* lo, const float* hi,
                        const cv_constraints* cons, int passes, float* lb, float* ub,
                        float* beta, uint8_t* infeasible, hipStream_t stream);

/* CROWN backward bound propagation for the objective rows C y + t
 * (specification matrix and threshold) of every subdomain, the
 * concretization of the resulting input plane over the box and,
 * when cons != NULL, complete clipping of that plane against the
 * subdomain's constraints (lb = the larger of the two).
 * Starting from Omega = C, each linear layer maps Omega to Psi = Omega W and
 * adds Omega b to the intercept; each ReLU neuron uses the relaxation of
 * Lemma A.3 chosen by the sign of Psi: slope 1 (l >= 0), 0 (u <= 0), alpha
 * (unstable, Psi >= 0) or the upper line u/(u-l)(z-l) (unstable, Psi < 0).
 * C: device [P, M, n_out], t: device [P, M] (P = 1 for a single root;
 * subdomain b uses the rows of its property pid[b]).  l, u: device [B, n_hidden]
 * (per-subdomain pre-activation bounds, e.g. from cv_concretize_planes).
 * alpha: device [B, M, n_hidden] in [0,1] or NULL (alpha_default for all).
 * lo, hi: device [B, n_in], inside the root box of `root` (the root's bounds
 * feed the rigorous rounding-error bounds; l, u must lie inside the root
 * bounds, as cv_concretize_planes guarantees).  infeasible: device [B]
 * in/out or NULL: flagged subdomains get +inf; complete clipping sets the
 * flag when a constraint is empty over the box.
 * Outputs (device): lb [B, M]; A_out [B, M, n_in] or NULL (the input plane,
 * rounded to float32); c_out [B, M] or NULL (its intercept, moved down by
 * the rounding error bound so that A_out, c_out is a valid plane).
 * ws: workspace of at least cv_bound_propagate_workspace(...) bytes. */
cv_status cv_bound_propagate(cv_net net, int B, int M, const float* C, const float* t,
                             const float* l, const float* u, const float* alpha,
                             float alpha_default, const float* lo, const float* hi,
                             uint8_t* infeasible, cv_root root, const int32_t* pid,
                             const cv_constraints* cons, int passes,
                             float* lb, float* A_out, float* c_out,
                             void* ws, size_t ws_bytes, hipStream_t stream);
/* P: number of properties of the root the call will use. */
cv_status cv_bound_propagate_workspace(cv_net net, int P, int B, int M, size_t* bytes);

/* One slope-optimisation step.  Computes the bound of cv_bound_propagate
 * (with complete clipping when cons != NULL) at the current alpha into lb,
 * then the gradient of sum(lb) with respect to every alpha entry that
 * selects a lower line (unstable neuron, Psi >= 0), holding the complete-
 * clipping multipliers fixed, by a hand-written adjoint of the backward
 * pass; then, when lr > 0, one projected Adam ascent step (bias-corrected
 * moments with beta1, beta2, eps; `step` >= 1 is the 1-based step index)
 * on alpha, clamped to [0,1] (the experimental settings' slope
 * optimisation: Adam, lr 0.1, 20 iterations).
 * alpha: device [B, M, n_hidden] in/out.  Step 1 starts an optimisation:
 * Adam's moments are taken as zero (adam_m, adam_v are written, not read)
 * and, when alpha_init is in [0, 1], every slope is alpha_init (alpha is
 * then written, not read); alpha_init < 0 reads alpha at step 1 as well,
 * and must be < 0 at later steps (CV_E_INVALID otherwise).
 * adam_m, adam_v: device [B, M, n_hidden] in/out (may be NULL when lr == 0).
 * best: device [B, M] in/out or NULL: the running best bound over the steps,
 * max(best, lb) (lb itself at step 1, where best is not read); +inf for an
 * infeasible subdomain.  grad: device [B, M, n_hidden] out or NULL.
 * ws: at least cv_alpha_step_workspace(...) bytes. */
cv_status cv_alpha_step(cv_net net, int B, int M, const float* C, const float* t,
                        const float* l, const float* u, float* alpha, float alpha_init,
                        const float* lo, const float* hi, uint8_t* infeasible,
                        cv_root root, const int32_t* pid, const cv_constraints* cons,
                        int passes, float* adam_m, float* adam_v, int step, float lr,
                        float beta1, float beta2, float eps,
                        float* lb, float* best, float* grad, void* ws, size_t ws_bytes,
                        hipStream_t stream);
cv_status cv_alpha_step_workspace(cv_net net, int P, int B, int M, size_t* bytes);

/* CROWN bounds of every hidden neuron over each subdomain's own box (the
 * bounding of a fresh input box, as opposed to re-concretizing the root
 * planes): for hidden layers 2..L-1 in order, a backward pass with the
 * objectives +I and -I on that layer's pre-activations through the layers
 * below (Lemma A.3 with the root slope, the subdomain's bounds of the
 * earlier layers), concretized over the box and intersected with the
 * bounds passed in.  l, u: device [B, n_hidden] in/out, valid bounds on
 * entry (e.g. from cv_concretize_planes, which gives layer 1 exactly); lo,
 * hi: device [B, n_in] inside the root box.  infeasible: [B] in/out or
 * NULL: flagged boxes are skipped; a box whose bounds cross (l > u) is
 * flagged. */
cv_status cv_intermediate_bounds(cv_net net, cv_root root, int B, const float* lo, const float* hi,
                                 float* l, float* u, uint8_t* infeasible, void* ws,
                                 size_t ws_bytes, hipStream_t stream);
cv_status cv_intermediate_bounds_workspace(cv_net net, int B, size_t* bytes);

/* ---------------------------------------------------- branch and bound */

/* ReLU branching (Alg. 5): each parent subdomain b (splits, box lo/hi
 * [B, n_in], bounds l/u [B, n_hidden]) is split on the unstable neuron
 * (l < 0 < u) not split yet with the largest BaBSR intercept score
 * max(0,-l) max(0,u) / (u-l) * weight[j] (ties to the lower index; weight
 * [P, n_hidden], row pid[b] for subdomain b) into
 * child 2b (branch z <= 0) and child 2b+1 (branch z >= 0): the parent's
 * splits plus the new one, and the parent's box.  chosen[b] = -1 when no
 * unstable neuron is left or the parent already uses all kmax_out slots
 * (the children then equal the parent).
 * Outputs (device): chosen [B]; neuron2, sign2 [2B, kmax_out]; count2 [2B];
 * lo2, hi2 [2B, n_in].  kmax_out >= splits->kmax (else CV_E_SHAPE). */
cv_status cv_branch_relu(cv_root root, const int32_t* pid, int B, const float* l, const float* u,
                         const float* weight,
                         const cv_constraints* splits, const float* lo, const float* hi,
                         int kmax_out, int32_t* chosen, int32_t* neuron2, int8_t* sign2,
                         int32_t* count2, float* lo2, float* hi2, hipStream_t stream);

/* Input branching (Alg. 4): each box b is halved along the dimension with
 * the largest (hi_d - lo_d) * sum_m |A[b,m,d]| (A: the parent's final planes
 * [B, M, n]; ties to the lower index) at the float32 midpoint: child 2b is
 * the lower half, child 2b+1 the upper half (they share the cut).
 * Outputs (device): dim [B]; lo2, hi2 [2B, n]. */
cv_status cv_branch_input(int B, int M, int n, const float* lo, const float* hi, const float* A,
                          int32_t* dim, float* lo2, float* hi2, hipStream_t stream);

/* ------------------------------------------------------ kernel timing */

/* Instrumentation for benchmarks.  While enabled, every kernel the library
 * enqueues is bracketed by two HIP events recorded on the stream it is
 * launched on, together with that launch's algorithmic work (floating-point
 * operations and bytes, counted from the shapes).  Process-global and not
 * thread-safe.  cv_profile_collect (after the streams are synchronised)
 * aggregates the records by kernel name and returns the number of names;
 * cv_profile_entry(i, ...) reads aggregate i (host outputs, any may be
 * NULL); cv_profile_reset drops the records. */
cv_status cv_profile_enable(int on);
cv_status cv_profile_reset(void);
cv_status cv_profile_collect(int* entries);
cv_status cv_profile_entry(int i, const char** name, int* launches, double* ms,
                           double* flops, double* bytes);

/* Roofline denominators measured on the current device (benchmark
 * instrumentation, not a hot call: it allocates 2 GiB, synchronises `stream`
 * and frees): the HBM bandwidth of a streaming copy of 1 GiB (bytes read +
 * written per second) and the float64 matrix-core rate of a loop of
 * independent v_mfma_f64_16x16x4_f64 on 2048 workgroups, each the best of
 * five timed runs after one warm-up.  Host outputs in GB/s and TFLOP/s. */
cv_status cv_measure_peaks(double* hbm_gbs, double* f64_mfma_tflops, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CLIPVERIFY_H */
