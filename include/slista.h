/*
 * slista.h -- C ABI of the MI355X (gfx950) library for batched unfolded ISTA /
 * Step-LISTA.
 *
 * Paper: Ablin, Moreau, Massias, Gramfort, "Learning step sizes for unfolded
 * sparse coding", NeurIPS 2019 (arXiv 1905.11071).
 *
 * The library evaluates, for a batch of N samples x_i in R^n, a dictionary
 * D in R^{n x m}, a regularisation lambda > 0 and T step sizes alpha_t > 0,
 * the Step-LISTA network of Section 4, Eq. (14):
 *
 *     z^(0) = 0,
 *     z^(t+1) = ST( z^(t) - alpha_t D^T (D z^(t) - x), lambda alpha_t ),
 *     ST(u, theta) = sign(u) max(|u| - theta, 0)        (Section 1, Eq. (2)),
 *
 * which is proximal gradient descent with a step sequence (Section 3, Eq. (5))
 * and ISTA (Eq. (2)) when every alpha_t = 1/L. The Lasso cost it descends is
 * F_x(z) = 1/2 ||x - D z||^2 + lambda ||z||_1 (Section 1, Eq. (1)); the
 * training loss is its mean over the batch (Section 4, Eq. (15)), and the
 * library returns the derivative of that loss with respect to every alpha_t.
 *
 * The device computes the gradient in Gram form, D^T (D z - x) = G z - c with
 * G = D^T D (m x m) and c = D^T x, so that every layer is one dense
 * contraction P = Z G over the batch, run on the MFMA units, followed by the
 * step, the threshold and the objective in FP32.
 *
 * Conventions (every entry point)
 *  - Pointers named "device" are HIP device pointers owned by the caller; the
 *    library never frees or keeps them beyond the call (a batch keeps the
 *    pointers of its problems until it is destroyed). The library owns
 *    device memory only in a slista_dict (its Gram matrices and D^T,
 *    allocated in slista_dict_create, released in slista_dict_destroy), in a
 *    slista_batch (argument tables and work lists, allocated when it is bound,
 *    released when it is destroyed), in the plans of slista_batched_fwd_bwd
 *    (released by slista_batched_release), and in the static array of
 *    slista_forward_scratch. Every other call allocates nothing: workspaces
 *    come from the caller.
 *  - All matrices are row-major and sample-major: X is [N, n] (row i is x_i),
 *    Z and dZ are [N, m] (row i is z_i), D is [n, m].
 *  - `stream` is a hipStream_t (NULL = the legacy default stream). Work is
 *    enqueued on it and the call returns without waiting, except where a
 *    function says it synchronises.
 *  - Every function returns an slista_status. Arguments are checked on the
 *    host before anything is enqueued; a failed check enqueues nothing. The
 *    text of the last failure on the calling thread is slista_last_error().
 *  - Device values are not inspected: alpha_t > 0 (Section 4, parameters in
 *    R+*) and finite inputs are preconditions. Non-finite inputs propagate
 *    by IEEE arithmetic (into F and the loss; the soft-threshold maps a NaN
 *    argument to 0, so codes may stay finite), unless the finite-value check
 *    (SLISTA_OPT_CHECK_FINITE) is on: then the dictionary, forward and backward entry points count
 *    NaN/Inf in their inputs and outputs on the device, synchronise, and
 *    return SLISTA_ENONFINITE if there are any.
 *  - Calls that overlap on the same workspace race; calls on distinct
 *    workspaces may run concurrently on different streams.
 */
#ifndef SLISTA_H_
#define SLISTA_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLISTA_API __attribute__((visibility("default")))
#define SLISTA_ABI_VERSION 1

typedef enum {
  SLISTA_OK = 0,
  SLISTA_EINVAL = -1,     /* bad argument: size, null pointer, lambda, precision, workspace */
  SLISTA_ENOMEM = -2,     /* device allocation failed (slista_dict_create), or no workspace
                             fits the budget (slista_ckpt_for_budget); a batch's table
                             allocation failing reports SLISTA_EHIP */
  SLISTA_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
  SLISTA_ENOTSUP = -4,    /* valid request the library does not support (e.g. no gfx950 device) */
  SLISTA_ENOTCONV = -5,   /* power iteration reached max_iter before rtol */
  SLISTA_ENONFINITE = -6  /* the finite-value check found NaN or Inf (SLISTA_OPT_CHECK_FINITE) */
} slista_status;

/* Arithmetic of the contraction P = Z G. The step, threshold and objective
 * are FP32 in both modes. */
typedef enum {
  SLISTA_FP32 = 0,  /* FP32 operands on MFMA (v_mfma_f32_16x16x4_f32), FP32 accumulate */
  SLISTA_BF16 = 1   /* BF16 operands on MFMA (v_mfma_f32_16x16x32_bf16), FP32 accumulate;
                       z is rounded to BF16 only as the operand of the product */
} slista_prec;

/* A precision schedule for the forward / backward entry points and batches:
 * BF16 contractions in layers 0 .. T-tail-1 and FP32 contractions in the last
 * `tail` layers (and in the adjoint of those layers). BF16 operands leave
 * the iterates at a rounding floor that FP32 layers then contract away, so a
 * short FP32 tail recovers FP32 objective-gap accuracy on converged problems
 * at a fraction of the FP32 cost. 0 <= tail <= T; with layer checkpointing
 * (ckpt_every > 1) T - tail must be a multiple of ckpt_every (the first FP32
 * layer starts from a checkpoint). Pass it wherever an `int prec` is taken
 * by slista_forward, slista_backward, slista_forward_backward,
 * slista_forward_scratch, slista_batch_create and slista_batched_*; other
 * entry points take SLISTA_FP32 or SLISTA_BF16 only. */
#define SLISTA_BF16_FP32_TAIL(tail) (SLISTA_BF16 | ((tail) << 8))

typedef struct slista_dict slista_dict;

/* Version of this ABI (SLISTA_ABI_VERSION). */
SLISTA_API int slista_abi_version(void);

/* Static text for a status code. Never NULL. */
SLISTA_API const char* slista_status_string(int status);

/* Detail of the last failed call on the calling thread ("" if none). */
SLISTA_API const char* slista_last_error(void);

/* ---------------------------------------------------------------------------
 * Dictionary
 * ------------------------------------------------------------------------- */

/* Build the per-dictionary state from D (device, FP32, [n, m] row-major,
 * 1 <= n <= 65536, 1 <= m <= 8192): the Gram matrix G = D^T D accumulated in
 * FP64 and stored in FP32 and BF16, and D^T, each zero-padded to
 * m_pad = m rounded up to a multiple of 64. Allocates device memory (the only
 * allocation the library makes) and synchronises `stream` before returning.
 * On success *out owns that memory until slista_dict_destroy. */
SLISTA_API int slista_dict_create(const float* D, int n, int m, void* stream, slista_dict** out);

/* Release a dictionary (NULL is accepted). Synchronises the device first. */
SLISTA_API int slista_dict_destroy(slista_dict* dict);

/* Sizes of a dictionary: n, m and the padded m used in the workspace. */
SLISTA_API int slista_dict_dims(const slista_dict* dict, int* n, int* m, int* m_pad);

/* Copy G = D^T D (FP32, [m, m], row-major) to device buffer G_out. */
SLISTA_API int slista_dict_gram(const slista_dict* dict, float* G_out, void* stream);

/* L = greatest eigenvalue of D^T D (Section 1, after Eq. (2)), by power
 * iteration in FP64 on the FP32 Gram matrix, stopped when two successive
 * Rayleigh quotients differ by at most rtol (relative) or after max_iter
 * iterations (1 <= max_iter <= 10^7). Writes L to *L_out (host) and the
 * iteration count to *iters (host, may be NULL). Synchronises `stream`.
 * Returns SLISTA_ENOTCONV, with the last estimate in *L_out, if rtol was not
 * reached. */
SLISTA_API int slista_dict_lipschitz(slista_dict* dict, int max_iter, double rtol, double* L_out,
                                     int* iters, void* stream);

/* Layer checkpointing for a memory budget: the smallest ckpt_every (fewest
 * recomputed layers) whose forward/backward workspace for (N, T, prec) fits
 * in `budget` bytes; *bytes (may be NULL) gets that workspace size.
 * SLISTA_ENOMEM if even the smallest workspace does not fit. Host only. */
SLISTA_API int slista_ckpt_for_budget(const slista_dict* dict, int N, int T, int prec, size_t budget,
                                      int* ckpt_every, size_t* bytes);

/* ---------------------------------------------------------------------------
 * Forward and backward through T layers
 *
 * Common arguments:
 *   X        device, FP32 [N, n]: the samples.           0 <= N <= 2^26
 *   lambda   regularisation, finite and > 0 (Eq. (1)).
 *   alpha    device, FP32 [T]: the step sizes alpha_0 .. alpha_{T-1} (Eq. (14)).
 *   T        number of layers, 0 <= T <= 100000.
 *   prec     slista_prec of the contraction.
 *   ckpt_every  layer checkpointing of the tape kept for the backward:
 *            0  = keep no tape (forward only),
 *            1  = keep every iterate z^(1) .. z^(T),
 *            k>1 = keep z^(k), z^(2k), ... and z^(T); the backward recomputes
 *                  the layers in between, segment by segment.
 *   ws, ws_bytes  device workspace of at least slista_workspace_size() bytes
 *            for the same (dict, N, T, prec, ckpt_every); 256-byte aligned.
 * ------------------------------------------------------------------------- */

/* Workspace bytes for the given sizes. */
SLISTA_API int slista_workspace_size(const slista_dict* dict, int N, int T, int prec, int ckpt_every,
                                     size_t* bytes);

/* Forward pass. Writes
 *   Z     device FP32 [N, m]: z^(T) (required),
 *   F     device FP32: if f_trace == 0, [N] with F_{x_i}(z_i^(T)); if f_trace
 *         != 0, [T+1, N] with row t = F_{x_i}(z_i^(t)) (Eq. (1)); NULL = skip,
 *   loss  device FP32 [1]: mean_i F_{x_i}(z_i^(T)) (Eq. (15)); NULL = skip.
 * F and loss are evaluated in FP32 from G z, c and ||x||^2 (monitoring
 * accuracy). With ckpt_every >= 1 the workspace keeps the tape that
 * slista_backward reads. */
SLISTA_API int slista_forward(const slista_dict* dict, const float* X, int N, float lambda,
                              const float* alpha, int T, int prec, float* Z, float* F, int f_trace,
                              float* loss, int ckpt_every, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the forward
 * pass of slista_forward with ckpt_every = 0 (no tape), whose workspace is a
 * static array of 64 MiB (67108864 bytes) inside the library instead of a
 * caller buffer. The caller still passes X, alpha and the outputs Z, F, loss
 * (as for slista_forward). Each GPU the library runs on holds its own copy of
 * that array from the first call on it until the process ends; the call
 * neither allocates nor frees device memory. Sizes whose forward workspace
 * (slista_workspace_size with ckpt_every = 0) exceeds 64 MiB are rejected
 * with SLISTA_EINVAL (e.g. m = 1024 allows N up to about 4000; m = 256 about
 * 16000). The current device must be the dictionary's, and kernel timing
 * (slista_profile_begin) must be off. Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (on different streams or threads)
 * race; calls ordered on one stream do not. Nothing in the array needs to
 * start at zero: the pass overwrites everything it reads. */
SLISTA_API int slista_forward_scratch(const slista_dict* dict, const float* X, int N, float lambda,
                                      const float* alpha, int T, int prec, float* Z, float* F, int f_trace,
                                      float* loss, void* stream);

/* FP64 forward of ISTA (Eq. (2), alpha_t = 1/L) or of Step-LISTA with given
 * steps (Section 4, Eq. (14)): z^(0) = 0, z^(t+1) = ST(z^(t) - alpha_t D^T (D
 * z^(t) - x), lambda alpha_t), every quantity in double precision and the
 * gradient in the factored form of the layer, with the dictionary's FP32
 * values of D widened exactly. For the small double-precision workloads
 * (one wave per sample; no MFMA): a reference-grade device path, not the
 * fast one.
 *   X     device FP64 [N, n], row-major.
 *   alpha device FP64 [T].
 *   Z     device FP64 [N, m]: z^(T).
 *   F     device FP64: with f_trace, [T + 1, N] (F[t][i] = F_{x_i}(z_i^(t)),
 *         Eq. (1), from the residual x - D z); else [N] (F of z^(T)); or NULL.
 *   loss  device FP64 scalar: the mean of F(z^(T)) over the samples
 *         (Eq. (15) at the output), or NULL. Without F the loss needs a
 *         workspace of slista_forward_f64_workspace_size bytes (256-byte
 *         aligned); otherwise ws may be NULL.
 * Errors: SLISTA_EINVAL for NULL or out-of-range arguments, SLISTA_ENOTSUP
 * for n > 512 (the lanes hold at most eight residual entries each). Does not
 * synchronise; does not use the tape record of the FP32/BF16 entry points. */
SLISTA_API int slista_forward_f64_workspace_size(const slista_dict* dict, int N, size_t* bytes);
SLISTA_API int slista_forward_f64(const slista_dict* dict, const double* X, int N, double lambda,
                                  const double* alpha, int T, double* Z, double* F, int f_trace, double* loss,
                                  void* ws, size_t ws_bytes, void* stream);

/* Lasso cost of given codes, Eq. (1): F[i] = 1/2 ||x_i - D z_i||^2 + lambda ||z_i||_1
 * for Z (device FP32 [N, m]), written to F (device FP32 [N]). The residual is
 * formed in FP32 from the non-zero coordinates of z_i (one wave per sample,
 * columns of D read K-contiguously) and the sums are accumulated in FP64, so
 * the value does not depend on the precision that produced Z. Needs no
 * workspace. */
SLISTA_API int slista_objective(const slista_dict* dict, const float* X, int N, float lambda, const float* Z,
                                float* F, void* stream);

/* Reverse pass (derivation in Section 4 / Appendix D: the paper uses
 * automatic differentiation; here it is written out by hand). Differentiates
 *     J = sum_i dF_i F_{x_i}(z_i^(T)) + <dZ, Z^(T)>
 * with respect to alpha and writes dalpha (device FP32 [T]). dZ (device FP32
 * [N, m]) and dF (device FP32 [N]) may each be NULL (= 0) but not both; with
 * dF_i = 1/N and dZ = 0, J is the loss of Eq. (15). The derivative of ST is
 * taken as 1 where |u| > lambda alpha_t and 0 elsewhere, and sign(0) = 0 in
 * the sub-gradient of |z| (a valid sub-gradient at the kinks).
 * ckpt_every >= 1. The call does not depend on an earlier slista_forward:
 * the library records on the host which workspace holds the tape of which
 * forward pass (slista_forward or slista_forward_backward with ckpt_every >=
 * 1: same dict, X and alpha pointers, N, lambda, T, prec, ckpt_every, kernel
 * family and tile variants). If ws holds such a tape it is used; otherwise
 * the backward first runs the forward pass into ws itself (and records it).
 * Calls of this library that write ws for anything else drop the record;
 * the caller must not modify ws, X or alpha's values in between (the record
 * cannot see writes from outside the library). */
SLISTA_API int slista_backward(const slista_dict* dict, const float* X, int N, float lambda,
                               const float* alpha, int T, int prec, const float* dZ, const float* dF,
                               float* dalpha, int ckpt_every, void* ws, size_t ws_bytes, void* stream);

/* Forward and backward of the mean loss (Eq. (15)) in one call: Z, F (as
 * slista_forward with f_trace = 0; may be NULL), loss (may be NULL) and
 * dalpha = d loss / d alpha (required). ckpt_every must be >= 1. */
SLISTA_API int slista_forward_backward(const slista_dict* dict, const float* X, int N, float lambda,
                                       const float* alpha, int T, int prec, float* Z, float* F,
                                       float* loss, float* dalpha, int ckpt_every, void* ws,
                                       size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Checks of a result
 *
 * slista_kkt: per sample, in FP64 on the device, the optimality conditions of
 * the Lasso (Lemma 2.1, Eq. (3)): with r_j = D_j^T (x_i - D z_i),
 *     kkt[i] = max_j ( |r_j - lambda sign z_ij|   if z_ij != 0,
 *                      max(|r_j| - lambda, 0)     if z_ij == 0 ),
 * zero exactly at the Lasso solution, and F[i] = F_{x_i}(z_i) (Eq. (1)),
 * both from the FP32 values of D, X and Z with every product and sum in FP64.
 * X device FP32 [N, n], Z device FP32 [N, m], kkt device FP64 [N], F device
 * FP64 [N] or NULL. n <= 8192 (SLISTA_ENOTSUP above). No workspace.
 *
 * slista_lambda_max: lambda_max (Section 2): below it the Lasso solution of a
 * sample is non-zero, at or above it exactly zero. Writes
 *     lam_max_rows[i] = ||D^T x_i||_inf  (device FP32 [N], or NULL),
 *     *lam_max = max_i lam_max_rows[i]   (device FP32 [1]),
 * from the same FP32 correlation product c = D^T x (same kernel and order)
 * that the forward pass uses, so that any lambda >= *lam_max gives
 * z^(t) = 0 exactly in every layer. Workspace of
 * slista_lambda_max_workspace_size bytes, 256-byte aligned.
 * ------------------------------------------------------------------------- */
SLISTA_API int slista_kkt(const slista_dict* dict, const float* X, int N, float lambda, const float* Z, double* kkt,
                          double* F, void* stream);
SLISTA_API int slista_lambda_max_workspace_size(const slista_dict* dict, int N, size_t* bytes);
SLISTA_API int slista_lambda_max(const slista_dict* dict, const float* X, int N, float* lam_max, float* lam_max_rows,
                                 void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Uneven batches: many independent Lasso problems (each its own dictionary,
 * n, m, N, lambda and steps; one common T) run forward + backward of their
 * mean losses together. Problems are grouped by column-pass bucket (m_pad up
 * to 256, 512, 1024, 2048); each bucket runs as one persistent launch per
 * phase over a work list of (problem, tile) pairs ordered longest first, and
 * the buckets run concurrently: each on a stream of the batch's own, forked
 * from the caller's stream and joined back into it with events (a captured
 * graph has one branch per bucket). `prec` may carry an FP32 tail
 * (SLISTA_BF16_FP32_TAIL).
 *
 * Usage: slista_batch_create -> slista_batch_workspace_size -> allocate ->
 * slista_batch_bind (builds the device argument tables and the bucket
 * streams, synchronises) -> slista_batch_run (enqueue) or
 * slista_batch_capture once and then slista_batch_replay (HIP graph) ->
 * slista_batch_destroy. A batch owns small device tables (argument records
 * and work lists), its streams and events and the captured graph; the
 * problems' buffers and the workspace stay the caller's and must outlive the
 * batch's use of them.
 * ------------------------------------------------------------------------- */
typedef struct {
  const slista_dict* dict;   /* dictionary of this problem (m_pad <= 2048) */
  const float* X;            /* device FP32 [N, n] */
  int N;                     /* >= 1 */
  float lambda;              /* finite, > 0 */
  const float* alpha;        /* device FP32 [T] */
  float* Z;                  /* device FP32 [N, m] out: z^(T) */
  float* F;                  /* device FP32 [N] out: F(z^(T)), or NULL */
  float* loss;               /* device FP32 [1] out: mean F, or NULL */
  float* dalpha;             /* device FP32 [T] out: d(mean F)/d alpha */
} slista_problem;

typedef struct slista_batch slista_batch;

/* Plan a batch of P >= 1 problems (the array is copied). ckpt_every >= 1. */
SLISTA_API int slista_batch_create(const slista_problem* problems, int P, int T, int prec, int ckpt_every,
                                   slista_batch** out);
SLISTA_API int slista_batch_workspace_size(const slista_batch* batch, size_t* bytes);
/* Attach a workspace (256-byte aligned, >= slista_batch_workspace_size) and
 * upload the argument tables; synchronises `stream`. */
SLISTA_API int slista_batch_bind(slista_batch* batch, void* ws, size_t ws_bytes, void* stream);
/* Enqueue forward + backward of every problem on `stream`. */
SLISTA_API int slista_batch_run(slista_batch* batch, void* stream);
/* Record slista_batch_run into a HIP graph owned by the batch (stream
 * capture on `stream`; nothing runs). Replaces a previous capture. */
SLISTA_API int slista_batch_capture(slista_batch* batch, void* stream);
/* Launch the captured graph on `stream`. */
SLISTA_API int slista_batch_replay(slista_batch* batch, void* stream);
/* Autotune a bound batch: for each column-pass bucket in turn, run the whole
 * batch once per tile variant (after a warm-up run) and keep the fastest;
 * records the choices in the table slista_autotune fills. Writes the variant
 * of the buckets np = 1, 2, 4, 8 to variants[0..3] (0: no such bucket) if
 * variants is not NULL. Overwrites the batch's outputs; releases a captured
 * graph (capture again afterwards). Synchronises. */
SLISTA_API int slista_batch_autotune(slista_batch* batch, void* stream, int* variants);
SLISTA_API int slista_batch_destroy(slista_batch* batch);

/* One call for a whole batch: forward + backward of every problem (as
 * slista_batch_run). On the first call with a given problem array (its
 * contents), T, prec, ckpt_every and workspace the library plans the batch
 * (argument tables, work lists: device allocations and a synchronisation)
 * and, with use_graph != 0, records it into a HIP graph on a stream of its
 * own; later calls with the same key only launch that graph (use_graph) or
 * the batch's kernels on `stream`. Up to 8 plans are kept, least recently
 * used dropped first; slista_batched_release drops all of them (and
 * synchronises the device). The workspace must hold
 * slista_batched_workspace_size bytes (256-byte aligned) and must not be
 * used for anything else while its plan is kept. Thread-safe; calls that
 * share a workspace must not overlap. */
SLISTA_API int slista_batched_workspace_size(const slista_problem* problems, int P, int T, int prec, int ckpt_every,
                                             size_t* bytes);
SLISTA_API int slista_batched_fwd_bwd(const slista_problem* problems, int P, int T, int prec, int ckpt_every,
                                      void* ws, size_t ws_bytes, void* stream, int use_graph);
SLISTA_API int slista_batched_release(void);

/* ---------------------------------------------------------------------------
 * Options (process-wide, not thread-safe; set before enqueuing work)
 *
 * SLISTA_OPT_KERNEL_FAMILY: which kernels run the layers.
 *   0 (default) automatic: the persistent kernels (one workgroup carries a
 *     tile of samples through all layers) when m_pad <= 2048, else the
 *     per-layer kernels (one fused contraction launch per layer);
 *   1 always the per-layer kernels;
 *   2 the persistent kernels where they apply.
 * Both families compute bitwise-identical iterates and step-size gradients,
 * but keep the forward's tape in different layouts (per-layer: row-major;
 * persistent: four rows of a column together). The tape record (see
 * slista_backward) includes the family and the tile variants, so a backward
 * call under other settings than its forward recomputes the tape instead of
 * reading the other layout.
 * ------------------------------------------------------------------------- */
#define SLISTA_OPT_KERNEL_FAMILY 1
/* SLISTA_OPT_PERSIST_VARIANT: tile configuration of the persistent kernels.
 *   0 (default) the library's choice for (precision, m);
 *   1 tiles of 64 samples (32 for FP32 with m_pad > 512, 16 above 1024),
 *     one workgroup per CU;
 *   2 tiles of half that many samples, two workgroups per CU (m_pad <= 1024);
 *   3 the tiles of variant 1 in one 8-wave workgroup, rows split in two
 *     (m_pad <= 1024);
 *   4 the tiles of variant 1 in one 8-wave workgroup, columns split in
 *     eight 32-column slabs.
 * Codes Z are bitwise identical across variants; F and dalpha differ only
 * by the grouping of their partial sums. A variant that does not exist for
 * the dictionary's m_pad falls back to the default. */
#define SLISTA_OPT_PERSIST_VARIANT 2
/* SLISTA_OPT_CHECK_FINITE: 1 = count NaN/Inf in the inputs (D, X, alpha,
 * dZ, dF) and outputs (Z, F, loss, dalpha) of slista_dict_create,
 * slista_forward, slista_backward and slista_forward_backward on the device;
 * each such call then synchronises its stream and returns
 * SLISTA_ENONFINITE if any was found (outputs are written regardless).
 * 0 (default) = no checks, no synchronisation. Not for use during stream
 * capture. */
#define SLISTA_OPT_CHECK_FINITE 3

/* Options are process-wide: set them before other threads call the library.
 * The autotuners use per-thread overrides while timing, and the tuning table
 * they fill is shared and guarded, so tuning in one thread leaves the
 * options other threads see unchanged. Calls on one stream are ordered by it;
 * calls that share a workspace must not overlap. */
SLISTA_API int slista_set_option(int option, int value);

/* ---------------------------------------------------------------------------
 * FISTA (Beck & Teboulle), the accelerated baseline of the paper's Figures 2
 * and D.2: from z^0 = y^0 = 0, for t = 0 .. T-1
 *   z^{t+1} = ST(y^t - alpha_t (G y^t - c), lam alpha_t),
 *   y^{t+1} = z^{t+1} + beta_t (z^{t+1} - z^t),
 * beta_t = (tau_t - 1) / tau_{t+1}, tau_0 = 1, tau_{t+1} = (1 + sqrt(1 +
 * 4 tau_t^2)) / 2 (computed on the device). Forward only. For m_pad <= 512
 * (and the automatic or persistent kernel family) one persistent launch
 * carries each tile's z and y through all layers (tile variants 2 and 4);
 * otherwise one per-layer launch per layer (G y^t on MFMA in the given
 * precision, the update fused). Both give bitwise-equal codes. Z [N, m] out;
 * F [N] (F(z^T)) and loss (mean F) out if not NULL. Workspace of
 * slista_fista_workspace_size bytes, 256-byte aligned. Errors as for
 * slista_forward.
 * ------------------------------------------------------------------------- */
SLISTA_API int slista_fista_workspace_size(const slista_dict* dict, int N, int T, int prec, size_t* bytes);
SLISTA_API int slista_fista(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha,
                            int T, int prec, float* Z, float* F, float* loss, void* ws, size_t ws_bytes,
                            void* stream);

/* ---------------------------------------------------------------------------
 * Oracle-ISTA (Section 3, Algorithm 1): per sample and layer, S = supp(z^t),
 * L_S = greatest eigenvalue of G restricted to S (L_S = L for an empty
 * support), by Lanczos in FP64 from a fixed start vector: the largest
 * eigenvalue of the Lanczos tridiagonal matrix, evaluated every 8 steps,
 * rises to L_S; the recurrence stops when two evaluations agree to
 * power_rtol (relative), after min(|S|, max_power_iter, 128) steps, or when
 * the Krylov space is exhausted. The step 1/L_S is taken when the support
 * condition (*)
 * holds and 1/L otherwise. For z_j = 0 the condition fails exactly when
 * |(G z^t - c)_j| > lam, whatever the step, so one contraction per layer
 * decides it. L: the dictionary's Lipschitz constant (slista_dict_lipschitz).
 * Z [N, m] out; F [N] (F(z^T)) and loss out if not NULL; steps: device
 * [T, N] (the step each sample took at each layer) or NULL. Per-layer
 * kernels; m <= 2048. Workspace of slista_oista_workspace_size bytes.
 * ------------------------------------------------------------------------- */
SLISTA_API int slista_oista_workspace_size(const slista_dict* dict, int N, int T, int prec, size_t* bytes);
SLISTA_API int slista_oista(const slista_dict* dict, const float* X, int N, float lambda, double L, int T, int prec,
                            int max_power_iter, double power_rtol, float* Z, float* F, float* loss, float* steps,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Coupled LISTA (Section 4, Eq. (11)-(12)): T layers with their own
 * parameters theta_t = (W_t, alpha_t, beta_t), from z^(0) = 0,
 *     z^(t+1) = ST(z^(t) - alpha_t W_t^T (D z^(t) - x), beta_t lambda),
 * the architecture whose deep layers Theorem 4.4 shows must reduce to
 * Step-LISTA (alpha_t W_t -> beta_t D). W_t = D and alpha_t = beta_t give
 * slista_forward's recursion.
 *
 * Computed in the factored form: per layer the residual R = Z D^T - X (a
 * contraction over m) and R W_t (over n), both on MFMA in the given
 * precision, with the soft-threshold and the objective partials fused into
 * their epilogues. Where a 32-sample tile fits in LDS (n_pad, m_pad up to a
 * few hundred) persistent kernels carry each tile through all layers in one
 * launch per direction; otherwise, or with SLISTA_OPT_KERNEL_FAMILY = 1, one
 * launch per contraction. The two families keep different tapes in ws, so a
 * backward call must see the family of its forward call.
 *
 *   W      device FP32 [T, n, m] (row-major per layer; W_t has D's shape).
 *   alpha, beta  device FP32 [T] (alpha_t, beta_t > 0 is a precondition).
 *   Z      device FP32 [N, m] out: z^(T).
 *   F      device FP32 [N] out or NULL: F_{x_i}(z_i^(T)) (Eq. (1)) from the
 *          FP32 residual, accumulated in FP64.
 *   loss   device FP32 [1] out or NULL: mean_i F_{x_i}(z_i^(T)) (Eq. (15)).
 *   tape   nonzero: keep z^(0..T) and D z^(t) - x for slista_lista_backward.
 *   ws     device workspace of slista_lista_workspace_size(dict, N, T,
 *          prec, tape) bytes, 256-byte aligned; it also holds the operand
 *          copies of D and W that the backward reads.
 *
 * slista_lista_backward differentiates J = sum_i dF_i F_{x_i}(z_i^(T)) +
 * <dZ, Z^(T)> (dF [N] and dZ [N, m] device, each may be NULL but not both)
 * with respect to every layer's parameters: dW device FP32 [T, n, m] (NULL
 * = skip the weight gradient), dalpha and dbeta device FP32 [T]. The
 * derivative of ST is 1 where |u| > beta_t lambda and 0 elsewhere; sign(0) =
 * 0 in the sub-gradient of |z|. The weight gradient dW_t = -alpha_t sum_i
 * r_i v_i^T is a sum over the samples, computed with FP32 operands in both
 * precisions. Precondition: ws holds the tape of a slista_lista_forward call
 * with tape != 0 and the same dict, N, lambda, W, alpha, beta, T, prec and
 * kernel family.
 * slista_lista_forward_backward does both for the mean loss (dF_i = 1/N).
 *
 * Errors: SLISTA_EINVAL for a NULL dict or required pointer, N or T out of
 * range, lambda not finite and > 0, an unknown precision, or a short or
 * misaligned workspace. N = 0 writes zero gradients and loss.
 * ------------------------------------------------------------------------- */
SLISTA_API int slista_lista_workspace_size(const slista_dict* dict, int N, int T, int prec, int tape, size_t* bytes);
SLISTA_API int slista_lista_forward(const slista_dict* dict, const float* X, int N, float lambda, const float* W,
                                    const float* alpha, const float* beta, int T, int prec, float* Z, float* F,
                                    float* loss, int tape, void* ws, size_t ws_bytes, void* stream);
SLISTA_API int slista_lista_backward(const slista_dict* dict, int N, float lambda, const float* alpha,
                                     const float* beta, int T, int prec, const float* dZ, const float* dF, float* dW,
                                     float* dalpha, float* dbeta, void* ws, size_t ws_bytes, void* stream);
SLISTA_API int slista_lista_forward_backward(const slista_dict* dict, const float* X, int N, float lambda,
                                             const float* W, const float* alpha, const float* beta, int T, int prec,
                                             float* Z, float* F, float* loss, float* dW, float* dalpha, float* dbeta,
                                             void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Learning the step sizes (Appendix D, "Training the networks"): full-batch
 * sub-gradient descent on the mean loss of Eq. (15) with a backtracking
 * learning rate. From steps alpha with loss J and gradient g, each iteration
 * tries alpha' = max(alpha - eta g, 0) (FP64 arithmetic, rounded to FP32):
 * if J(alpha') < J it is accepted and eta doubles, otherwise eta halves and
 * the next candidate is tried, at most max_halvings times; an iteration with
 * no decrease ends the loop. J is the FP64 mean of the per-sample objectives.
 *
 * alpha   device [T], in: the starting steps, out: the learned steps.
 * Z       device [N, m], out: the codes of the last evaluated candidate.
 * losses  host [iters + 1] or NULL: J at the start and after each accepted
 *         iteration; *accepted (host, may be NULL) = accepted iterations;
 *         *lr_out (host, may be NULL) = the final learning rate.
 * ws      device workspace of slista_train_workspace_size bytes, 256-byte
 *         aligned (the forward/backward workspace with the full tape plus
 *         the gradient, the candidate and the loss weights).
 * Synchronises `stream` once per candidate (the accept test is on the host).
 * Errors: SLISTA_EINVAL for NULL pointers, N or T < 1, iters < 0, lr not
 * finite and positive, max_halvings outside [0, 1000], a short or misaligned
 * workspace, or kernel timing switched on.
 * ------------------------------------------------------------------------- */
SLISTA_API int slista_train_workspace_size(const slista_dict* dict, int N, int T, int prec, size_t* bytes);
SLISTA_API int slista_train(const slista_dict* dict, const float* X, int N, float lambda, float* alpha, int T,
                            int prec, int iters, double lr, int max_halvings, float* Z, double* losses,
                            int* accepted, double* lr_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Autotuning of the persistent kernels' tile variant
 *
 * slista_autotune runs slista_forward_backward once per tile variant
 * available for this dictionary (after one warm-up call each), times two
 * calls of each with HIP events on `stream`, and records the fastest in a
 * process-wide table keyed by (precision, column-pass bucket of m_pad,
 * floor(log2 N)). While SLISTA_OPT_PERSIST_VARIANT is 0, later calls with a
 * matching key use the recorded variant. Writes the chosen variant to *best
 * and, if ms is not NULL, the mean milliseconds per call of variants 1..4 to
 * ms[0..3] (0 for a variant that does not apply). Arguments as for
 * slista_forward_backward (Z and dalpha are overwritten). Synchronises.
 * slista_tune_save / slista_tune_load write / read the table as text, one
 * "precision np log2N variant" record per line.
 * ------------------------------------------------------------------------- */
SLISTA_API int slista_autotune(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha,
                               int T, int prec, int ckpt_every, float* Z, float* dalpha, void* ws, size_t ws_bytes,
                               void* stream, int* best, double* ms);
SLISTA_API int slista_tune_save(const char* path);
SLISTA_API int slista_tune_load(const char* path);

/* ---------------------------------------------------------------------------
 * Kernel timing (diagnostics)
 *
 * While recording is on, the library brackets every launch it makes with a
 * pair of HIP events on the launch stream, keyed by kernel class:
 *   0 correlation product c = D^T x     1 forward layer (fused)
 *   2 objective F(z^T) (fused)          3 backward seed (fused)
 *   4 backward layer (fused)            5 elementwise and reductions
 * slista_profile_end synchronises on the recorded events and returns, per
 * class, the number of launches and the summed event-measured time in
 * milliseconds. Up to 65536 launches are recorded per begin/end pair; later
 * launches are counted in *dropped. Recording creates HIP events, so it must
 * not be on during stream capture. Process-wide, not thread-safe.
 * ------------------------------------------------------------------------- */
#define SLISTA_PROFILE_KINDS 6

SLISTA_API int slista_profile_begin(void);

/* launches[6], total_ms[6] (host arrays); dropped may be NULL. */
SLISTA_API int slista_profile_end(int* launches, double* total_ms, int* dropped);

#ifdef __cplusplus
}
#endif

#endif /* SLISTA_H_ */
