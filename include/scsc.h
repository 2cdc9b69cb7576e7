/*
 * scsc.h -- C ABI of the MI355X (gfx950) stochastic convolutional sparse coding library.
 *
 * Method: Xiong, Richtarik, Heidrich, "Stochastic Convolutional Sparse Coding"
 * (VMV 2019).  The library computes the data-parallel hot path of that method:
 * the Bernoulli-subsampled code update (Sec. 3.1, eqs. 2-4, solved here by
 * proximal gradient), the filter update of eq. (5), the online surrogates of
 * eqs. (8)-(9), and the objective of eq. (1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller unless
 *   the comment says "host".  The library never frees caller memory.  It owns
 *   device workspaces inside the handle and grows them on demand.
 * Stream.  Work is enqueued on the handle's HIP stream.  Calls that return
 *   host values (objective, statistics, L_d, the surrogate count) synchronise
 *   that stream before returning; the others are asynchronous.  With eager
 *   launches some work of a call runs on two further streams that the handle
 *   owns (same device, default priority): two of three parts of a code step's
 *   images (one of two for two images), and in the online filter step the
 *   B_bar increment, the corner products and the power iteration.  They are
 *   forked from and joined back to the handle's stream with events inside the
 *   call, so stream order is as if all ran on the handle's stream.  Graph
 *   replay and per-kernel timing keep one stream.
 * Errors.  Every int-returning function returns CSC_OK (0) or a negative
 *   csc_status.  Arguments are validated before any work is enqueued: on
 *   CSC_EINVAL / CSC_EUNSUPPORTED no output has been written.  The message of
 *   the last failure is available from csc_last_error().
 * Images.  A call processes a batch of n images of sizes H_i x W_i (they may
 *   differ).  Packed layouts:
 *     x, r, y, W (observation mask) : image i at offset off_i = sum_{j<i} H_j W_j,
 *                                     row-major [H_i][W_i];
 *     z (codes), g                  : image i at offset K * off_i, as [K][H_i][W_i];
 *     d (filters), G                : [K][m][m], row-major; m odd, anchor at the centre.
 * Operators (Sec. 3.1 and eq. 5; zero outside each image, "same" size, c = m / 2):
 *     (D z)[p]     = sum_k sum_{s in [-c,c]^2} d_k[s] z_k[p - s]        (synthesis)
 *     (D^T r)_k[q] = sum_s d_k[s] r[q + s]                              (adjoint)
 *     (Z^T r)_k[s] = sum_q z_k[q] r[q + s]                              (filter correlation)
 *   with d_k[s] = d[k][s_y + c][s_x + c].
 * Subsampling (eq. 2).  Coordinate (k, y, x) of image i is selected iff
 *   word (l & 3) of Philox4x32-10(counter = (lo32(l >> 2), hi32(l >> 2),
 *   index_base + i, draw), key = (lo32(seed), hi32(seed))) is below
 *   floor(p * 2^32), where l = (y * W_i + x) * K + k.  (Philox: Salmon et al.,
 *   SC'11.)  The selection depends only on (seed, draw, image index, k, y, x).
 * Supported sizes: 1 <= K <= 1024, m in {3, 5, 7, 9, 11}, 1 <= H, W,
 *   total pixels < 2^31, total selected coordinates < 2^32.
 */
#ifndef SCSC_H
#define SCSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSC_VERSION 100 /* 1.00 */

typedef struct csc_ctx *csc_handle;

typedef enum {
    CSC_OK = 0,
    CSC_EINVAL = -1,       /* invalid argument (nothing written)              */
    CSC_ENOMEM = -2,       /* device workspace allocation failed (or would     *
                            * exceed the limit SCSC_WORKSPACE_LIMIT, in bytes,  *
                            * that the environment held at csc_create)          */
    CSC_EHIP = -3,         /* a HIP runtime call or kernel launch failed      */
    CSC_EUNSUPPORTED = -4  /* valid but unsupported size / option             */
} csc_status;

typedef enum {
    CSC_FP32 = 0, /* FP32 operands and accumulation                                        */
    CSC_BF16 = 1  /* synthesis, adjoint and filter-gradient contractions with BF16 operands
                     on the matrix cores and FP32 accumulation; codes, filters and the
                     residual stay FP32                                                    */
} csc_precision;

/* A batch of images (host struct). */
typedef struct {
    int32_t n;          /* number of images, >= 1                                  */
    const int32_t *hw;  /* host array of 2n ints: H_0, W_0, H_1, W_1, ...           */
    int32_t index_base; /* image i uses image index index_base + i in the sampler   */
} csc_images;

/* Statistics of one code step (host struct, filled when non-NULL). */
typedef struct {
    int64_t sampled;      /* |S|: selected coordinates, summed over images                */
    int64_t nnz;          /* non-zero codes after the step                                 */
    double L_z;           /* Lipschitz bound used (0 when the caller passed a step)        */
    double step;          /* step size used                                                */
    int64_t nnz_iter_sum; /* sum over the iterations of the non-zero count entering each
                             iteration's synthesis (the work of the synthesis kernel)      */
} csc_code_stats;

/* Online surrogates of eq. (8), kept as unscaled sums:
 *   C_bar = sum_t sum_{i in batch t} Z_i^T W_i Z_i,  B_bar = sum_t sum_i Z_i^T W_i x_i,
 * so that C^t = C_bar / t and B^t = B_bar / t equal the recursion of eq. (8).
 * C_bar is symmetric: only its K (K + 1) / 2 blocks (k, k2 >= k) of m^2 x m^2
 * entries are stored, in row-major order of the upper triangle, each in the lag
 * layout (csc_surrogate_index gives the position of any dense entry; entry
 * (k, s; k2, s2) with k > k2 is the stored entry (k2, s2; k, s)).  B is
 * [K][m][m].  t and Ld_sum live on the host and are updated by csc_dict_step.
 * Start from C = 0, B = 0, t = 0, Ld_sum = 0. */
typedef struct {
    double *C;     /* device, csc_surrogate_size(K, m) doubles                       */
    double *B;     /* device, K*m*m doubles                                          */
    int64_t t;     /* mini-batches accumulated so far                                */
    double Ld_sum; /* sum over batches of the power-iteration estimate of L_d        */
} csc_surrogate;

/* ---- handle ---------------------------------------------------------------- */

/* Create a handle bound to HIP device `device` and stream `stream` (a
 * hipStream_t; NULL = the default stream).  *out receives the handle. */
int csc_create(csc_handle *out, int device, void *stream);
/* Release the handle and its workspaces (synchronises its stream). */
int csc_destroy(csc_handle h);
/* Rebind the handle to another stream of the same device. */
int csc_set_stream(csc_handle h, void *stream);
/* Message of the last failure on this handle ("" if none).  Owned by the handle. */
const char *csc_last_error(csc_handle h);
/* CSC_VERSION of the built library. */
int csc_version(void);

/* ---- hot path ---------------------------------------------------------------- */

/* Code update for every image of the batch: eqs. (2)-(4).
 * Draws the selection S (see "Subsampling"), starts from z restricted to S,
 * runs n_iter proximal-gradient iterations on the subsampled LASSO of eq. (3)
 *     r = W (x - D z);  u = z + step * D^T r;  z = sign(u) max(|u| - step*lambda, 0) on S,
 * with every coordinate off S held at zero, and writes the upsampled codes
 * (eq. 4) back to z (dense [K][H][W] per image; in/out).
 *   x      : images, packed, FP32.                W : observation mask (0/1 bytes), or NULL = all ones.
 *   d      : filters [K][m][m], FP32.             z : codes, packed, FP32, in/out.
 *   lambda : L1 weight, >= 0.                     p : sampling rate in (0, 1].
 *   seed, draw : sampler key and counter word (the outer iteration or mini-batch index).
 *   n_iter : proximal-gradient iterations, >= 0.
 *   step   : > 0 to force a step; <= 0 selects 1 / L_z with L_z from csc_lipschitz_code
 *            (max_side = the largest image side of the batch).
 *   precision : csc_precision.  CSC_BF16: per 16 x 16 pixel tile the adjoint correlation
 *            is one GEMM on the matrix cores (filters x pixels x taps) and the synthesis
 *            one GEMM per tap row (taps x pixels x filters) followed by a shifted sum,
 *            with d, r and z rounded to BF16 and FP32 accumulation; the selected-set
 *            update, the residual and the codes stay FP32.
 *   stats  : host, may be NULL (filling it synchronises). */
int csc_code_step(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                  const float *d, int K, int m, float *z, double lambda, double p,
                  uint64_t seed, uint32_t draw, int n_iter, double step, int precision,
                  csc_code_stats *stats);

/* Code update with the unselected coordinates held (Sec. 3.1, the paragraph on
 * the randomization: each iteration changes only the pDK sampled variables and
 * the rest remain unchanged).  As csc_code_step, except that z starts from its
 * own values, the coordinates off S keep them throughout, and their codes enter
 * every residual:
 *     r = W (x - D z),  z = z_prev off S,
 * which the library forms as r = W (x_eff - D z_S) with x_eff = x - D z_off
 * (one synthesis of the held codes, in `precision`, before the iterations).
 * Only the coordinates in S are written back to z; the others are untouched.
 * Arguments, layouts, ownership and errors as csc_code_step; stats counts the
 * sample (sampled, nnz of the codes on S). */
int csc_code_step_hold(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                       const float *d, int K, int m, float *z, double lambda, double p,
                       uint64_t seed, uint32_t draw, int n_iter, double step, int precision,
                       csc_code_stats *stats);

/* Code update by the paper's solver (Sec. 3.2, the paragraph after Alg. 1): ADMM
 * on the subsampled LASSO of eq. (3), splitting the data term from the L1 term.
 * With A = W D M^T restricted to the selection S (drawn as in csc_code_step),
 * scaled dual u and split variable v, each of n_admm iterations does
 *     zt: n_cg conjugate-gradient iterations on (A^T A + rho I) zt = A^T W x + rho (v - u),
 *         warm-started from the previous zt;
 *     zh = alpha zt + (1 - alpha) v   (over-relaxation);
 *     v  = sign(zh + u) max(|zh + u| - lambda / rho, 0);   u = u + zh - v.
 * zt and v start from z restricted to S, u from 0; v is written back (zero off S).
 *   rho   : > 0, or <= 0 for the paper's 10 * lambda (then lambda must be > 0).
 *   alpha : in (0, 2); the paper uses 1.8.   n_admm, n_cg >= 0 (the paper: 10 ADMM iterations).
 *   FP32 throughout (the CG dot products in FP64, their scalars in device memory).
 *   stats : sampled = |S|, nnz of the result, step = rho; L_z and nnz_iter_sum are 0.
 * Other arguments, layouts, ownership and errors as csc_code_step. */
int csc_code_step_admm(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                       const float *d, int K, int m, float *z, double lambda, double p,
                       uint64_t seed, uint32_t draw, int n_admm, int n_cg, double rho, double alpha,
                       csc_code_stats *stats);

/* Filter update.
 * sur == NULL: batch problem eq. (5), n_iter projected-gradient steps
 *     d <- P(d + step * sum_i Z_i^T W_i (x_i - Z_i d)),   P = projection onto ||d_k|| <= 1,
 *   step <= 0 selects 1 / L_d, L_d = power-iteration estimate (n_power iterations from
 *   the normalised all-ones vector, last Rayleigh quotient) of lambda_max(A):
 *   with an observation mask A = sum_i Z_i^T W_i Z_i; without one A is the
 *   zero-padded normal matrix (codes embedded in c zero pixels), whose entry
 *   (k, s; k2, s2) is the lag sum sum_q z_k[q] z_k2[q + s - s2]; it dominates
 *   sum_i Z_i^T Z_i, so 1 / L_d stays a descent step.  When L_d = 0 the codes are
 *   all zero and d is only projected.
 * sur != NULL: online problem, eqs. (8)-(9): C_bar += sum_i Z_i^T W_i Z_i,
 *   B_bar += sum_i Z_i^T W_i x_i, t += 1, Ld_sum += L_d(this batch); then n_iter steps
 *     d <- P(d - (C_bar d - B_bar) / Ld_sum)      (= P(d - (C^t d - B^t) / (Ld_sum / t))).
 *   step is ignored in this mode.
 *   precision : CSC_BF16 computes the batch gradient Z^T W r (and, with an observation
 *     mask, the power-iteration products Z^T y) on the matrix cores with BF16 operands and
 *     FP32 accumulation; the surrogates, their products and the lag-sum power iteration
 *     are FP64 in both precisions.
 *   z : codes, packed, FP32 (read only).   d : filters, in/out.
 *   L_d_out : host, may be NULL; receives this batch's L_d (synchronises). */
int csc_dict_step(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                  const float *z, float *d, int K, int m, csc_surrogate *sur, int n_iter,
                  double step, int n_power, int precision, double *L_d_out);

/* One step of the online algorithm (Alg. 2) on a mini-batch, in one call: the codes of
 * eqs. (3)-(4) from zero by n_iter ISTA iterations on the Bernoulli sample (as
 * csc_code_step with z = 0 on entry), then the surrogate update of eq. (8) and n_dict_iter
 * steps of eq. (9) on the filters (as csc_dict_step with sur).  The result equals those two
 * calls in sequence; joined, the filter step takes the code step's final lists instead of
 * rebuilding them from the dense codes, and the host waits for the GPU twice instead of
 * three times (the selection count, then L_d together with the code statistics).
 *   d : filters, in/out (the code step reads the filters given, the filter step updates them).
 *   z : codes, out, packed [K][pixels] per image; may be NULL (the codes then stay on the
 *       device as lists only and are not written out).
 *   sur : surrogates (required), updated as by csc_dict_step.
 *   n_dict_iter >= 0 : filter iterations (csc_dict_step's n_iter); n_power >= 1.
 *   stats, L_d_out : host, may be NULL; as csc_code_step and csc_dict_step fill them.
 *   Other arguments as csc_code_step.  Argument errors are reported before any output is
 *   written; a failure after the code step has run leaves d and sur as the failing
 *   filter step left them. */
int csc_online_step(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                    float *d, int K, int m, float *z, double lambda, double p, uint64_t seed,
                    uint32_t draw, int n_iter, double step, int precision, csc_surrogate *sur,
                    int n_dict_iter, int n_power, csc_code_stats *stats, double *L_d_out);

/* Objective of eq. (1) summed over the batch, in FP64:
 *   F = sum_i 1/2 ||W_i (x_i - D z_i)||^2 + lambda sum_i ||z_i||_1.
 * f_out (host) receives F; terms_out (host, may be NULL) receives {data term, L1 norm}.
 * Synchronises. */
int csc_objective(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                  const float *d, int K, int m, const float *z, double lambda,
                  double *f_out, double *terms_out);

/* Bytes of the library's fixed device scratch array (one copy per GPU, held until the
 * process ends), used by csc_objective_noalloc. */
#define CSC_NOALLOC_SCRATCH_BYTES (8u << 20)

/* csc_objective for callers that cannot allocate device memory (code inside HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and synchronisation as csc_objective, computed by the same kernels, but the
 * call allocates nothing: the batch records, the per-tile FP64 partial sums and the two
 * reduced terms live in the fixed scratch array of CSC_NOALLOC_SCRATCH_BYTES instead of
 * the handle's workspaces, and the handle's cached batch geometry is left as it was.
 * Limit: 256*ceil(40n/256) + 256*ceil(16T/256) + 256*ceil(16T/256) + 256 bytes must not
 * exceed CSC_NOALLOC_SCRATCH_BYTES, where n is the number of images and T the number of
 * 16x16 tiles, sum_i ceil(H_i/16) ceil(W_i/16) (about 262,000 tiles, 6.7e7 pixels);
 * a larger batch returns CSC_EINVAL before any work, with nothing written.  Every call on
 * one GPU shares that GPU's scratch array: calls that overlap on one GPU (from other
 * handles, streams or threads) race and must be serialised by the caller.  Returns
 * CSC_EHIP if the scratch array's address could not be obtained when the handle was
 * created. */
int csc_objective_noalloc(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                          const float *d, int K, int m, const float *z, double lambda,
                          double *f_out, double *terms_out);

/* ---- operators and helpers --------------------------------------------------- */

/* y = D z for every image (y packed like x). */
int csc_synthesize(csc_handle h, const csc_images *im, const float *d, int K, int m,
                   const float *z, float *y, int precision);
/* g = D^T r at every coordinate (g packed like z).  CSC_BF16: BF16 operands on the
 * matrix cores, FP32 accumulation. */
int csc_adjoint(csc_handle h, const csc_images *im, const float *d, int K, int m,
                const float *r, float *g, int precision);
/* G = sum_i Z_i^T r_i  ([K][m][m]). */
int csc_filter_corr(csc_handle h, const csc_images *im, const float *z, int K, int m,
                    const float *r, float *G, int precision);
/* The selection of eq. (2) as bytes (1 = selected), packed like z. */
int csc_mask(csc_handle h, const csc_images *im, int K, double p, uint64_t seed,
             uint32_t draw, uint8_t *mask);
/* Upper bound on ||D||^2: max over the P x P DFT grid of sum_k |DFT_P(d_k)|^2, with P the
 * smallest power of two >= max_side + m - 1.  FP64.  L_out is host.  Synchronises. */
int csc_lipschitz_code(csc_handle h, const float *d, int K, int m, int max_side, double *L_out);

/* Number of doubles of the stored surrogate C for K filters of side m (= K (K + 1) / 2 m^4). */
int64_t csc_surrogate_size(int K, int m);
/* Position of the dense entry C[(k, s), (k2, s2)], where s = (sy, sx) and s2 = (sy2, sx2)
 * are tap offsets in [-c, c].  Layout: blocks (k, k2 >= k) in row-major order of the upper
 * triangle, each of m^4 doubles; inside a block, lags delta = s - s2 in [-(m-1), m-1]^2
 * row-major, each holding the (m-|delta_y|) x (m-|delta_x|) valid s, row-major.  For
 * k > k2 the position of (k2, s2; k, s) is returned.  Returns -1 when an argument is out
 * of range.  Host only. */
int64_t csc_surrogate_index(int K, int m, int k, int sy, int sx, int k2, int sy2, int sx2);

/* ---- per-kernel timing -------------------------------------------------------- */

/* Kernel classes timed by csc_profile_read. */
typedef enum {
    CSC_PK_SELECT = 0,   /* Bernoulli selection and the prefix scan of list capacities   */
    CSC_PK_GATHER = 1,   /* warm start: selected non-zero codes into lists              */
    CSC_PK_SYNTH = 2,    /* synthesis / masked residual from code lists                  */
    CSC_PK_ADJOINT = 3,  /* proximal-gradient step: adjoint at S + soft-threshold         */
    CSC_PK_SCATTER = 4,  /* upsampling of eq. (4): lists back to dense codes             */
    CSC_PK_LISTS = 5,    /* non-zero lists from dense codes                              */
    CSC_PK_CORR = 6,     /* filter correlation Z^T r (and Z^T W x) with its reduction    */
    CSC_PK_UPDATE = 7,   /* power-iteration and projected filter updates                */
    CSC_PK_SUR_ACC = 8,  /* surrogate accumulation C_bar += Z^T W Z with an observation mask */
    CSC_PK_SUR_MV = 9,   /* surrogate product C_bar d                                    */
    CSC_PK_OBJECTIVE = 10,
    CSC_PK_LIPSCHITZ = 11,
    CSC_PK_DENSE = 12,   /* dense operator helpers (csc_adjoint)                         */
    CSC_PK_SUR_LAG = 13, /* surrogate lag sums R and the band sums of the image border    */
    CSC_PK_SUR_EXPAND = 14, /* C_bar += R - band terms, all blocks                       */
    CSC_PK_SUR_CORNER = 15, /* corner-ring correction of C_bar                            */
    CSC_PK_POWER = 16,   /* power-iteration products with the lag-sum normal matrix      */
    CSC_PK_GRAPH = 17,   /* replay of the captured proximal-gradient iterations (csc_set_graph) */
    CSC_PK_COUNT = 18
} csc_kernel_class;

/* enable != 0: time every kernel class from now on, clearing previous records;
 * enable == 0: stop.  Each timed scope of a class is measured with two HIP events
 * that its kernels record themselves (hipExtLaunchKernel): the first kernel's start
 * and the last kernel's end, on the handle's stream.  A graph replay
 * (CSC_PK_GRAPH) is timed with an event pair recorded on the stream around it.
 * While profiling is on, a code step runs on the handle's stream only. */
int csc_profile_enable(csc_handle h, int enable);
/* Number of timed scopes and their summed time (milliseconds) of one kernel class
 * since profiling was enabled.  Host outputs.  Synchronises the stream. */
int csc_profile_read(csc_handle h, int kernel_class, int64_t *launches, double *total_ms);

/* ---- Unrolled proximal-gradient layers (differentiable code updates) ----------
 * One layer is one iteration of the subsampled code update of eqs. (3)-(4) with a
 * fixed selection `mask` (u8, packed like z: 1 = selected), step eta > 0 and
 * threshold eta * lambda:
 *     r = W (x - D z_in),   u = z_in + eta D^T r,   z_out = mask * shrink(u, eta * lambda).
 * Dense packed codes; x, W as in csc_code_step.  precision CSC_FP32, or CSC_BF16: every
 * product (D z, D^T r and, in the backward pass, the filter correlations) takes BF16
 * operands on the matrix cores with FP32 accumulation; codes, residuals and gradients
 * stay FP32.  z_out may alias z_in.  Asynchronous apart from list sizing, which
 * synchronises. */
int csc_ista_forward(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                     const float *d, int K, int m, const uint8_t *mask, const float *z_in, float *z_out,
                     double eta, double lambda, int precision);
/* Reverse mode of one layer, recomputing r and u from z_in (only the layer input
 * is kept between the passes).  Given g_out = dL/dz_out:
 *     g_u = g_out on {mask, |u| > eta lambda}, 0 elsewhere;   t = W (D g_u);
 *     g_z = g_u - eta D^T t   [packed like z],
 *     g_d = eta (sum_i Z(g_u)_i^T r_i - sum_i Z(z_in)_i^T t_i)   [K][m][m],
 *     g_x = eta t   [packed like x; may be NULL].
 * Z(a)^T b is the filter correlation of csc_filter_corr.  Outputs are overwritten. */
int csc_ista_backward(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                      const float *d, int K, int m, const uint8_t *mask, const float *z_in,
                      const float *g_out, double eta, double lambda, float *g_z, float *g_d, float *g_x,
                      int precision);

/* enable != 0: csc_code_step captures its n_iter proximal-gradient iterations
 * (synthesis + adjoint launches of every image of the batch) into one HIP graph
 * and replays it on later calls with the same shapes, options and workspaces;
 * x, W and d are first copied into handle-owned buffers, and the step and
 * threshold are read from device memory, so new values need no re-capture.
 * Results are identical to the eager launches.  A graph is captured only once
 * the synthesis variant is settled (autotuned or fixed).  enable == 0 (the
 * default): eager launches; the cached graph is released. */
int csc_set_graph(csc_handle h, int enable);

/* Launch-variant autotuning (tile shape / threads per output pixel) of the
 * kernels that have several variants.  enable != 0 (the default): the first
 * call with a new (kernel, m, K, batch size class) times every variant on that
 * call's own data and keeps the fastest for the handle's lifetime; this first
 * call synchronises the stream and is skipped while the stream is being
 * captured.  enable == 0: the first variant is always used and the tuned
 * choices are forgotten.  enable = -(v + 1) < 0: variant v is always used where
 * it exists (the first variant elsewhere), for testing.  Every variant computes
 * bit-identical results, so the setting changes timing only. */
int csc_set_autotune(csc_handle h, int enable);

#ifdef __cplusplus
}
#endif

#endif /* SCSC_H */
