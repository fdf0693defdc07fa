/*
 * ap.h -- C ABI of the alternating-projection (AP) solver for Gaussian-process
 * kernel systems on AMD MI355X (gfx950).
 *
 * Problem (Section 2, "Hyperparameter Training" and "Linear Solves"; Algorithm 1
 * input/output): solve the batched system K^ W = B for W = K^^{-1} B, where
 *   K^ = K + sigma^2 I,  K_ij = s * k(x_i, x_j),
 * k is an RBF or Matern kernel with one lengthscale per feature (Section 5,
 * "Datasets and Models"), B holds l right-hand sides.
 *
 * The method (Section 3, Algorithm 1): partition [n] into m = ceil(n/b) blocks
 * of b consecutive rows (the last block holds the remainder), cache a factor of
 * every diagonal block K^_{I,I} once per hyperparameter setting ("Cached
 * Cholesky Factors"), then repeat epochs of m block updates
 *   W_I <- W_I + K^_{I,I}^{-1} R_I                (eq. text_update_of_w)
 *   R   <- R   - K^_{:,I} K^_{I,I}^{-1} R_I       (eq. text_update_of_r)
 * with the block I chosen cyclically or by the modified Gauss-Southwell rule
 * I = argmax_I ||R_{I,:}||_F^2 (eq. approximate_gauss_southwell), until the mean
 * over columns of ||r_c|| / ||b_c|| is below a tolerance (Section 5,
 * "Alternating Projection Details").
 *
 * Conventions for every entry point:
 *  - Matrices are row-major. [dev] marks device (HBM) pointers, [host] host
 *    pointers. Every [dev] buffer belongs to the caller; the library never
 *    allocates or frees device memory. The handle borrows X and the workspace
 *    for its whole life.
 *  - Every call returns an ap_status. Nothing is thrown across the ABI, and
 *    nothing aborts or exits. Out-parameters are left untouched on error unless
 *    stated otherwise.
 *  - Work is enqueued on the given HIP stream in stream order. Only
 *    ap_factor_blocks, ap_solve, ap_solve_from, ap_mll_grad, ap_rel_residual
 *    and ap_residual with a non-NULL col_rel synchronize that stream
 *    (ap_batch_peek synchronizes a stream of its own). A handle is used by one host thread at a
 *    time, and calls that overlap on one handle race, except ap_batch_peek,
 *    which only reads and may watch a call running on another thread.
 *  - Errors the device detects (a non-positive pivot, a non-finite residual)
 *    are kept in a status word in the workspace and reported by the next
 *    synchronizing call.
 */
#ifndef AP_H
#define AP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AP_OK = 0,
  AP_NOT_CONVERGED = 1,      /* warning: max_epochs reached above tolerance */
  AP_ERR_INVALID_ARG = -1,   /* a pointer, size or option is out of range */
  AP_ERR_NOT_PD = -2,        /* a block K^_{I,I} has a non-positive Cholesky pivot */
  AP_ERR_NONFINITE = -3,     /* NaN or Inf reached the residual norms */
  AP_ERR_WORKSPACE = -4,     /* the workspace is smaller than ap_workspace_bytes */
  AP_ERR_HIP = -5,           /* a HIP runtime call failed */
  AP_ERR_UNSUPPORTED = -6    /* a size this build does not handle (see limits) */
} ap_status;

typedef enum { AP_RBF = 0, AP_MATERN32 = 1, AP_MATERN52 = 2 } ap_kernel;

/* Block selection (Section 3, "Block Selection"): AP_CYCLIC takes block
 * (u mod m) at update u of every epoch, starting at block 0; AP_GREEDY takes
 * argmax_I ||R_{I,:}||_F^2, ties to the lowest block index; AP_RANDOM draws
 * I uniformly from the partition: update u since the last reset (counted
 * over epochs) takes block floor(h * m / 2^32), h the high 32 bits of output
 * u of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) started from the
 * config's seed, i.e. of z = seed + (u + 1) * 0x9e3779b97f4a7c15 after
 * z ^= z >> 30, z *= 0xbf58476d1ce4e5b9, z ^= z >> 27,
 * z *= 0x94d049bb133111eb, z ^= z >> 31. An epoch is m selections in all
 * three. ap_update with an explicit block does not consume a draw. */
typedef enum { AP_CYCLIC = 0, AP_GREEDY = 1, AP_RANDOM = 2 } ap_order;

/* Arithmetic of the fused residual update (the kernel tiles K^_{:,I} and their
 * product with the block step). Block factors, block solves, W and the true
 * residual are FP64 in all; R is FP32 in all.
 *  AP_TILE_FP32:  r^2 by exact differencing of (hi, lo) FP32 features, kernel
 *                 map in FP32, product with the step on FP32 matrix cores.
 *  AP_TILE_BF16:  x.x' on BF16 matrix cores with a two-term (hi + lo) split of
 *                 every feature, kernel map in FP32, tile and step rounded to
 *                 BF16 for the product, FP32 accumulation. About 8 significant
 *                 bits per product: for well-conditioned systems only.
 *  AP_TILE_SPLIT: r^2 by exact differencing in FP32, kernel map in FP32, tile
 *                 and step each split into three BF16 terms and multiplied on
 *                 BF16 matrix cores (six partial products), FP32 accumulation
 *                 per 32 columns and FP64 across them: FP32-grade products.
 *  AP_TILE_FP64:  kernel values in FP64 (exact differencing, FP64 map) and the
 *                 product on FP64 matrix cores; only R is stored in FP32. For
 *                 systems so ill-conditioned that FP32 kernel values let the
 *                 maintained residual drift away from B - K^ W. */
typedef enum { AP_TILE_FP32 = 0, AP_TILE_BF16 = 1, AP_TILE_SPLIT = 2, AP_TILE_FP64 = 3 } ap_tile;

/* Limits of this build: 1 <= d <= 20, 1 <= l <= 32, 1 <= b <= 4096, b <= n,
 * n < 2^31. Larger sizes return AP_ERR_UNSUPPORTED. */
typedef struct {
  int64_t n;                  /* number of points, >= 1 */
  int32_t d;                  /* features per point */
  int32_t l;                  /* right-hand sides (columns of B, W, R) */
  int32_t b;                  /* block size; m = ceil(n / b) blocks */
  int32_t kernel;             /* ap_kernel */
  const double* lengthscale;  /* [host] d lengthscales, each > 0 (copied) */
  double outputscale;         /* s > 0 */
  double noise;               /* sigma^2 >= 0, added on the diagonal by index */
  int32_t order;              /* ap_order */
  int32_t tile;               /* ap_tile */
  int32_t refine_every;       /* ap_solve: replace R by the FP64 true residual
                                 after every k-th epoch; 0 = never */
  double tol;                 /* ap_solve: stop when the ratio is < tol */
  int32_t min_epochs;         /* ap_solve: never stop before this many epochs */
  int32_t max_epochs;         /* ap_solve: stop after this many epochs */
  uint64_t seed;              /* AP_RANDOM: seed of the block draws (else unused) */
} ap_config;

/* Per-problem device state, all [dev], n x l row-major:
 *  B: right-hand sides (FP32, read only), W: weights (FP64), R: residual (FP32). */
typedef struct {
  const float* B;
  double* W;
  float* R;
} ap_state;

typedef struct {
  int32_t epochs;             /* epochs run */
  int32_t refines;            /* FP64 true-residual passes run */
  double rho_maintained;      /* mean_c ||R_c|| / ||B_c|| of the maintained R */
  double rho_true;            /* the same for B - K^ W in FP64 (NaN if not computed) */
  double t_epochs;            /* seconds in epochs (HIP events) */
  double t_refine;            /* seconds in true-residual passes */
  int32_t tile;               /* ap_tile in use when the solve ended */
  int32_t escalated_at;       /* epoch after which FP64 tiles took over, -1 if never */
  int32_t restarted_at;       /* epoch after which the solve restarted from W = 0 on
                                 FP64 tiles (non-finite norms, or a drifted W whose
                                 true ratio was >= 1), -1 if never */
} ap_stats;

typedef struct ap_problem* ap_handle;

/* Bytes of device workspace a problem of this shape needs (factors m b^2 FP64
 * plus O(n (d + l)) of staging). Returns 0 if cfg is NULL or invalid. */
size_t ap_workspace_bytes(const ap_config* cfg);

/* Validate cfg, lay out the workspace, prepare the features and cache the
 * inverse of every diagonal block K^_{I,I} (Section 3, "Cached Cholesky
 * Factors": a batched FP64 Cholesky of all blocks, then the inverse from the
 * factor, so each block solve is one FP64 product).
 *  X   [dev]  n x d FP32, borrowed until ap_destroy.
 *  ws  [dev]  at least ap_workspace_bytes(cfg) bytes, borrowed; 256-byte aligned.
 *  out [host] receives the handle on AP_OK.
 *  bad_block [host, may be NULL] receives the first failing block on
 *             AP_ERR_NOT_PD.
 * The handle also keeps a stream and a small pinned host buffer of its own for
 * ap_batch_peek. Synchronizes the stream once. */
ap_status ap_factor_blocks(const ap_config* cfg, const float* X, void* ws, size_t ws_bytes,
                           hipStream_t stream, ap_handle* out, int64_t* bad_block);

/* Algorithm 1 initialization: W = 0, R = B; also caches ||B_c|| and, for the
 * greedy and random orders, makes the first selection. Asynchronous. */
ap_status ap_reset(ap_handle h, const ap_state* st, hipStream_t stream);

/* Run `epochs` epochs of m block updates on each of `count` problems (h[i],
 * st[i]); each problem's arithmetic is the same whatever count is. The
 * problems' epochs are enqueued one after another on the stream, each as that
 * handle's captured epoch graph (one replay per epoch); ap_batch_step is the
 * entry point that groups many problems into one launch per phase. After each
 * epoch the maintained-residual ratio is stored on the device (read it with
 * ap_rel_residual). Asynchronous. */
ap_status ap_epoch(const ap_handle* h, const ap_state* st, int32_t count, int32_t epochs,
                   hipStream_t stream);

/* Switch the fused update of this handle to `tile`: AP_TILE_FP64 from any
 * mode, or back to the mode it was created with (AP_ERR_INVALID_ARG
 * otherwise). The cached factors do not depend on the mode. */
ap_status ap_set_tile(ap_handle h, int32_t tile);

/* One block update on block `block` (0 <= block < m): the inner loop body of
 * Algorithm 1. Asynchronous. */
ap_status ap_update(ap_handle h, const ap_state* st, int32_t block, hipStream_t stream);

/* Synchronize the stream and read the maintained residual ratio after the last
 * epoch: *rho = mean_c ||R_c|| / ||B_c|| (a zero column of B counts 0);
 * col_ratio [host, may be NULL] receives the l per-column ratios. Returns
 * AP_ERR_NONFINITE if a norm was NaN or Inf. */
ap_status ap_rel_residual(ap_handle h, hipStream_t stream, double* rho, double* col_ratio);

/* Algorithm 1 with the stopping rule: reset, then epochs until rho < tol with
 * at least min_epochs epochs, or max_epochs. After refine_every epochs, and on
 * a tolerance hit when refine_every > 0 or the tile mode is not FP32, R is
 * replaced by the FP64 true residual (exact by Lemma residual_equality) and the
 * test is repeated on it; the interval between these scheduled true residuals
 * doubles, up to 16 refine_every, while the true and maintained ratios agree to
 * 1e-5, and returns to refine_every when they do not. If that true residual's
 * ratio and the maintained one differ by more than 5%, the rest of the solve
 * runs on FP64 tiles: from the current W when its true ratio is below 1 (the
 * ratio of W = 0), else from W = 0; if an epoch's norms are not finite, the
 * solve restarts from W = 0 on FP64 tiles (stats.tile, stats.escalated_at,
 * stats.restarted_at). The handle's tile mode on return, errors included, is
 * the one it had on entry. Synchronizes once per epoch. Returns AP_OK,
 * AP_NOT_CONVERGED or an error; out [host, may be NULL] gets the statistics. */
ap_status ap_solve(ap_handle h, const ap_state* st, hipStream_t stream, ap_stats* out);

/* Restart Algorithm 1 from the caller's W instead of W = 0 (a warm start, e.g.
 * from the solve at the previous hyperparameters of a training loop): the
 * control block as after ap_reset, W kept, R = B - K^ W as the FP64 true
 * residual (Lemma residual_equality: Algorithm 1's residual for any W), and
 * the first selection made from it. Asynchronous. */
ap_status ap_warm_start(ap_handle h, const ap_state* st, hipStream_t stream);

/* ap_solve from the caller's W: ap_warm_start in place of the reset, then the
 * same epochs, true residuals and stopping rule. */
ap_status ap_solve_from(ap_handle h, const ap_state* st, hipStream_t stream, ap_stats* out);

/* True residual B - K^ W over all n^2 kernel entries in FP64 (Lemma
 * residual_equality), written as FP32 to R_out [dev] (NULL: st->R, which
 * refines the maintained residual). col_rel [host, may be NULL] receives the l
 * ratios ||r_c|| / ||b_c|| of the FP64 values; passing it synchronizes. */
ap_status ap_residual(ap_handle h, const ap_state* st, float* R_out, double* col_rel,
                      hipStream_t stream);

/* For callers that cannot allocate device memory and keep no solver workspace
 * (code under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): ap_residual's FP64 true residual R_out = B - K^ W (Lemma
 * residual_equality) without a handle, for the kernel and hyperparameters in
 * cfg (n, d, l, kernel, lengthscale, outputscale, noise; the block size,
 * order, tile and stopping fields are not used). Same kernels as ap_residual:
 * R_out and col_rel are bitwise what ap_residual gives after ap_reset of the
 * same B.
 *  X     [dev] n x d FP32;  B [dev] n x l FP32;  W [dev] n x l FP64;
 *  R_out [dev] n x l FP32, written;
 *  col_rel [host, may be NULL] the l ratios ||r_c|| / ||b_c|| of the FP64
 *          values (passing it synchronizes the stream; pass NULL under capture).
 * Its scratch (column norms, ratios and per-workgroup column partials) is a
 * device array of AP_NOALLOC_SCRATCH_BYTES that the library holds on every GPU
 * it runs on until the process ends; the call allocates nothing. n above
 * AP_NOALLOC_MAX_N returns AP_ERR_UNSUPPORTED. All calls on one GPU share that
 * GPU's scratch, which keeps the last call's contents: calls that overlap on
 * one device (other streams, other threads) race, so the caller orders them. */
#define AP_NOALLOC_MAX_N 4194304
#define AP_NOALLOC_SCRATCH_BYTES 4198400
ap_status ap_residual_noalloc(const ap_config* cfg, const float* X, const float* B,
                              const double* W, float* R_out, double* col_rel,
                              hipStream_t stream);

/* Stochastic gradient of the negative log marginal likelihood
 * (y^T K^^{-1} y + log det K^) / 2 (Section 2, eq. loss_grad_unbiased) from a
 * solve's W = K^^{-1} B, where B = [y, z_1, .., z_P] holds the targets and
 * P = l - 1 probe vectors (zero mean, identity covariance, e.g. Rademacher):
 *   grad_theta = -1/2 w_0^T (dK^/dtheta) w_0 + 1/(2P) sum_p w_p^T (dK^/dtheta) z_p
 * (the second term absent when l = 1), for theta = the d lengthscales, the
 * outputscale and the noise, over all n^2 kernel entries in FP64 without
 * storing any of them.
 *  grad     [host] d + 2 values: d/d ell_1 .. d/d ell_d, d/ds, d/d sigma^2.
 *  partials [dev, may be NULL] ceil(n/64) x 22 FP64: the same sums over each
 *           64-row slice of the double sum (columns d + 2 .. 21 zero), which
 *           add up to grad (summed by the library in a fixed order).
 * Synchronizes the stream. AP_ERR_NONFINITE if a component is not finite. */
ap_status ap_mll_grad(ap_handle h, const ap_state* st, double* grad, double* partials,
                      hipStream_t stream);

/* Posterior mean at test points (Section 2, GP regression): with weights
 * W = K^^{-1} B from a solve, mean = K(X*, X) W, the test points' kernel
 * against the training points (no noise term). FP64 kernel values (exact
 * differencing, FP64 map) and FP64 products, on the matrix cores for l > 8.
 *  W    [dev] n x l FP64 (the state's W after ap_solve or epochs).
 *  Xs   [dev] ns x d FP32 test points (ns >= 0; 0 does nothing).
 *  mean [dev] ns x l FP64, written.
 * Asynchronous. */
ap_status ap_predict(ap_handle h, const double* W, const float* Xs, int64_t ns, double* mean,
                     hipStream_t stream);

/* Copy the cached inverse of block j, len_j x len_j FP64 row-major, to dst
 * [dev] (len_j = b, or the remainder for the last block). Asynchronous. */
ap_status ap_block_inverse(ap_handle h, int32_t j, double* dst, hipStream_t stream);

/* Per-phase timing: when enabled, HIP events are recorded on the stream around
 * every launch group of this handle, in five phases: 0 block solve, 1 fused
 * residual update, 2 greedy selection, 3 epoch-end check, 4 FP64 true
 * residual. Enabling (or disabling) clears the totals. */
ap_status ap_profile(ap_handle h, int32_t enable);

/* Synchronize the stream and read the totals since the last ap_profile call:
 * seconds [host, 5] and launches [host, 5], in the phase order above. */
ap_status ap_profile_read(ap_handle h, hipStream_t stream, double* seconds, int64_t* launches);

/* ---- Batch steps: many problems advanced together (continuous batching) ----
 *
 * A batch step gives every problem of a group its next block update of
 * Algorithm 1 (the problems may differ in n, d, l, b, kernel, hyperparameters
 * and tile mode) in grouped launches: one launch for the block solves of all of
 * them, one for the fused updates of all problems on AP_TILE_SPLIT (one launch
 * per problem on another mode), and one that advances every problem's cursor and,
 * after the last block of an epoch, runs its epoch-end check. The epoch state
 * lives on the device, so the host does not wait between steps. After the
 * check a problem is held (its updates become no-ops) while the host has to act:
 *  AP_HOLD_REFINE     an FP64 true residual is due: epoch % refine_every == 0,
 *                     or the epoch the last ap_batch_release named,
 *  AP_HOLD_TOL        rho < tol with at least min_epochs epochs,
 *  AP_HOLD_MAX        epoch == max_epochs,
 *  AP_HOLD_NONFINITE  the norms were not finite.
 * The host reads the state with ap_batch_peek, acts (for instance ap_residual
 * to replace R by the true residual and test it, ap_set_tile, ap_reset) and
 * resumes the problem with ap_batch_release. A problem's arithmetic depends
 * only on its own data and these decisions, never on the rest of the group or
 * on when the host acted: its results are bitwise those of the same problem
 * run alone. Each problem must have been ap_reset first. */
typedef enum {
  AP_RUN = 0,
  AP_HOLD_REFINE = 1,
  AP_HOLD_TOL = 2,
  AP_HOLD_MAX = 3,
  AP_HOLD_NONFINITE = 4
} ap_batch_state;

typedef struct {
  int32_t state;     /* ap_batch_state */
  int32_t epoch;     /* epochs completed since ap_reset */
  int32_t cursor;    /* block updates done in the current epoch */
  int32_t status;    /* 0, or AP_ERR_NONFINITE when the last check saw NaN/Inf */
  double rho;        /* maintained ratio after the last epoch */
  double rho_true;   /* ratio of the last FP64 true residual (ap_residual) */
} ap_progress;

/* Enqueue `steps` batch steps of the `count` problems (h[i], st[i]), 1 <= count
 * <= 32, each handle at most once, all on the device of h[0]; asynchronous on
 * `stream`. Problems on split tiles with d > 8 and problems on other tiles are
 * updated on a second stream the library keeps per device, forked from and
 * joined back to `stream` within every step, so batch steps on one device are
 * issued from one host thread at a time. Every buffer of every problem must
 * stay allocated until the work completes. */
ap_status ap_batch_step(const ap_handle* h, const ap_state* st, int32_t count, int32_t steps,
                        hipStream_t stream);

/* Snapshot of a problem's progress, read on a stream of the handle's own (it
 * does not wait for work queued on other streams), into a pinned host buffer
 * the handle keeps. The state of a held problem and every value written before
 * it was held are exact; a running problem's fields may be mid-update. Also
 * shows epoch and rho while ap_solve or ap_epoch runs. Synchronizes that stream
 * only. */
ap_status ap_batch_peek(ap_handle h, ap_progress* out);

/* Resume a held problem from the next batch step (stream order). next_refine
 * > 0 moves its next AP_HOLD_REFINE to the end of epoch next_refine (for
 * instance later when the last true residual showed no drift); 0 keeps the
 * refine_every schedule. */
ap_status ap_batch_release(ap_handle h, int32_t next_refine, hipStream_t stream);

/* Free the host-side handle. The caller frees X and the workspace afterwards. */
void ap_destroy(ap_handle h);

/* Static description of a status code. */
const char* ap_status_str(ap_status s);

/* Description of the last HIP failure behind an AP_ERR_HIP on the calling
 * thread: the failing call and the HIP error name ("" if none). Entry points
 * that launch work first take off an error that an earlier HIP call outside
 * the library left unread, so that it is not reported as theirs; the text then
 * records that error. Valid until the next call on this thread. */
const char* ap_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
