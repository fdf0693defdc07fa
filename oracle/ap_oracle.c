/*
 * FP64 CPU oracle for alternating projection (AP) on Gaussian-process kernel
 * systems (K + sigma^2 I) W = B.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package's smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU path never links,
 * loads or calls it, and the two share no source, header, table or helper.
 *
 * Source: Wu, Wenger, Jones, Pleiss, Gardner, "Large-Scale Gaussian Processes
 * via Alternating Projection" (AISTATS 2024, arXiv 2310.17137). Section and
 * equation names below refer to that paper.
 *
 * Everything is FP64, written for a reader to check against the paper by eye:
 * the kernel is evaluated by exact differencing (never the norm expansion), the
 * block factor is a hand-written Cholesky, the block solve is forward then back
 * substitution, and every residual update visits all n rows. OpenMP splits the
 * loop over rows only; each row is computed by one thread in a fixed order, so
 * results do not depend on the thread count.
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *  - noise enters by index, K^ = K + sigma^2 I (footnote to the GP regression
 *    paragraph writes an indicator on equal inputs; by index keeps K^ positive
 *    definite when inputs repeat);
 *  - RBF k = s exp(-r^2/2), Matern-3/2 k = s (1 + sqrt3 r) exp(-sqrt3 r),
 *    Matern-5/2 k = s (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r), r = ||(x - x')/ell||
 *    with one lengthscale per dimension (Section 5, "Datasets and Models");
 *  - partition: block j holds rows [j b, min((j+1) b, n)), the last block is
 *    the remainder ("Cached Cholesky Factors", "Alternating Projection Details");
 *  - cyclic order starts at block 0 in every epoch; the greedy rule breaks ties
 *    towards the lowest block index; the random rule draws each update's block
 *    from SplitMix64 (below); an epoch is m selections in every order;
 *  - stopping: mean over columns of ||r_c|| / ||b_c||, strictly below tol, after
 *    at least min_epochs epochs, or at max_epochs ("Alternating Projection
 *    Details"); a column with ||b_c|| = 0 contributes 0;
 *  - a non-positive Cholesky pivot is an error reported with its block; no
 *    jitter is added.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ap_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops use (1 without OpenMP). */
int32_t apo_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---- kernel function (Section 2 "Notation"; Section 5 kernels) ---------- */

/* Squared ARD distance r^2 = sum_k ((x_k - y_k) / ell_k)^2, exact differencing. */
static double apo_r2(const apo_config* c, const double* x, const double* y) {
  double r2 = 0.0;
  for (int k = 0; k < c->d; ++k) {
    double t = (x[k] - y[k]) / c->lengthscale[k];
    r2 += t * t;
  }
  return r2;
}

double apo_kernel(const apo_config* c, const double* x, const double* y) {
  double r2 = apo_r2(c, x, y);
  double s = c->outputscale;
  switch (c->kernel) {
    case APO_RBF:
      return s * exp(-0.5 * r2);
    case APO_MATERN32: {
      double t = sqrt(3.0) * sqrt(r2);
      return s * (1.0 + t) * exp(-t);
    }
    case APO_MATERN52: {
      double r = sqrt(r2);
      double t = sqrt(5.0) * r;
      return s * (1.0 + t + 5.0 * r2 / 3.0) * exp(-t);
    }
    default:
      return NAN;
  }
}

/* Entry (i, j) of K^ = K + sigma^2 I: the noise is added by index. */
static double apo_khat(const apo_config* c, const double* X, int64_t i, int64_t j) {
  double v = apo_kernel(c, X + i * c->d, X + j * c->d);
  if (i == j) v += c->noise;
  return v;
}

void apo_khat_block(const apo_config* c, const double* X, int64_t i0, int64_t i1,
                    int64_t j0, int64_t j1, double* out) {
  int64_t w = j1 - j0;
#pragma omp parallel for schedule(static)
  for (int64_t i = i0; i < i1; ++i)
    for (int64_t j = j0; j < j1; ++j) out[(i - i0) * w + (j - j0)] = apo_khat(c, X, i, j);
}

/* ---- partition P ("Cached Cholesky Factors") --------------------------- */

int64_t apo_num_blocks(const apo_config* c) { return (c->n + c->b - 1) / c->b; }

int64_t apo_block_start(const apo_config* c, int64_t j) { return j * (int64_t)c->b; }

int64_t apo_block_len(const apo_config* c, int64_t j) {
  int64_t s = j * (int64_t)c->b;
  int64_t e = s + c->b;
  if (e > c->n) e = c->n;
  return e - s;
}

/* ---- block factor (Section 3 "Cached Cholesky Factors") ----------------- */

/* In-place Cholesky of a len x len row-major SPD matrix: on return the lower
 * triangle holds L with A = L L^T and the strict upper triangle is zero.
 * Returns -1 on success, else the index of the first non-positive pivot. */
int64_t apo_cholesky(double* A, int64_t len) {
  for (int64_t k = 0; k < len; ++k) {
    double p = A[k * len + k];
    for (int64_t t = 0; t < k; ++t) p -= A[k * len + t] * A[k * len + t];
    if (!(p > 0.0)) return k;
    double lkk = sqrt(p);
    A[k * len + k] = lkk;
    for (int64_t i = k + 1; i < len; ++i) {
      double v = A[i * len + k];
      for (int64_t t = 0; t < k; ++t) v -= A[i * len + t] * A[k * len + t];
      A[i * len + k] = v / lkk;
    }
  }
  for (int64_t i = 0; i < len; ++i)
    for (int64_t j = i + 1; j < len; ++j) A[i * len + j] = 0.0;
  return -1;
}

/* Factor the single diagonal block j into Lj (len_j x len_j). Returns -1 on
 * success, else the non-positive pivot's index. */
int64_t apo_factor_one(const apo_config* c, const double* X, int64_t j, double* Lj) {
  int64_t s = apo_block_start(c, j), len = apo_block_len(c, j);
  apo_khat_block(c, X, s, s + len, s, s + len, Lj);
  return apo_cholesky(Lj, len);
}

/* Factor every diagonal block K^_{I,I}, I in P. Block j's factor occupies
 * L[j*b*b ...] as a len_j x len_j row-major matrix. Returns -1 on success, else
 * the first failing block, with its pivot index in *bad_pivot. */
int64_t apo_factor(const apo_config* c, const double* X, double* L, int64_t* bad_pivot) {
  int64_t m = apo_num_blocks(c);
  int64_t bb = (int64_t)c->b * c->b;
  int64_t* piv = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  /* blocks are independent: one thread per block, each factor sequential */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j = 0; j < m; ++j) {
    int64_t s = apo_block_start(c, j), len = apo_block_len(c, j);
    double* Lj = L + j * bb;
    for (int64_t i = 0; i < len; ++i)
      for (int64_t q = 0; q < len; ++q) Lj[i * len + q] = apo_khat(c, X, s + i, s + q);
    piv[j] = apo_cholesky(Lj, len);
  }
  int64_t first_bad = -1, first_piv = -1;
  for (int64_t j = 0; j < m; ++j)
    if (piv[j] >= 0) {
      first_bad = j;
      first_piv = piv[j];
      break;
    }
  free(piv);
  if (bad_pivot) *bad_pivot = first_piv;
  return first_bad;
}

/* ---- block solve (Algorithm 1, weight update) -------------------------- */

/* delta = K^_{I,I}^{-1} R_I = L^{-T} (L^{-1} R_I): forward then back
 * substitution, column by column. R_I and delta are len x l row-major. */
void apo_block_solve(const double* Lj, int64_t len, int32_t l, const double* RI, double* delta) {
  for (int32_t c = 0; c < l; ++c) {
    for (int64_t i = 0; i < len; ++i) { /* L y = r */
      double v = RI[i * l + c];
      for (int64_t t = 0; t < i; ++t) v -= Lj[i * len + t] * delta[t * l + c];
      delta[i * l + c] = v / Lj[i * len + i];
    }
    for (int64_t i = len - 1; i >= 0; --i) { /* L^T x = y */
      double v = delta[i * l + c];
      for (int64_t t = i + 1; t < len; ++t) v -= Lj[t * len + i] * delta[t * l + c];
      delta[i * l + c] = v / Lj[i * len + i];
    }
  }
}

/* ---- residual update (eq. text_update_of_r) ----------------------------- */

/* R <- R - K^_{:,I} delta, over all n rows (the rows of I included). */
void apo_apply_update(const apo_config* c, const double* X, double* R, int64_t blk,
                      const double* delta) {
  int64_t s = apo_block_start(c, blk), len = apo_block_len(c, blk);
  int32_t l = c->l;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < c->n; ++i) {
    for (int64_t q = 0; q < len; ++q) {
      double k = apo_khat(c, X, i, s + q);
      for (int32_t col = 0; col < l; ++col) R[i * l + col] -= k * delta[q * l + col];
    }
  }
}

/* One AP update on block blk (inner loop of Algorithm 1), given that block's
 * factor Lj:
 *   W_I += K^_{I,I}^{-1} R_I          (eq. text_update_of_w)
 *   R   -= K^_{:,I} K^_{I,I}^{-1} R_I  (eq. text_update_of_r)
 * If delta_out is not NULL, the step K^_{I,I}^{-1} R_I (len x l) is copied there. */
void apo_update_block(const apo_config* c, const double* X, const double* Lj, double* W,
                      double* R, int64_t blk, double* delta_out) {
  int64_t s = apo_block_start(c, blk), len = apo_block_len(c, blk);
  int32_t l = c->l;
  double* delta = (double*)malloc(sizeof(double) * (size_t)(len * l));
  apo_block_solve(Lj, len, l, R + s * l, delta);
  for (int64_t q = 0; q < len; ++q)
    for (int32_t col = 0; col < l; ++col) W[(s + q) * l + col] += delta[q * l + col];
  apo_apply_update(c, X, R, blk, delta);
  if (delta_out) memcpy(delta_out, delta, sizeof(double) * (size_t)(len * l));
  free(delta);
}

/* The same with block blk's factor taken from the array of all factors. */
void apo_update(const apo_config* c, const double* X, const double* L, double* W, double* R,
                int64_t blk, double* delta_out) {
  apo_update_block(c, X, L + blk * (int64_t)c->b * c->b, W, R, blk, delta_out);
}

/* ---- block selection (Section 3 "Block Selection") ---------------------- */

/* ||R_{I,:}||_F^2 for every block I in P. */
void apo_block_norms(const apo_config* c, const double* R, double* out) {
  int64_t m = apo_num_blocks(c);
  for (int64_t j = 0; j < m; ++j) {
    int64_t s = apo_block_start(c, j), len = apo_block_len(c, j);
    double acc = 0.0;
    for (int64_t i = s; i < s + len; ++i)
      for (int32_t col = 0; col < c->l; ++col) acc += R[i * c->l + col] * R[i * c->l + col];
    out[j] = acc;
  }
}

/* Modified Gauss-Southwell rule (eq. approximate_gauss_southwell):
 * argmax_I ||R_{I,:}||_F^2, ties to the lowest block index. */
int64_t apo_select_greedy(const apo_config* c, const double* R) {
  int64_t m = apo_num_blocks(c);
  double* nrm = (double*)malloc(sizeof(double) * (size_t)m);
  apo_block_norms(c, R, nrm);
  int64_t best = 0;
  for (int64_t j = 1; j < m; ++j)
    if (nrm[j] > nrm[best]) best = j;
  free(nrm);
  return best;
}

/* Random rule (I drawn uniformly from the partition). The draws come from
 * SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): the generator adds the
 * constant 0x9e3779b97f4a7c15 to its state at every call and returns the
 * state through the mixing function below, so output k (from 0) of a
 * generator seeded with `seed` is mix(seed + (k + 1) * 0x9e37...). */
uint64_t apo_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t state = seed + (k + 1) * 0x9e3779b97f4a7c15ULL;
  state ^= state >> 30;
  state *= 0xbf58476d1ce4e5b9ULL;
  state ^= state >> 27;
  state *= 0x94d049bb133111ebULL;
  state ^= state >> 31;
  return state;
}

/* Block of update u (counted from the start of the solve, over epochs):
 * floor(h * m / 2^32) with h the high 32 bits of draw u, i.e. h / 2^32 is a
 * uniform fraction and the block is its share of the m blocks. */
int64_t apo_select_random(const apo_config* c, uint64_t u) {
  uint64_t h = apo_splitmix64(c->seed, u) >> 32;
  return (int64_t)((h * (uint64_t)apo_num_blocks(c)) >> 32);
}

/* ---- stopping rule (Algorithm 1 test; "Alternating Projection Details") -- */

/* Mean over columns of ||r_c||_2 / ||b_c||_2; a zero column of B counts 0. */
double apo_rel_residual(const apo_config* c, const double* R, const double* B) {
  double acc = 0.0;
  for (int32_t col = 0; col < c->l; ++col) {
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
      rr += R[i * c->l + col] * R[i * c->l + col];
      bb += B[i * c->l + col] * B[i * c->l + col];
    }
    if (bb > 0.0) acc += sqrt(rr) / sqrt(bb);
  }
  return acc / c->l;
}

/* One epoch: m updates, cyclic (block u at step u), greedy, or random (draw
 * epoch * m + u at step u; `epoch` counts the epochs before this one). If
 * sel_out is not NULL it receives the m selected block indices. */
void apo_epoch(const apo_config* c, const double* X, const double* L, double* W, double* R,
               int64_t epoch, int64_t* sel_out) {
  int64_t m = apo_num_blocks(c);
  for (int64_t u = 0; u < m; ++u) {
    int64_t blk = u;
    if (c->order == APO_GREEDY)
      blk = apo_select_greedy(c, R);
    else if (c->order == APO_RANDOM)
      blk = apo_select_random(c, (uint64_t)(epoch * m + u));
    if (sel_out) sel_out[u] = blk;
    apo_update(c, X, L, W, R, blk, NULL);
  }
}

/* Algorithm 1. W and R are n x l outputs (W starts at 0, R at B). rho_trace
 * (max_epochs entries, may be NULL) receives the stopping metric after every
 * epoch. Returns 0 if the tolerance was met, 1 if max_epochs ran out first,
 * -2 if a block factor failed (bad block in *epochs_out). */
int32_t apo_solve(const apo_config* c, const double* X, const double* B, double* W, double* R,
                  double* rho_trace, int32_t* epochs_out) {
  int64_t m = apo_num_blocks(c);
  double* L = (double*)malloc(sizeof(double) * (size_t)(m * (int64_t)c->b * c->b));
  int64_t piv = -1;
  int64_t bad = apo_factor(c, X, L, &piv);
  if (bad >= 0) {
    free(L);
    if (epochs_out) *epochs_out = (int32_t)bad;
    return -2;
  }
  int64_t nl = c->n * c->l;
  for (int64_t i = 0; i < nl; ++i) {
    W[i] = 0.0;
    R[i] = B[i];
  }
  int32_t status = 1, t = 0;
  while (t < c->max_epochs) {
    apo_epoch(c, X, L, W, R, t, NULL);
    ++t;
    double rho = apo_rel_residual(c, R, B);
    if (rho_trace) rho_trace[t - 1] = rho;
    if (rho < c->tol && t >= c->min_epochs) {
      status = 0;
      break;
    }
  }
  if (epochs_out) *epochs_out = t;
  free(L);
  return status;
}

/* ---- block coordinate descent (Algorithm 2), for the equivalence check --- */

/* W_I <- K^_{I,I}^{-1} (B_I - K^_{I,not I} W_{not I}), computed from B and W
 * without any maintained residual. */
void apo_bcd_update(const apo_config* c, const double* X, const double* L, const double* B,
                    double* W, int64_t blk) {
  int64_t s = apo_block_start(c, blk), len = apo_block_len(c, blk);
  int32_t l = c->l;
  double* rhs = (double*)malloc(sizeof(double) * (size_t)(len * l));
  double* sol = (double*)malloc(sizeof(double) * (size_t)(len * l));
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < len; ++q) {
    int64_t i = s + q;
    for (int32_t col = 0; col < l; ++col) rhs[q * l + col] = B[i * l + col];
    for (int64_t j = 0; j < c->n; ++j) {
      if (j >= s && j < s + len) continue;
      double k = apo_khat(c, X, i, j);
      for (int32_t col = 0; col < l; ++col) rhs[q * l + col] -= k * W[j * l + col];
    }
  }
  apo_block_solve(L + blk * (int64_t)c->b * c->b, len, l, rhs, sol);
  for (int64_t q = 0; q < len; ++q)
    for (int32_t col = 0; col < l; ++col) W[(s + q) * l + col] = sol[q * l + col];
  free(rhs);
  free(sol);
}

/* ---- true residual (Lemma residual_equality) ---------------------------- */

/* out[r, :] = B[row_r, :] - K^_{row_r, :} W for the listed rows (all n columns). */
void apo_residual_rows(const apo_config* c, const double* X, const double* B, const double* W,
                       const int64_t* rows, int64_t nrows, double* out) {
  int32_t l = c->l;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    double* o = out + r * l;
    for (int32_t col = 0; col < l; ++col) o[col] = B[i * l + col];
    for (int64_t j = 0; j < c->n; ++j) {
      double k = apo_khat(c, X, i, j);
      for (int32_t col = 0; col < l; ++col) o[col] -= k * W[j * l + col];
    }
  }
}

/* ---- posterior mean (Section 2, GP regression) ---------------------------- */

/* out[r, :] = sum_j k(xs_r, x_j) W[j, :] for the ns test points xs (ns x d):
 * with W = K^^{-1} B this is the posterior mean K(X*, X) K^^{-1} B. The noise
 * term belongs to the training points only, so it does not appear here. */
void apo_predict(const apo_config* c, const double* X, const double* W, const double* Xs,
                 int64_t ns, double* out) {
  int32_t l = c->l, d = c->d;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < ns; ++r) {
    double* o = out + r * l;
    for (int32_t col = 0; col < l; ++col) o[col] = 0.0;
    for (int64_t j = 0; j < c->n; ++j) {
      double k = apo_kernel(c, Xs + r * d, X + j * d);
      for (int32_t col = 0; col < l; ++col) o[col] += k * W[j * l + col];
    }
  }
}

#define APO_MAX_D 64

/* ---- stochastic MLL gradient (Section 2, eq. loss_grad_unbiased) ---------- */

/* Derivative factor of the kernel in r: dk/dell_m = g(r) * (x_m - x'_m)^2 / ell_m^3
 * with g = k for RBF, 3 s exp(-sqrt3 r) for Matern-3/2 and
 * (5/3) s (1 + sqrt5 r) exp(-sqrt5 r) for Matern-5/2 (chain rule through
 * r^2 = sum_m ((x_m - x'_m) / ell_m)^2). */
static double apo_dk_factor(const apo_config* c, double r2) {
  double s = c->outputscale;
  switch (c->kernel) {
    case APO_RBF:
      return s * exp(-0.5 * r2);
    case APO_MATERN32:
      return 3.0 * s * exp(-sqrt(3.0) * sqrt(r2));
    case APO_MATERN52: {
      double r = sqrt(r2);
      return (5.0 / 3.0) * s * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r);
    }
    default:
      return NAN;
  }
}

/* The estimate of d ell / d theta for theta = (ell_1..ell_d, s, sigma^2), the
 * negative log marginal likelihood ell = (y^T K^^{-1} y + log det K^) / 2,
 * from W = K^^{-1} B with B = [y, z_1, ..., z_P] (P = l - 1 probes with zero
 * mean and identity covariance):
 *   grad_theta = -1/2 w_0^T (dK^/dtheta) w_0 + 1/(2P) sum_p w_p^T (dK^/dtheta) z_p
 *             = sum_{i,j} C_ij (dK^/dtheta)_ij,
 *   C_ij = -1/2 W_i0 W_j0 + 1/(2P) sum_p W_ip B_jp,
 * with dK^/dell_m as above, dK^/ds = K / s, dK^/dsigma^2 = I. Sums over rows
 * i in [i0, i1) and all columns j; out has d + 2 entries. */
void apo_mll_grad_rows(const apo_config* c, const double* X, const double* B, const double* W,
                       int64_t i0, int64_t i1, double* out) {
  int32_t d = c->d, l = c->l, P = l - 1;
  if (d > APO_MAX_D) {
    for (int32_t m = 0; m < d + 2; ++m) out[m] = NAN;
    return;
  }
  double acc[APO_MAX_D + 2];
  for (int32_t m = 0; m < d + 2; ++m) acc[m] = 0.0;
#pragma omp parallel
  {
    double loc[APO_MAX_D + 2];
    for (int32_t m = 0; m < d + 2; ++m) loc[m] = 0.0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = i0; i < i1; ++i) {
      const double* xi = X + i * d;
      for (int64_t j = 0; j < c->n; ++j) {
        const double* xj = X + j * d;
        double cij = -0.5 * W[i * l] * W[j * l];
        for (int32_t p = 1; p <= P; ++p) cij += W[i * l + p] * B[j * l + p] / (2.0 * P);
        double r2 = apo_r2(c, xi, xj);
        double g = apo_dk_factor(c, r2);
        for (int32_t m = 0; m < d; ++m) {
          double dm = xi[m] - xj[m];
          double ell = c->lengthscale[m];
          loc[m] += cij * g * dm * dm / (ell * ell * ell);
        }
        loc[d] += cij * apo_kernel(c, xi, xj) / c->outputscale;
        if (i == j) loc[d + 1] += cij;
      }
    }
#pragma omp critical
    for (int32_t m = 0; m < d + 2; ++m) acc[m] += loc[m];
  }
  for (int32_t m = 0; m < d + 2; ++m) out[m] = acc[m];
}

void apo_mll_grad(const apo_config* c, const double* X, const double* B, const double* W,
                  double* out) {
  apo_mll_grad_rows(c, X, B, W, 0, c->n, out);
}

/* B - K^ W over all rows. */
void apo_residual(const apo_config* c, const double* X, const double* B, const double* W,
                  double* out) {
  int32_t l = c->l;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < c->n; ++i) {
    double* o = out + i * l;
    for (int32_t col = 0; col < l; ++col) o[col] = B[i * l + col];
    for (int64_t j = 0; j < c->n; ++j) {
      double k = apo_khat(c, X, i, j);
      for (int32_t col = 0; col < l; ++col) o[col] -= k * W[j * l + col];
    }
  }
}
