/*
 * FP64 CPU oracle for alternating projection -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
 * this header and its library. All pointers are host pointers; matrices are
 * row-major FP64: X is n x d, B / W / R are n x l, a block factor is len x len.
 * Nothing here allocates memory that the caller must free.
 */
#ifndef AP_ORACLE_H
#define AP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { APO_RBF = 0, APO_MATERN32 = 1, APO_MATERN52 = 2 };
enum { APO_CYCLIC = 0, APO_GREEDY = 1, APO_RANDOM = 2 };

typedef struct {
  int64_t n;                  /* number of points */
  int32_t d, l, b;            /* features, right-hand sides, block size */
  int32_t kernel;             /* APO_RBF, APO_MATERN32, APO_MATERN52 */
  const double* lengthscale;  /* d ARD lengthscales */
  double outputscale, noise;  /* s and sigma^2 */
  int32_t order;              /* APO_CYCLIC, APO_GREEDY or APO_RANDOM */
  double tol;                 /* stop when the mean column ratio is < tol */
  int32_t min_epochs, max_epochs;
  uint64_t seed;              /* APO_RANDOM: seed of the block draws */
} apo_config;

int32_t apo_num_threads(void);
double apo_kernel(const apo_config* c, const double* x, const double* y);
void apo_khat_block(const apo_config* c, const double* X, int64_t i0, int64_t i1, int64_t j0,
                    int64_t j1, double* out);
int64_t apo_num_blocks(const apo_config* c);
int64_t apo_block_start(const apo_config* c, int64_t j);
int64_t apo_block_len(const apo_config* c, int64_t j);
int64_t apo_cholesky(double* A, int64_t len);
int64_t apo_factor_one(const apo_config* c, const double* X, int64_t j, double* Lj);
int64_t apo_factor(const apo_config* c, const double* X, double* L, int64_t* bad_pivot);
void apo_block_solve(const double* Lj, int64_t len, int32_t l, const double* RI, double* delta);
void apo_apply_update(const apo_config* c, const double* X, double* R, int64_t blk,
                      const double* delta);
void apo_update_block(const apo_config* c, const double* X, const double* Lj, double* W,
                      double* R, int64_t blk, double* delta_out);
void apo_update(const apo_config* c, const double* X, const double* L, double* W, double* R,
                int64_t blk, double* delta_out);
void apo_block_norms(const apo_config* c, const double* R, double* out);
int64_t apo_select_greedy(const apo_config* c, const double* R);
uint64_t apo_splitmix64(uint64_t seed, uint64_t k);
int64_t apo_select_random(const apo_config* c, uint64_t u);
double apo_rel_residual(const apo_config* c, const double* R, const double* B);
void apo_epoch(const apo_config* c, const double* X, const double* L, double* W, double* R,
               int64_t epoch, int64_t* sel_out);
int32_t apo_solve(const apo_config* c, const double* X, const double* B, double* W, double* R,
                  double* rho_trace, int32_t* epochs_out);
void apo_bcd_update(const apo_config* c, const double* X, const double* L, const double* B,
                    double* W, int64_t blk);
void apo_residual_rows(const apo_config* c, const double* X, const double* B, const double* W,
                       const int64_t* rows, int64_t nrows, double* out);
void apo_predict(const apo_config* c, const double* X, const double* W, const double* Xs,
                 int64_t ns, double* out);
void apo_mll_grad_rows(const apo_config* c, const double* X, const double* B, const double* W,
                       int64_t i0, int64_t i1, double* out);
void apo_mll_grad(const apo_config* c, const double* X, const double* B, const double* W,
                  double* out);
void apo_residual(const apo_config* c, const double* X, const double* B, const double* W,
                  double* out);

#ifdef __cplusplus
}
#endif
#endif
