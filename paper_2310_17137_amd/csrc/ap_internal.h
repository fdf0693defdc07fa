// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ap {

// Rows of the residual handled by one workgroup of the fused update: 4 waves,
// each owning two 32-row MFMA tiles.
constexpr int kRowsWG = 256;
// Block columns consumed per step of the fused update's inner loop.
constexpr int kChunk = 32;
// Right-hand sides handled by one pass (the M dimension of the 32x32 MFMA).
constexpr int kMaxL = 32;
// FP64 tile edge of the batched factorization.
constexpr int kT = 64;
// K-split of the FP64 block solve.
constexpr int kBsSplit = 16;
constexpr int kMaxD = 20;

// Device control block at the start of the workspace.
struct Ctl {
  unsigned long long fail;  // first non-positive pivot: (block << 32) | pivot, ~0 if none
  int32_t status;           // 0 ok, else an ap_status (non-finite residual)
  int32_t sel;              // selected block of the next update (greedy, random order)
  int32_t epoch;            // epochs completed since the last reset
  int32_t pad0;
  double rho;               // mean column ratio after the last epoch
  double rho_true;          // the same for the last FP64 true residual
  double bnorm2[kMaxL];     // ||B_c||^2
  double colrel[kMaxL];     // ||R_c|| / ||B_c|| after the last epoch
  double colrel_true[kMaxL];
  double mu[kMaxD];         // feature centre used by the prepared copies
  // batch steps (ap_batch_step): this problem's progress, kept on the device
  int32_t cursor;           // updates done in the current epoch
  int32_t state;            // 0 runs; else why the problem is held (ap_batch_state)
  int32_t run;              // latched at the end of every batch step from state
  int32_t next_refine;      // > 0: epoch of the next true-residual hold; 0: every refine_every
  double mll_grad[kMaxD + 2];  // last ap_mll_grad: lengthscales, outputscale, noise
  unsigned long long draws; // random order: block draws made since the last reset
};

// Block argument of the solve and update launches: >= 0 names the block;
// kBlockSel takes the selection in ctl->sel (greedy or random order); the
// batch codes take the problem's own cursor (cyclic) or ctl->sel and make the
// launch a no-op while the problem is held.
constexpr int kBlockSel = -1;
constexpr int kBlockBatchCyclic = -2;
constexpr int kBlockBatchSel = -3;

// Random order (Section 3, "Block Selection": I drawn uniformly from the
// partition): draw u since the reset takes block floor(h m / 2^32), with h the
// high 32 bits of output u of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
// started from the seed: z = seed + (u + 1) * 0x9e3779b97f4a7c15, then
// z ^= z >> 30, z *= 0xbf58476d1ce4e5b9, z ^= z >> 27, z *= 0x94d049bb133111eb,
// z ^= z >> 31.
__host__ __device__ inline int32_t random_block(unsigned long long seed, unsigned long long u,
                                                int32_t m) {
  unsigned long long z = seed + (u + 1ull) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (int32_t)(((z >> 32) * (unsigned long long)m) >> 32);
}

// Block of this launch, or -1 when a batch step skips a held problem (uniform
// over the workgroup). An index read from the control block outside [0, m)
// (which the selection kernels never write) also gives -1, so a launch never
// addresses a block that does not exist.
__device__ __forceinline__ int resolve_block(int block, const struct Ctl* ctl, int m) {
  int b = block;
  if (block < 0) {
    if (block != kBlockSel && !ctl->run) return -1;
    b = block == kBlockBatchCyclic ? ctl->cursor : ctl->sel;
  }
  return b >= 0 && b < m ? b : -1;
}

// Kernel map constants. The prepared features v = (x - mu) / ell * c_feat make
// the map a function of |v_i - v_j|^2 only:
//  RBF:        k/s = exp2(-|dv|^2)                      (c_feat = sqrt(log2(e) / 2))
//  Matern-3/2: t = |dv| ; k/s = (1 + t / log2 e) exp2(-t)         (c_feat = sqrt3 log2 e)
//  Matern-5/2: t = |dv| ; k/s = (1 + t / log2 e + t^2 / (3 log2^2 e)) exp2(-t)
//                                                                   (c_feat = sqrt5 log2 e)
constexpr double kLog2e = 1.4426950408889634;

struct Layout {
  int64_t n, n_pad;      // n_pad >= n + 32, multiple of kRowsWG
  int32_t d, l, b, m, b_pad, last_len;
  int32_t kernel, order, tile;
  unsigned long long seed;  // random order: seed of the block draws
  int32_t ks;            // BF16 K-steps of 16 feature slots (3d + 6 slots)
  int32_t dp;            // prepared-feature stride (d rounded up to 4)
  int32_t nwg;           // workgroups of the fused update: n_pad / kRowsWG
  int32_t nwg_res;       // workgroups of the true residual
  size_t off_ctl, off_xs, off_xn, off_xu, off_xun, off_xrow, off_xcol, off_kinv, off_dinv,
      off_panel, off_delta,
      off_bspart, off_dtile, off_rowsq, off_colsq, off_blocknorm, off_respart, off_mupart,
      off_desc, off_gpart;
  int32_t nwg_mll;       // workgroups of the MLL gradient: 64 rows each
  size_t total;
};

struct Dev {  // device pointers into one problem's workspace
  Ctl* ctl;
  double* xv;            // FP32 and split paths: n_pad x dp prepared features
  double* xn;            // FP32 and split paths: n_pad norms |v|^2 of the prepared features
  double* xu;            // FP64 tiles: n_pad x dp centred features u = (x - mu) / ell
  double* xun;           // FP64 tiles: n_pad norms |u|^2
  uint16_t* xrow;        // BF16 path: n_pad x 16 ks (row-role operand)
  uint16_t* xcol;        // BF16 path: n_pad x 16 ks (column-role operand)
  double* kinv;          // m x b_pad x b_pad
  double* dinv;          // factor scratch: m x (b_pad/64) x 64 x 64
  double* panel;         // factor scratch: m x (b_pad/64) x 64 x 64
  double* delta;         // b_pad x 32 FP64 block step
  double* bspart;        // kBsSplit x b_pad x 32 partial products
  void* dtile;           // block step as the fused update's MFMA operand
  float* rowsq;          // n_pad per-row sums of squares of R (greedy order)
  float* colsq;          // nwg x 32 per-workgroup column sums of squares
  double* blocknorm;     // m block norms ||R_I||_F^2
  double* respart;       // nwg_res x 32 FP64 column partials of the true residual
  double* mupart;        // feature-centre partial sums
  double* gpart;         // nwg_mll x (kMaxD + 2) partial sums of the MLL gradient
};

struct Params {  // hyperparameters as the kernels need them
  double ell[kMaxD];
  double s, noise;
};

// Everything a grouped (batch) launch needs to know about one problem, kept in
// its workspace and written once when its factors are built.
struct Desc {
  Layout L;
  Dev D;
  Params P;
  const float* X;
  double tol;
  int32_t min_epochs, max_epochs, refine_every, pad;
};

// Problems of one grouped launch: workgroups [wg0[p], wg0[p+1]) serve problem p.
constexpr int kMaxBatch = 32;
struct Group {
  int32_t count;
  int32_t wg0[kMaxBatch + 1];
  const Desc* desc[kMaxBatch];
  float* R[kMaxBatch];
  double* W[kMaxBatch];
  int32_t tile[kMaxBatch];
};

// Problem of this workgroup in a grouped launch and its workgroup index there.
__device__ __forceinline__ int group_job(const Group& g, int* local) {
  int p = 0;
  while (p + 1 < g.count && (int)blockIdx.x >= g.wg0[p + 1]) ++p;
  *local = (int)blockIdx.x - g.wg0[p];
  return p;
}

// Record a failure for ap_last_error (this thread): a HIP call and its error,
// or a plain message. note_error returns AP_ERR_HIP (-5).
int note_error(const char* where, hipError_t e);
void note_text(const char* msg);
// Take off (and keep for ap_last_error) an error an earlier HIP call outside
// the library left unread, before launching.
void take_foreign_error();

bool make_layout(int64_t n, int32_t d, int32_t l, int32_t b, int32_t kernel, int32_t order,
                 int32_t tile, Layout* L);
Dev bind(const Layout& L, void* ws);

// ---- launchers (each enqueues on `st` and returns the launch status) -------
hipError_t launch_prep(const Layout& L, const Dev& D, const Params& P, const float* X,
                       hipStream_t st);
hipError_t launch_factor(const Layout& L, const Dev& D, const Params& P, const float* X,
                         hipStream_t st);
// Workgroups of the reset's column-norm partials (D.respart holds as many rows).
constexpr int kResetGroups = 1024;
// R = B, the column norms of B, a fresh control block; W = 0 unless keep_w
hipError_t launch_reset(const Layout& L, const Dev& D, const float* B, double* W, float* R,
                        bool keep_w, hipStream_t st);
// only the column norms of B and a fresh control block (D.ctl, D.respart)
hipError_t launch_bnorm(const Layout& L, const Dev& D, const float* B, hipStream_t st);
// workgroups of the true residual over n rows (its column partials in D.respart)
int residual_groups(int64_t n);
// block: >= 0, kBlockSel or a batch code (see resolve_block)
hipError_t launch_block_solve(const Layout& L, const Dev& D, const Params& P, int32_t block,
                              const float* R, double* W, hipStream_t st);
hipError_t launch_fused_update(const Layout& L, const Dev& D, int32_t block, float* R,
                               bool want_rowsq, bool want_colsq, hipStream_t st);
hipError_t launch_fused_update64(const Layout& L, const Dev& D, const Params& P, const float* X,
                                 int32_t block, float* R, bool want_rowsq, bool want_colsq,
                                 hipStream_t st);
hipError_t launch_select(const Layout& L, const Dev& D, hipStream_t st);
hipError_t launch_epoch_check(const Layout& L, const Dev& D, hipStream_t st);
hipError_t launch_residual(const Layout& L, const Dev& D, const Params& P, const float* X,
                           const float* B, const double* W, float* Rout, bool in_place,
                           hipStream_t st);
hipError_t launch_copy_inverse(const Layout& L, const Dev& D, int32_t j, double* dst,
                               hipStream_t st);
// stochastic MLL gradient from W = K^^{-1} [y, probes]: per-64-row partials
// into D.gpart, their fixed-order sum into ctl->mll_grad
hipError_t launch_mll_grad(const Layout& L, const Dev& D, const Params& P, const float* X,
                           const float* B, const double* W, hipStream_t st);
// mean (ns x l, FP64) = K(Xs, X) W for ns test points Xs (ns x d, FP32)
hipError_t launch_predict(const Layout& L, const Params& P, const float* X, const double* W,
                          const float* Xs, int64_t ns, double* mean, hipStream_t st);

// ---- grouped launches of a batch step (one launch for many problems) -------
hipError_t launch_group_solve(const Group& gp, const Group& gf, hipStream_t st);
// wide: the group's feature strides are 12 to 20 (else 4 or 8)
hipError_t launch_group_split(const Group& g, bool wide, hipStream_t st);
hipError_t launch_group_select(const Group& gn, const Group& ga, hipStream_t st);
// random order: draw the next block into ctl->sel (grouped: for the problems
// whose update ran in this batch step)
hipError_t launch_random_select(const Layout& L, const Dev& D, hipStream_t st);
hipError_t launch_group_random(const Group& g, hipStream_t st);
hipError_t launch_group_advance(const Group& g, hipStream_t st);
hipError_t launch_release(const Dev& D, int32_t next_refine, hipStream_t st);

}  // namespace ap
