// Batched FP64 block factorization: for every block I of the partition, form
// K^_{I,I} = s k(X_I, X_I) + sigma^2 I, factor it by Cholesky, invert the factor
// and form K^_{I,I}^{-1} = L^{-T} L^{-1} (Section 3, "Cached Cholesky Factors":
// all blocks share one batched call; the cost is O(n b^2) once per
// hyperparameter setting).
//
// Each block lives in a b_pad x b_pad row-major slot (b_pad = b rounded up to
// 64). Rows and columns past the block's length hold the identity, so every
// slot is factored the same way and its inverse is [[A^{-1}, 0], [0, I]].
// The work is split in 64 x 64 FP64 tiles staged through LDS, their products on
// the FP64 matrix cores; each launch covers one tile step for all m blocks at
// once:
//   Cholesky  (left-looking):  update of the tile column by the earlier panels,
//             diag factor + diag inverse, panel solve
//   L^{-1}    (column blocks from the right, through a panel buffer)
//   L^{-T}L^{-1} (block rows from the top, in place), then mirror to the upper half.
#include <algorithm>

#include "ap_internal.h"

namespace ap {
namespace {

constexpr int LDT = kT + 1;  // padded LDS row stride (doubles)

__device__ inline double kernel_fp64(int kern, const float* __restrict__ xi,
                                     const float* __restrict__ xj, int d, const Params& P) {
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = ((double)xi[k] - (double)xj[k]) / P.ell[k];
    r2 = fma(t, t, r2);
  }
  if (kern == 0) return P.s * exp(-0.5 * r2);
  if (kern == 1) {
    double t = 1.7320508075688772 * sqrt(r2);
    return P.s * (1.0 + t) * exp(-t);
  }
  double r = sqrt(r2), t = 2.23606797749979 * r;
  return P.s * (1.0 + t + (5.0 / 3.0) * r2) * exp(-t);
}

// A 64 x 64 tile moves global -> registers -> LDS: each of the 256 threads
// loads 16 elements, all issued before the first is stored.
constexpr int kPerThread = kT * kT / 256;

__device__ inline void fetch_tile(double v[kPerThread], const double* __restrict__ g, int ld) {
#pragma unroll
  for (int u = 0; u < kPerThread; ++u) {
    const int e = threadIdx.x + 256 * u;
    v[u] = g[(size_t)(e / kT) * ld + e % kT];
  }
}

__device__ inline void put_tile(double* s, const double v[kPerThread], bool trans, int lds) {
#pragma unroll
  for (int u = 0; u < kPerThread; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int r = e / kT, c = e % kT;
    if (trans) s[c * lds + r] = v[u]; else s[r * lds + c] = v[u];
  }
}

__device__ inline void load_tile(double* s, const double* __restrict__ g, int ld, bool trans,
                                 int lds) {
  double v[kPerThread];
  fetch_tile(v, g, ld);
  put_tile(s, v, trans, lds);
}

// 64 x 64 x 64 tile products on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
// Wave w computes rows 16 w .. 16 w + 15 of the product as four 16 x 16
// accumulators; lane holds C[16 w + lane / 16 + 4 q][16 ct + lane % 16] in
// acc[ct][q]. A tiles (the left operand) are staged with row stride LDA, B
// tiles with LDB: 4 and 16 mod 32 doubles, so that the 64 lanes' operand reads
// spread over the LDS banks.
constexpr int LDA = kT + 4;
constexpr int LDB = kT + 16;
typedef __attribute__((ext_vector_type(4))) double f64x4;

__device__ inline void mma_tile(const double* sA, const double* sB, f64x4 acc[4]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const double* a_row = sA + (16 * w + ln) * LDA + lg;  // A[m = lane % 16][k = lane / 16]
#pragma unroll 4
  for (int s = 0; s < kT / 4; ++s) {
    const double a = a_row[4 * s];
    const double* b_row = sB + (4 * s + lg) * LDB + ln;  // B[k = lane / 16][n = lane % 16]
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b_row[16 * ct], acc[ct], 0, 0, 0);
  }
}

__device__ inline void zero_acc(f64x4 acc[4]) {
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// element (row, col) of the 64 x 64 product this lane holds as acc[ct][q]
#define AP_ACC_FOR(BODY)                                   \
  do {                                                     \
    const int lane_ = threadIdx.x % 64, w_ = threadIdx.x / 64; \
    _Pragma("unroll") for (int ct = 0; ct < 4; ++ct)       \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {      \
        const int row = 16 * w_ + lane_ / 16 + 4 * q;      \
        const int col = 16 * ct + lane_ % 16;              \
        BODY;                                              \
      }                                                    \
  } while (0)

__device__ inline void store_acc(double* __restrict__ g, int ld, const f64x4 acc[4],
                                 double scale) {
  AP_ACC_FOR(g[(size_t)row * ld + col] = scale * acc[ct][q]);
}

// XCD-aware workgroup order: the dispatcher deals consecutive workgroups to
// the 8 XCDs in turn, so the workgroups of one block (which stream the same
// panel tiles) would be spread over all 8 L2 caches. Renumbered, XCD x runs a
// contiguous range of logical indices (a bijection of 0 .. gridDim.x - 1).
__device__ inline int64_t xcd_order() {
  const int64_t nwg = gridDim.x, b = blockIdx.x;
  const int64_t per = nwg / 8, rem = nwg % 8;
  const int64_t x = b % 8, r = b / 8;
  return x * per + (x < rem ? x : rem) + r;
}

__device__ inline double* slot(const Layout& L, double* base, int64_t j) {
  return base + (size_t)j * L.b_pad * L.b_pad;
}
__device__ inline double* tile(const Layout& L, double* A, int I, int J) {
  return A + (size_t)I * kT * L.b_pad + (size_t)J * kT;
}
// factor scratch: per block, nt tiles of 64 x 64 (tile index i)
__device__ inline double* scratch_tile(const Layout& L, double* base, int64_t j, int i) {
  return base + ((size_t)j * (L.b_pad / kT) + i) * kT * kT;
}

// ---- form -----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_form(Layout L, Params P, const float* __restrict__ X,
                                              double* __restrict__ A) {
  const int nt = L.b_pad / kT;
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  const int64_t j = blockIdx.x / tiles;
  int64_t t = blockIdx.x % tiles;
  int I = 0;
  while (t > I) { t -= I + 1; ++I; }  // lower-triangle tile index -> (I, J)
  const int J = (int)t;
  const int64_t start = j * L.b;
  const int len = (int)min<int64_t>(L.b, L.n - start);
  double* S = tile(L, slot(L, A, j), I, J);
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    int r = e / kT, c = e % kT;
    int p = I * kT + r, q = J * kT + c;
    double v;
    if (p < len && q < len) {
      v = kernel_fp64(L.kernel, X + (start + p) * L.d, X + (start + q) * L.d, L.d, P);
      if (p == q) v += P.noise;
    } else {
      v = (p == q) ? 1.0 : 0.0;
    }
    S[(size_t)r * L.b_pad + c] = v;
  }
}

// ---- Cholesky ---------------------------------------------------------------

// Factor the diagonal tile k of every block in LDS, write L_kk (upper part
// zero) and its inverse into the scratch tile dinv[j][k].
__global__ __launch_bounds__(256) void k_potrf_diag(Layout L, double* __restrict__ A,
                                                    double* __restrict__ dinv, Ctl* ctl, int k) {
  __shared__ double s[kT * LDT];
  __shared__ double x[kT * LDT];
  const int64_t j = blockIdx.x;
  double* G = tile(L, slot(L, A, j), k, k);
  load_tile(s, G, L.b_pad, false, LDT);
  __syncthreads();
  const int t = threadIdx.x;
  for (int kk = 0; kk < kT; ++kk) {
    if (t == 0) {
      double p = s[kk * LDT + kk];
      if (!(p > 0.0)) {
        unsigned long long code = ((unsigned long long)j << 32) | (unsigned)(k * kT + kk);
        atomicMin(&ctl->fail, code);
        p = 1.0;  // keep the arithmetic finite; the call reports the failure
      }
      s[kk * LDT + kk] = sqrt(p);
    }
    __syncthreads();
    if (t > kk && t < kT) s[t * LDT + kk] /= s[kk * LDT + kk];
    __syncthreads();
    for (int e = t; e < kT * kT; e += blockDim.x) {
      int r = e / kT, c = e % kT;
      if (r > kk && c > kk && c <= r) s[r * LDT + c] -= s[r * LDT + kk] * s[c * LDT + kk];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular tile, one column per thread
  if (t < kT) {
    const int c = t;
    for (int r = 0; r < c; ++r) x[r * LDT + c] = 0.0;
    x[c * LDT + c] = 1.0 / s[c * LDT + c];
    for (int r = c + 1; r < kT; ++r) {
      double acc = 0.0;
      for (int q = c; q < r; ++q) acc = fma(s[r * LDT + q], x[q * LDT + c], acc);
      x[r * LDT + c] = -acc / s[r * LDT + r];
    }
  }
  __syncthreads();
  double* Dg = scratch_tile(L, dinv, j, k);
  for (int e = t; e < kT * kT; e += blockDim.x) {
    int r = e / kT, c = e % kT;
    G[(size_t)r * L.b_pad + c] = (c <= r) ? s[r * LDT + c] : 0.0;
    Dg[e] = x[r * LDT + c];
  }
}

// L_ik = A_ik L_kk^{-T} for the tiles i > k of column k.
__global__ __launch_bounds__(256) void k_trsm(Layout L, double* __restrict__ A,
                                              const double* __restrict__ dinv, int k) {
  __shared__ double sA[kT * LDA];
  __shared__ double sB[kT * LDB];
  const int nt = L.b_pad / kT;
  const int rows = nt - k - 1;
  const int64_t wg = xcd_order();
  const int64_t j = wg / rows;
  const int i = k + 1 + (int)(wg % rows);
  double* G = tile(L, slot(L, A, j), i, k);
  load_tile(sA, G, L.b_pad, false, LDA);
  load_tile(sB, scratch_tile(L, const_cast<double*>(dinv), j, k), kT, true, LDB);
  __syncthreads();
  f64x4 acc[4];
  zero_acc(acc);
  mma_tile(sA, sB, acc);
  store_acc(G, L.b_pad, acc, 1.0);
}

// Left-looking update of tile column k before its factorization:
// A_ik -= sum_{p<k} L_ip L_kp^T for the tiles i >= k, the sum accumulated in
// registers over the earlier panels (tiles prefetched one step ahead), so each
// target tile is read and written once.
__global__ __launch_bounds__(256) void k_herk(Layout L, double* __restrict__ A, int k) {
  __shared__ double sA[kT * LDA];
  __shared__ double sB[kT * LDB];
  const int nt = L.b_pad / kT;
  const int rows = nt - k;
  const int64_t wg = xcd_order();
  const int64_t j = wg / rows;
  const int i = k + (int)(wg % rows);
  double* Aj = slot(L, A, j);
  f64x4 acc[4];
  zero_acc(acc);
  double va[kPerThread], vb[kPerThread];
  fetch_tile(va, tile(L, Aj, i, 0), L.b_pad);
  fetch_tile(vb, tile(L, Aj, k, 0), L.b_pad);
  for (int p = 0; p < k; ++p) {
    put_tile(sA, va, false, LDA);
    put_tile(sB, vb, true, LDB);
    __syncthreads();
    if (p + 1 < k) {
      fetch_tile(va, tile(L, Aj, i, p + 1), L.b_pad);
      fetch_tile(vb, tile(L, Aj, k, p + 1), L.b_pad);
    }
    mma_tile(sA, sB, acc);
    __syncthreads();
  }
  double* G = tile(L, Aj, i, k);
  AP_ACC_FOR({
    const size_t o = (size_t)row * L.b_pad + col;
    G[o] = G[o] - acc[ct][q];
  });
}

// ---- L^{-1}: column block j, tiles i > j:  X_ij = -(sum_{k=j+1..i} X_ik L_kj) X_jj
// where columns > j already hold X. Results go to the panel scratch.
__global__ __launch_bounds__(256) void k_trtri_panel(Layout L, const double* __restrict__ A,
                                                     const double* __restrict__ dinv,
                                                     double* __restrict__ panel, int jc) {
  __shared__ double sA[kT * LDA];
  __shared__ double sB[kT * LDB];
  const int nt = L.b_pad / kT;
  const int rows = nt - jc - 1;
  const int64_t wg = xcd_order();
  const int64_t j = wg / rows;
  const int i = jc + 1 + (int)(wg % rows);
  const double* Aj = slot(L, const_cast<double*>(A), j);
  f64x4 acc[4];
  zero_acc(acc);
  // the next step's tiles are fetched into registers while this step's
  // products run
  double va[kPerThread], vb[kPerThread];
  fetch_tile(va, tile(L, const_cast<double*>(Aj), i, jc + 1), L.b_pad);
  fetch_tile(vb, tile(L, const_cast<double*>(Aj), jc + 1, jc), L.b_pad);
  for (int k = jc + 1; k <= i; ++k) {
    put_tile(sA, va, false, LDA);
    put_tile(sB, vb, false, LDB);
    __syncthreads();
    if (k < i) {
      fetch_tile(va, tile(L, const_cast<double*>(Aj), i, k + 1), L.b_pad);
      fetch_tile(vb, tile(L, const_cast<double*>(Aj), k + 1, jc), L.b_pad);
    }
    mma_tile(sA, sB, acc);
    __syncthreads();
  }
  // sA <- T, sB <- X_jj
  AP_ACC_FOR(sA[row * LDA + col] = acc[ct][q]);
  load_tile(sB, scratch_tile(L, const_cast<double*>(dinv), j, jc), kT, false, LDB);
  __syncthreads();
  f64x4 acc2[4];
  zero_acc(acc2);
  mma_tile(sA, sB, acc2);
  store_acc(scratch_tile(L, panel, j, i), kT, acc2, -1.0);
}

// Column block j of A <- [X_jj; panel tiles].
__global__ __launch_bounds__(256) void k_trtri_writeback(Layout L, double* __restrict__ A,
                                                         const double* __restrict__ dinv,
                                                         const double* __restrict__ panel,
                                                         int jc) {
  const int nt = L.b_pad / kT;
  const int rows = nt - jc;
  const int64_t j = blockIdx.x / rows;
  const int i = jc + (int)(blockIdx.x % rows);
  const double* src = (i == jc) ? scratch_tile(L, const_cast<double*>(dinv), j, jc)
                                : scratch_tile(L, const_cast<double*>(panel), j, i);
  double* G = tile(L, slot(L, A, j), i, jc);
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x)
    G[(size_t)(e / kT) * L.b_pad + e % kT] = src[e];
}

// ---- L^{-T} L^{-1} in place, block row i: tile (i, jc) = sum_{k>=i} X_ki^T X_kjc
__global__ __launch_bounds__(256) void k_lauum(Layout L, double* __restrict__ A, int i,
                                               int diag) {
  __shared__ double sA[kT * LDA];
  __shared__ double sB[kT * LDB];
  const int nt = L.b_pad / kT;
  const int cols = diag ? 1 : i;
  const int64_t wg = xcd_order();
  const int64_t j = wg / cols;
  const int jc = diag ? i : (int)(wg % cols);
  double* Aj = slot(L, A, j);
  f64x4 acc[4];
  zero_acc(acc);
  double va[kPerThread], vb[kPerThread];
  fetch_tile(va, tile(L, Aj, i, i), L.b_pad);
  fetch_tile(vb, tile(L, Aj, i, jc), L.b_pad);
  for (int k = i; k < nt; ++k) {
    put_tile(sA, va, true, LDA);
    put_tile(sB, vb, false, LDB);
    __syncthreads();
    if (k + 1 < nt) {
      fetch_tile(va, tile(L, Aj, k + 1, i), L.b_pad);
      fetch_tile(vb, tile(L, Aj, k + 1, jc), L.b_pad);
    }
    mma_tile(sA, sB, acc);
    __syncthreads();
  }
  store_acc(tile(L, Aj, i, jc), L.b_pad, acc, 1.0);
}

// Copy the lower triangle to the upper one.
__global__ __launch_bounds__(256) void k_mirror(Layout L, double* __restrict__ A) {
  const int nt = L.b_pad / kT;
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  const int64_t j = blockIdx.x / tiles;
  int64_t t = blockIdx.x % tiles;
  int I = 0;
  while (t > I) { t -= I + 1; ++I; }
  const int J = (int)t;  // J <= I: source tile (I, J), target (J, I)
  double* Aj = slot(L, A, j);
  const double* S = tile(L, Aj, I, J);
  double* T = tile(L, Aj, J, I);
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    int r = e / kT, c = e % kT;
    if (I == J && c <= r) continue;
    T[(size_t)c * L.b_pad + r] = S[(size_t)r * L.b_pad + c];
  }
}

__global__ void k_copy_block(Layout L, const double* __restrict__ A, int j, int len,
                             double* __restrict__ dst) {
  const double* S = A + (size_t)j * L.b_pad * L.b_pad;
  int64_t total = (int64_t)len * len;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e / len, c = e % len;
    dst[e] = S[r * L.b_pad + c];
  }
}

}  // namespace

hipError_t launch_factor(const Layout& L, const Dev& D, const Params& P, const float* X,
                         hipStream_t st) {
  const int nt = L.b_pad / kT;
  const int64_t m = L.m;
  const int64_t tri = (int64_t)nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_form, dim3((unsigned)(m * tri)), dim3(256), 0, st, L, P, X, D.kinv);
  for (int k = 0; k < nt; ++k) {
    if (k > 0)
      hipLaunchKernelGGL(k_herk, dim3((unsigned)(m * (nt - k))), dim3(256), 0, st, L, D.kinv, k);
    hipLaunchKernelGGL(k_potrf_diag, dim3((unsigned)m), dim3(256), 0, st, L, D.kinv, D.dinv,
                       D.ctl, k);
    const int r = nt - k - 1;
    if (r > 0)
      hipLaunchKernelGGL(k_trsm, dim3((unsigned)(m * r)), dim3(256), 0, st, L, D.kinv, D.dinv,
                         k);
  }
  for (int jc = nt - 1; jc >= 0; --jc) {
    const int rows = nt - jc - 1;
    if (rows > 0)
      hipLaunchKernelGGL(k_trtri_panel, dim3((unsigned)(m * rows)), dim3(256), 0, st, L,
                         D.kinv, D.dinv, D.panel, jc);
    hipLaunchKernelGGL(k_trtri_writeback, dim3((unsigned)(m * (rows + 1))), dim3(256), 0, st, L,
                       D.kinv, D.dinv, D.panel, jc);
  }
  for (int i = 0; i < nt; ++i) {
    if (i > 0)
      hipLaunchKernelGGL(k_lauum, dim3((unsigned)(m * i)), dim3(256), 0, st, L, D.kinv, i, 0);
    hipLaunchKernelGGL(k_lauum, dim3((unsigned)m), dim3(256), 0, st, L, D.kinv, i, 1);
  }
  hipLaunchKernelGGL(k_mirror, dim3((unsigned)(m * tri)), dim3(256), 0, st, L, D.kinv);
  return hipGetLastError();
}

hipError_t launch_copy_inverse(const Layout& L, const Dev& D, int32_t j, double* dst,
                               hipStream_t st) {
  int len = (int)std::min<int64_t>(L.b, L.n - (int64_t)j * L.b);
  int64_t total = (int64_t)len * len;
  unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 65535);
  hipLaunchKernelGGL(k_copy_block, dim3(g), dim3(256), 0, st, L, D.kinv, j, len, dst);
  return hipGetLastError();
}

}  // namespace ap
