// Stochastic gradient of the negative log marginal likelihood (Section 2,
// eq. loss_grad_unbiased) from a solve's W = K^^{-1} B, B = [y, z_1 .. z_P]:
//   grad_theta = -1/2 w_0^T (dK^/dtheta) w_0 + 1/(2P) sum_p w_p^T (dK^/dtheta) z_p
//             = sum_{i,j} C_ij (dK^/dtheta)_ij,
//   C_ij = W_i . bc_j,   bc_j = [-W_j0 / 2, B_j1 / (2P), .., B_jP / (2P)],
// for theta = the d lengthscales, the outputscale s and the noise sigma^2:
//   dk/dell_m = g(r) (x_m - x'_m)^2 / ell_m^3,  dK^/ds = K / s,  dK^/dsigma^2 = I,
// with g = k (RBF), 3 s e^{-sqrt3 r} (Matern-3/2), (5/3) s (1 + sqrt5 r)
// e^{-sqrt5 r} (Matern-5/2). Every term of the double sum over n^2 pairs is
// formed in registers in FP64 and never stored; the sigma^2 component, the
// trace of C, is a sum over rows.
//
// Workgroup: 4 waves x 16 rows; the columns are staged in LDS 64 at a time
// (prescaled features and bc, padded to a multiple of 4; the bc rows are
// 4 mod 32 doubles apart, so the 16 columns of a tile that a matrix
// instruction's B operand reads fall in different LDS banks). C_ij for a 16 x 16
// tile of pairs is the rank-l product W_tile bc_tile^T, formed on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: the wave's W rows are the A operand,
// held in registers; bc the B operand), which leaves each lane four pairs
// (rows lane / 16 + 4 q, column lane % 16) whose kernel value, derivative
// factor and d + 2 sums it forms on the vector units. The workgroup reduces
// the sums in a fixed order to one partial per 64 rows, and a last kernel adds
// the partials in order.
#include <algorithm>

#include "ap_internal.h"
#include "kmap64.h"

namespace ap {
namespace {

typedef __attribute__((ext_vector_type(4))) double f64x4;
constexpr int kColsG = 64;
constexpr int kRowsG = 64;

template <int KERN, int DV, int DP, int KS>
__global__ __launch_bounds__(256) void k_mll_grad(Layout L, Params P, const float* __restrict__ X,
                                                  const float* __restrict__ B,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ part) {
  constexpr int NG = DV + 2;
  constexpr int KP = 4 * KS;  // coefficients per point, padded to the matrix K step
  constexpr int KPS = KP == 4 ? 4 : 36;  // LDS row stride of bc (4 mod 32 doubles)
  constexpr int UNR = DP <= 8 ? 2 : 1;  // tiles in flight (register budget)
  __shared__ double sx[kColsG][DP];
  __shared__ double sb[kColsG][KPS];
  __shared__ double etab[kExpTab];
  __shared__ double red[4][NG];
  scaled_exp_table(etab, P.s);  // visible after the first barrier of the column loop
  const int d = L.d, l = L.l, np = L.l - 1;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsG + wave * 16;
  double inv_ell[DV];
#pragma unroll
  for (int k = 0; k < DV; ++k) inv_ell[k] = k < d ? 1.0 / P.ell[k] : 0.0;
  // A operand of v_mfma_f64_16x16x4f64: W[row0 + lane % 16][4 s + lane / 16]
  double a[KS];
  {
    const int64_t i = row0 + ln;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int c = 4 * s + lg;
      a[s] = (i < L.n && c < l) ? W[i * l + c] : 0.0;
    }
  }
  // the lane's output pairs are rows row0 + lane / 16 + 4 q (q = 0..3)
  double xi[4][DV];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = row0 + lg + 4 * q;
#pragma unroll
    for (int k = 0; k < DV; ++k)
      xi[q][k] = (i < L.n && k < d) ? (double)X[i * d + k] * inv_ell[k] : 0.0;
  }
  double g[NG];
#pragma unroll
  for (int m = 0; m < NG; ++m) g[m] = 0.0;
  const double inv2p = np > 0 ? 0.5 / np : 0.0;

  for (int64_t j0 = 0; j0 < L.n; j0 += kColsG) {
    __syncthreads();
    for (int e = threadIdx.x; e < kColsG * DP; e += 256) {
      const int jj = e / DP, k = e % DP;
      sx[jj][k] = (j0 + jj < L.n && k < d) ? (double)X[(j0 + jj) * d + k] * (1.0 / P.ell[k])
                                            : 0.0;
    }
    for (int e = threadIdx.x; e < kColsG * KP; e += 256) {
      const int jj = e / KP, c = e % KP;
      const int64_t j = j0 + jj;
      double v = 0.0;
      if (j < L.n && c < l) v = c == 0 ? -0.5 * W[j * l] : (double)B[j * l + c] * inv2p;
      sb[jj][c] = v;
    }
    __syncthreads();
#pragma unroll UNR
    for (int tile = 0; tile < kColsG / 16; ++tile) {
      const int jj = 16 * tile + ln;  // this lane's column in the 16 x 16 tile
      // C[m][n] = sum_k W[row0 + m][k] bc[j0 + 16 tile + n][k]; the lane receives
      // C at (m = lane / 16 + 4 q, n = lane % 16).
      f64x4 cc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s)
        cc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], sb[jj][4 * s + lg], cc, 0, 0, 0);
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[jj][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double q2[DV], r2 = 0.0;
#pragma unroll
        for (int k = 0; k < DV; ++k) {
          const double dq = xi[q][k] - xc[k];
          q2[k] = dq * dq;
          r2 += q2[k];
        }
        double kv, gv;
        if constexpr (KERN == 0) {
          kv = scaled_exp_nhalf(r2, etab);
          gv = kv;
        } else if constexpr (KERN == 1) {
          const double t = 1.7320508075688772 * sqrt(r2);
          const double e = scaled_exp(-t, etab);
          kv = (1.0 + t) * e;
          gv = 3.0 * e;
        } else {
          const double t = 2.23606797749979 * sqrt(r2);
          const double e = scaled_exp(-t, etab);
          kv = (1.0 + t + (5.0 / 3.0) * r2) * e;
          gv = (5.0 / 3.0) * (1.0 + t) * e;
        }
        const double cij = cc[q];
        const double cg = cij * gv;
#pragma unroll
        for (int k = 0; k < DV; ++k) g[k] = fma(cg, q2[k], g[k]);
        g[DV] = fma(cij, kv, g[DV]);
      }
    }
  }
  // dK^/dsigma^2 = I: the trace of C, sum_i W_i . bc_i, one row per lane of
  // the wave's first 16
  if (lane < 16 && row0 + lane < L.n) {
    const int64_t i = row0 + lane;
    double t = -0.5 * W[i * l] * W[i * l];
    for (int c = 1; c < l; ++c) t = fma(W[i * l + c], (double)B[i * l + c] * inv2p, t);
    g[DV + 1] = t;
  }
  // lanes -> wave (fixed butterfly) -> workgroup (waves in order)
#pragma unroll
  for (int m = 0; m < NG; ++m) {
    double v = g[m];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane == 0) red[wave][m] = v;
  }
  __syncthreads();
  if (threadIdx.x < kMaxD + 2) {
    const int m = threadIdx.x;
    double v = 0.0;
    // scale: q^2 = (dx / ell)^2 needs one more 1 / ell; K / s for the outputscale
    if (m < d)
      v = (((red[0][m] + red[1][m]) + red[2][m]) + red[3][m]) / P.ell[m];
    else if (m == d)
      v = (((red[0][DV] + red[1][DV]) + red[2][DV]) + red[3][DV]) / P.s;
    else if (m == d + 1)
      v = ((red[0][DV + 1] + red[1][DV + 1]) + red[2][DV + 1]) + red[3][DV + 1];
    part[(size_t)blockIdx.x * (kMaxD + 2) + m] = v;
  }
}

// Fixed-order sum of the per-64-row partials (one workgroup).
__global__ __launch_bounds__(256) void k_mll_final(Layout L, const double* __restrict__ part,
                                                   Ctl* ctl) {
  __shared__ double red[256];
  for (int m = 0; m < L.d + 2; ++m) {
    double acc = 0.0;
    for (int w = threadIdx.x; w < L.nwg_mll; w += 256) acc += part[(size_t)w * (kMaxD + 2) + m];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) ctl->mll_grad[m] = red[0];
    __syncthreads();
  }
}

template <int KERN, int DV, int DP>
void launch_lc(const Layout& L, const Dev& D, const Params& P, const float* X, const float* B,
               const double* W, hipStream_t st) {
  const dim3 g((unsigned)L.nwg_mll), t(256);
#define AP_MLL(KS) \
  hipLaunchKernelGGL((k_mll_grad<KERN, DV, DP, KS>), g, t, 0, st, L, P, X, B, W, D.gpart)
  if (L.l <= 4) AP_MLL(1);
  else if (L.l <= 8) AP_MLL(2);
  else if (L.l <= 16) AP_MLL(4);
  else AP_MLL(8);
#undef AP_MLL
}

template <int KERN>
void launch_dp(const Layout& L, const Dev& D, const Params& P, const float* X, const float* B,
               const double* W, hipStream_t st) {
  if (L.d == 3) {
    launch_lc<KERN, 3, 4>(L, D, P, X, B, W, st);
    return;
  }
  switch (L.dp) {
    case 4: launch_lc<KERN, 4, 4>(L, D, P, X, B, W, st); break;
    case 8: launch_lc<KERN, 8, 8>(L, D, P, X, B, W, st); break;
    case 12: launch_lc<KERN, 12, 12>(L, D, P, X, B, W, st); break;
    case 16: launch_lc<KERN, 16, 16>(L, D, P, X, B, W, st); break;
    default: launch_lc<KERN, 20, 20>(L, D, P, X, B, W, st); break;
  }
}

}  // namespace

hipError_t launch_mll_grad(const Layout& L, const Dev& D, const Params& P, const float* X,
                           const float* B, const double* W, hipStream_t st) {
  switch (L.kernel) {
    case 0: launch_dp<0>(L, D, P, X, B, W, st); break;
    case 1: launch_dp<1>(L, D, P, X, B, W, st); break;
    default: launch_dp<2>(L, D, P, X, B, W, st); break;
  }
  hipLaunchKernelGGL(k_mll_final, dim3(1), dim3(256), 0, st, L, D.gpart, D.ctl);
  return hipGetLastError();
}

}  // namespace ap
