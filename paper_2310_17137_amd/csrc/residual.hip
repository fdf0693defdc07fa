// FP64 true residual R = B - K^ W over all n^2 kernel entries (Lemma
// residual_equality: the maintained residual equals this in exact arithmetic,
// so recomputing it removes the drift of the reduced-precision update).
// The FP32 inputs are widened to FP64 and scaled by 1 / ell (as in the FP64-tile
// update), then differenced in FP64; FP64 kernel map, FP64 accumulation in a
// fixed column order on the FP64 matrix cores, and the noise term added per row
// after the column loop. The columns' features and weights are staged through
// LDS.
#include <algorithm>

#include "ap_internal.h"
#include "kmap64.h"

namespace ap {
namespace {

constexpr int kCols = 64;   // columns staged in LDS per step

// Row tiles (16 rows) per wave: a workgroup covers 64 TL rows. From 2^17 rows
// four (the staged columns serve more rows); below, one, so that enough
// workgroups exist to fill the chip.
inline int res_tiles(int64_t nr) { return nr >= (int64_t(1) << 17) ? 4 : 1; }

typedef __attribute__((ext_vector_type(4))) double f64x4;

// The product sum_j K_ij W_jc runs on v_mfma_f64_16x16x4f64: per step of 4
// columns a lane evaluates one kernel entry per row tile (row lane % 16, column
// lane / 16) in FP64 on the vector ALUs, and the matrix cores accumulate
// acc[c][i] += W^T[c][j] K^T[j][i] for 16 right-hand sides per half (NH halves).
// The noise term sigma^2 W_i of K^ W is added per row after the column loop.
//
// With PRED the rows are nr test points Xr instead of the training points: the
// kernel computes the posterior mean K(Xr, X) W (no noise term, Section 2 GP
// regression) into mean (nr x l, FP64) and skips the norms.
template <int KERN, int DV, int DP, int NH, int TL, bool PRED>
__global__ __launch_bounds__(256) void k_residual(Layout L, Params P, const float* __restrict__ X,
                                                  const float* __restrict__ Xr, int64_t nr,
                                                  const float* __restrict__ B,
                                                  const double* __restrict__ W,
                                                  float* __restrict__ Rout,
                                                  double* __restrict__ mean,
                                                  float* __restrict__ rowsq,
                                                  double* __restrict__ part) {
  __shared__ double sx[kCols][DP];
  __shared__ double sw[kCols][16 * NH];
  __shared__ double red[4][16 * NH];
  __shared__ double etab[kExpTab];  // s * 2^(j/256) for the exponential
  scaled_exp_table(etab, P.s);  // visible after the first barrier of the column loop
  const int d = L.d, l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * TL) + wave * (16 * TL);
  double inv_ell[DV], xi[TL][DV];
#pragma unroll
  for (int k = 0; k < DV; ++k) inv_ell[k] = k < d ? 1.0 / P.ell[k] : 0.0;
#pragma unroll
  for (int t = 0; t < TL; ++t) {
    const int64_t i = row0 + 16 * t + ln;
#pragma unroll
    for (int k = 0; k < DV; ++k)
      xi[t][k] = (i < nr && k < d) ? (double)Xr[i * d + k] * inv_ell[k] : 0.0;
  }
  f64x4 acc[TL][NH];
#pragma unroll
  for (int t = 0; t < TL; ++t)
#pragma unroll
    for (int h = 0; h < NH; ++h) acc[t][h] = f64x4{0.0, 0.0, 0.0, 0.0};

  for (int64_t j0 = 0; j0 < L.n; j0 += kCols) {
    __syncthreads();
    for (int e = threadIdx.x; e < kCols * DP; e += 256) {
      const int jj = e / DP, k = e % DP;
      sx[jj][k] = (j0 + jj < L.n && k < d) ? (double)X[(j0 + jj) * d + k] * (1.0 / P.ell[k])
                                            : 0.0;
    }
    for (int e = threadIdx.x; e < kCols * 16 * NH; e += 256) {
      const int jj = e / (16 * NH), c = e % (16 * NH);
      sw[jj][c] = (j0 + jj < L.n && c < l) ? W[(j0 + jj) * l + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int st = 0; st < kCols / 4; ++st) {
      const int jj = 4 * st + lg;
      double a[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) a[h] = sw[jj][16 * h + ln];
#pragma unroll
      for (int t = 0; t < TL; ++t) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < DV; ++k) {
          const double df = xi[t][k] - sx[jj][k];
          r2 = fma(df, df, r2);
        }
        const double kv = kernel_fp64<KERN>(r2, etab);
#pragma unroll
        for (int h = 0; h < NH; ++h)
          acc[t][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], kv, acc[t][h], 0, 0, 0);
      }
    }
  }
  // lane holds acc[t][h][q] for row row0 + 16 t + lane % 16 and right-hand side
  // c = 16 h + lane / 16 + 4 q (the FP64 16x16 accumulator layout)
  if constexpr (PRED) {
#pragma unroll
    for (int t = 0; t < TL; ++t) {
      const int64_t i = row0 + 16 * t + ln;
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = 16 * h + lg + 4 * q;
          if (i < nr && c < l) mean[i * l + c] = acc[t][h][q];
        }
    }
    return;
  }
  double csum[NH][4];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) csum[h][q] = 0.0;
#pragma unroll
  for (int t = 0; t < TL; ++t) {
    const int64_t i = row0 + 16 * t + ln;
    const bool live = i < nr;
    double rs = 0.0;
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 16 * h + lg + 4 * q;
        if (live && c < l) {
          const double kw = fma(P.noise, W[i * l + c], acc[t][h][q]);
          const double r = (double)B[i * l + c] - kw;
          Rout[i * l + c] = (float)r;
          rs = fma(r, r, rs);
          csum[h][q] = fma(r, r, csum[h][q]);
        }
      }
    rs += __shfl_xor(rs, 16);
    rs += __shfl_xor(rs, 32);
    if (rowsq && live && lg == 0) rowsq[i] = (float)rs;
  }
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double x = csum[h][q];
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 8);
      if (ln == 0) red[wave][16 * h + lg + 4 * q] = x;
    }
  __syncthreads();
  if (threadIdx.x < kMaxL) {
    const int c = threadIdx.x;
    double v = 0.0;
    if (c < 16 * NH) v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    part[(size_t)blockIdx.x * kMaxL + c] = c < l ? v : 0.0;
  }
}

// Few right-hand sides (l <= 8): the product on the vector units (as the FP64
// fused update does for l <= 8: an FP64 FMA and an FP64 matrix instruction
// retire multiply-adds at the same rate on gfx950, and the matrix tile would
// pad l to 16). Each lane accumulates the columns j = 4 st + lane / 16 of its
// four rows; the four lanes of a row add their partials in a fixed order.
template <int KERN, int DV, int DP, int NV, int TL, bool PRED>
__global__ __launch_bounds__(256) void k_residualv(Layout L, Params P, const float* __restrict__ X,
                                                   const float* __restrict__ Xr, int64_t nr,
                                                   const float* __restrict__ B,
                                                   const double* __restrict__ W,
                                                   float* __restrict__ Rout,
                                                   double* __restrict__ mean,
                                                   float* __restrict__ rowsq,
                                                   double* __restrict__ part) {
  constexpr int NQ = (NV + 3) / 4;
  __shared__ double sx[kCols][DP];
  __shared__ double sw[kCols][NV];
  __shared__ double red[4][kMaxL];
  __shared__ double etab[kExpTab];  // s * 2^(j/256) for the exponential
  scaled_exp_table(etab, P.s);  // visible after the first barrier of the column loop
  const int d = L.d, l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * TL) + wave * (16 * TL);
  double inv_ell[DV], xi[TL][DV];
#pragma unroll
  for (int k = 0; k < DV; ++k) inv_ell[k] = k < d ? 1.0 / P.ell[k] : 0.0;
#pragma unroll
  for (int t = 0; t < TL; ++t) {
    const int64_t i = row0 + 16 * t + ln;
#pragma unroll
    for (int k = 0; k < DV; ++k)
      xi[t][k] = (i < nr && k < d) ? (double)Xr[i * d + k] * inv_ell[k] : 0.0;
  }
  double acc[TL][NV];
#pragma unroll
  for (int t = 0; t < TL; ++t)
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[t][c] = 0.0;

  for (int64_t j0 = 0; j0 < L.n; j0 += kCols) {
    __syncthreads();
    for (int e = threadIdx.x; e < kCols * DP; e += 256) {
      const int jj = e / DP, k = e % DP;
      sx[jj][k] = (j0 + jj < L.n && k < d) ? (double)X[(j0 + jj) * d + k] * (1.0 / P.ell[k])
                                            : 0.0;
    }
    for (int e = threadIdx.x; e < kCols * NV; e += 256) {
      const int jj = e / NV, c = e % NV;
      sw[jj][c] = (j0 + jj < L.n && c < l) ? W[(j0 + jj) * l + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int st = 0; st < kCols / 4; ++st) {
      const int jj = 4 * st + lg;
      double a[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) a[c] = sw[jj][c];
#pragma unroll
      for (int t = 0; t < TL; ++t) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < DV; ++k) {
          const double df = xi[t][k] - sx[jj][k];
          r2 = fma(df, df, r2);
        }
        const double kv = kernel_fp64<KERN>(r2, etab);
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[t][c] = fma(kv, a[c], acc[t][c]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TL; ++t)
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      acc[t][c] += __shfl_xor(acc[t][c], 16);
      acc[t][c] += __shfl_xor(acc[t][c], 32);
    }
  if constexpr (PRED) {
#pragma unroll
    for (int t = 0; t < TL; ++t) {
      const int64_t i = row0 + 16 * t + ln;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = lg + 4 * q;
        double v = 0.0;
#pragma unroll
        for (int cc = 4 * q; cc < 4 * q + 4 && cc < NV; ++cc)
          if (cc == c) v = acc[t][cc];
        if (i < nr && c < l) mean[i * l + c] = v;
      }
    }
    return;
  }
  double csum[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) csum[q] = 0.0;
#pragma unroll
  for (int t = 0; t < TL; ++t) {
    const int64_t i = row0 + 16 * t + ln;
    const bool live = i < nr;
    double rs = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = lg + 4 * q;
      double v = 0.0;
#pragma unroll
      for (int cc = 4 * q; cc < 4 * q + 4 && cc < NV; ++cc)
        if (cc == c) v = acc[t][cc];
      if (live && c < l) {
        const double kw = fma(P.noise, W[i * l + c], v);
        const double r = (double)B[i * l + c] - kw;
        Rout[i * l + c] = (float)r;
        rs = fma(r, r, rs);
        csum[q] = fma(r, r, csum[q]);
      }
    }
    rs += __shfl_xor(rs, 16);
    rs += __shfl_xor(rs, 32);
    if (rowsq && live && lg == 0) rowsq[i] = (float)rs;
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = csum[q];
    x += __shfl_xor(x, 1);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 8);
    if (ln == 0 && lg + 4 * q < NV) red[wave][lg + 4 * q] = x;
  }
  __syncthreads();
  if (threadIdx.x < kMaxL) {
    const int c = threadIdx.x;
    double v = 0.0;
    if (c < NV) v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    part[(size_t)blockIdx.x * kMaxL + c] = c < l ? v : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_residual_final(Layout L, const double* __restrict__ part,
                                                        int groups, Ctl* ctl) {
  __shared__ double red[256];
  __shared__ double ratio[kMaxL];
  for (int c = 0; c < L.l; ++c) {
    double acc = 0.0;
    for (int g = threadIdx.x; g < groups; g += 256) acc += part[(size_t)g * kMaxL + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double bn = ctl->bnorm2[c];
      double r = bn > 0.0 ? sqrt(red[0]) / sqrt(bn) : 0.0;
      if (!isfinite(red[0])) r = NAN;
      ratio[c] = r;
      ctl->colrel_true[c] = r;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int c = 0; c < L.l; ++c) acc += ratio[c];
    ctl->rho_true = acc / L.l;
    if (!isfinite(ctl->rho_true)) ctl->status = -3;
  }
}

// Rows: nr points Xr (the training points for the residual, test points for
// the posterior mean); 64 res_tiles(nr) rows per workgroup.
struct ResArgs {
  const float* X;
  const float* Xr;
  int64_t nr;
  const float* B;
  const double* W;
  float* Rout;
  double* mean;
  float* rowsq;
  double* part;
};

template <int KERN, int NH, int TL, bool PRED>
void launch_res_d(const Layout& L, const Params& P, const ResArgs& a, hipStream_t st) {
  const dim3 g((unsigned)((a.nr + 64 * TL - 1) / (64 * TL))), t(256);
#define AP_RES(DV, DP)                                                                       \
  hipLaunchKernelGGL((k_residual<KERN, DV, DP, NH, TL, PRED>), g, t, 0, st, L, P, a.X, a.Xr,  \
                     a.nr, a.B, a.W, a.Rout, a.mean, a.rowsq, a.part)
  if (L.d == 3) {
    AP_RES(3, 4);
  } else {
    switch (L.dp) {
      case 4: AP_RES(4, 4); break;
      case 8: AP_RES(8, 8); break;
      case 12: AP_RES(12, 12); break;
      case 16: AP_RES(16, 16); break;
      default: AP_RES(20, 20); break;
    }
  }
#undef AP_RES
}

template <int KERN, int NV, int TL, bool PRED>
void launch_res_v(const Layout& L, const Params& P, const ResArgs& a, hipStream_t st) {
  const dim3 g((unsigned)((a.nr + 64 * TL - 1) / (64 * TL))), t(256);
#define AP_RESV(DV, DP)                                                                      \
  hipLaunchKernelGGL((k_residualv<KERN, DV, DP, NV, TL, PRED>), g, t, 0, st, L, P, a.X, a.Xr, \
                     a.nr, a.B, a.W, a.Rout, a.mean, a.rowsq, a.part)
  if (L.d == 3) {
    AP_RESV(3, 4);
  } else {
    switch (L.dp) {
      case 4: AP_RESV(4, 4); break;
      case 8: AP_RESV(8, 8); break;
      case 12: AP_RESV(12, 12); break;
      case 16: AP_RESV(16, 16); break;
      default: AP_RESV(20, 20); break;
    }
  }
#undef AP_RESV
}

template <int KERN, int TL, bool PRED>
void launch_res_t(const Layout& L, const Params& P, const ResArgs& a, hipStream_t st) {
  if (L.l <= 1)
    launch_res_v<KERN, 1, TL, PRED>(L, P, a, st);
  else if (L.l <= 2)
    launch_res_v<KERN, 2, TL, PRED>(L, P, a, st);
  else if (L.l <= 4)
    launch_res_v<KERN, 4, TL, PRED>(L, P, a, st);
  else if (L.l <= 8)
    launch_res_v<KERN, 8, TL, PRED>(L, P, a, st);
  else if (L.l <= 16)
    launch_res_d<KERN, 1, TL, PRED>(L, P, a, st);
  else
    launch_res_d<KERN, 2, TL, PRED>(L, P, a, st);
}

template <int KERN, bool PRED>
void launch_res_k(const Layout& L, const Params& P, const ResArgs& a, hipStream_t st) {
  if (res_tiles(a.nr) == 4)
    launch_res_t<KERN, 4, PRED>(L, P, a, st);
  else
    launch_res_t<KERN, 1, PRED>(L, P, a, st);
}

template <bool PRED>
void launch_res(const Layout& L, const Params& P, const ResArgs& a, hipStream_t st) {
  switch (L.kernel) {
    case 0: launch_res_k<0, PRED>(L, P, a, st); break;
    case 1: launch_res_k<1, PRED>(L, P, a, st); break;
    default: launch_res_k<2, PRED>(L, P, a, st); break;
  }
}

}  // namespace

int residual_groups(int64_t n) {
  const int tl = res_tiles(n);
  return (int)((n + 64 * tl - 1) / (64 * tl));
}

hipError_t launch_residual(const Layout& L, const Dev& D, const Params& P, const float* X,
                           const float* B, const double* W, float* Rout, bool in_place,
                           hipStream_t st) {
  // refining in place keeps the greedy rule's row norms in step with R
  const ResArgs a{X, X, L.n, B, W, Rout, nullptr, in_place ? D.rowsq : nullptr, D.respart};
  launch_res<false>(L, P, a, st);
  const int groups = residual_groups(L.n);
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, L, D.respart, groups, D.ctl);
  return hipGetLastError();
}

hipError_t launch_predict(const Layout& L, const Params& P, const float* X, const double* W,
                          const float* Xs, int64_t ns, double* mean, hipStream_t st) {
  if (ns == 0) return hipSuccess;
  const ResArgs a{X, Xs, ns, nullptr, W, nullptr, mean, nullptr, nullptr};
  launch_res<true>(L, P, a, st);
  return hipGetLastError();
}

}  // namespace ap
