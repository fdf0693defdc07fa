// Fused residual update with FP64 kernel tiles (eq. text_update_of_r):
//   R <- R - K^_{:,I} delta,  rows of I set to 0,
// for systems whose conditioning defeats FP32 tiles. The product K^_{:,I} delta
// cancels to |R| from terms as large as |K||delta| (far larger when K^_{I,I} is
// close to singular), so the rounding of the kernel values, not of R, decides
// whether the maintained residual stays true. Here every kernel value is FP64
// (squared distance of the centred inputs over the lengthscales, FP64 map) and the
// product runs on v_mfma_f64_16x16x4f64 with FP64 accumulation; only the stored
// residual is FP32, whose rounding is relative to |R| itself.
//
// Workgroup: 4 waves x 64 rows (four 16-row tiles each), the same 256-row
// geometry and per-workgroup column partials as the other tile modes. The
// block's columns are staged through LDS 64 at a time (features and step); per
// step of 4 columns a lane evaluates one kernel value per row tile (row
// lane % 16, column lane / 16) and the matrix cores accumulate
// acc[c][i] += delta^T[c][j] K^T[j][i] for 16 right-hand sides per half.
//
// The squared distance comes from the norm expansion of the centred features
// u = (x - mu) / ell: |u_i|^2 + |u_j|^2 - 2 u_i.u_j, with the column held as
// -2 u_j and its norm, d + 1 FP64 operations where differencing takes 2d. The
// cancellation costs an absolute error near 1e-13 in r^2 (|u|^2 is at most a
// few hundred), far below the FP32 rounding of the stored residual; the FP64
// references (true residual, posterior mean, MLL gradient) keep exact
// differencing.
#include <algorithm>

#include "ap_internal.h"
#include "kmap64.h"

namespace ap {
namespace {

typedef __attribute__((ext_vector_type(4))) double f64x4;
constexpr int kCols64 = 64;

// Row features centred and scaled, u = (x - mu) / ell (zero past d and n),
// and |u|^2 in the order the staged columns use.
template <int DV>
__device__ __forceinline__ void row_feat(const float* __restrict__ X, int64_t i, int64_t n,
                                         int d, const Params& P, const Ctl* ctl, double* u,
                                         double* nu) {
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < DV; ++k) {
    u[k] = (i < n && k < d) ? ((double)X[i * d + k] - ctl->mu[k]) / P.ell[k] : 0.0;
    a = fma(u[k], u[k], a);
  }
  *nu = a;
}

// A block's columns c0 .. c0 + kCols64 - 1 staged as -2 u_j (sx) and |u_j|^2
// (sn), one column per thread of the first kCols64; columns past len are zero.
// The caller brackets it with barriers.
template <int DV, int DP>
__device__ __forceinline__ void stage_cols64(const float* __restrict__ X, int64_t start, int c0,
                                             int len, int d, const Params& P, const Ctl* ctl,
                                             double (*sx)[DP], double* sn) {
  if (threadIdx.x < kCols64) {
    const int jj = threadIdx.x;
    const bool in = c0 + jj < len;
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < DP; ++k) {
      double u = 0.0;
      if (in && k < d) u = ((double)X[(start + c0 + jj) * d + k] - ctl->mu[k]) / P.ell[k];
      a = fma(u, u, a);
      sx[jj][k] = -2.0 * u;
    }
    sn[jj] = a;
  }
}

template <int DV>
__device__ __forceinline__ double dist2n64(const double* u, double nu, const double* m2, double nj) {
  double a = nu + nj;
#pragma unroll
  for (int k = 0; k < DV; ++k) a = fma(u[k], m2[k], a);
  return a;
}

template <int KERN, int DV, int DP, int NH>
__global__ __launch_bounds__(256) void k_fused_fp64(Layout L, Params P, const float* __restrict__ X,
                                                    const double* __restrict__ delta,
                                                    const Ctl* __restrict__ ctl, int block,
                                                    float* __restrict__ R,
                                                    float* __restrict__ rowsq,
                                                    float* __restrict__ colsq, int want_rowsq,
                                                    int want_colsq) {
  __shared__ double sx[kCols64][DP];
  __shared__ double sn[kCols64];
  __shared__ double sd[kCols64][16 * NH];
  __shared__ float red[4][kMaxL];
  __shared__ double etab[kExpTab];  // s * 2^(j/256) for the exponential
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  scaled_exp_table(etab, P.s);  // visible after the first barrier of the chunk loop
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int d = L.d, l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 64;

  double xi[4][DV], ni[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) row_feat<DV>(X, row0 + 16 * t + ln, L.n, d, P, ctl, xi[t], &ni[t]);
  f64x4 acc[4][NH];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int h = 0; h < NH; ++h) acc[t][h] = f64x4{0.0, 0.0, 0.0, 0.0};

  for (int c0 = 0; c0 < len; c0 += kCols64) {
    __syncthreads();
    stage_cols64<DV, DP>(X, start, c0, len, d, P, ctl, sx, sn);
    for (int e = threadIdx.x; e < kCols64 * 16 * NH; e += 256) {
      const int jj = e / (16 * NH), c = e % (16 * NH);
      sd[jj][c] = (c0 + jj < len) ? delta[(size_t)(c0 + jj) * kMaxL + c] : 0.0;
    }
    __syncthreads();
    const int steps = std::min(kCols64, len - c0 + 3) / 4;
    for (int st = 0; st < steps; ++st) {
      const int jj = 4 * st + lg;
      double a[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) a[h] = sd[jj][16 * h + ln];
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[jj][k];
      const double nc = sn[jj];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double r2 = dist2n64<DV>(xi[t], ni[t], xc, nc);
        if constexpr (KERN != 0) r2 = fmax(r2, 0.0);
        const double kv = kernel_fp64<KERN>(r2, etab);
#pragma unroll
        for (int h = 0; h < NH; ++h)
          acc[t][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], kv, acc[t][h], 0, 0, 0);
      }
    }
  }

  // lane holds acc[t][h][q]: row row0 + 16 t + lane % 16, column c = 16 h + lane / 16 + 4 q
  float csum[NH][4];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) csum[h][q] = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t row = row0 + 16 * t + ln;
    const bool live = row < L.n;
    const bool in_i = row >= start && row < start + len;
    float rs = 0.f;
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 16 * h + lg + 4 * q;
        if (live && c < l) {
          const float r = in_i ? 0.f : (float)((double)R[row * l + c] - acc[t][h][q]);
          R[row * l + c] = r;
          rs = fmaf(r, r, rs);
          csum[h][q] = fmaf(r, r, csum[h][q]);
        }
      }
    if (want_rowsq) {
      rs += __shfl_xor(rs, 16);
      rs += __shfl_xor(rs, 32);
      if (lg == 0 && row < L.n_pad) rowsq[row] = live ? rs : 0.f;
    }
  }
  if (want_colsq) {
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float x = csum[h][q];
        x += __shfl_xor(x, 1);
        x += __shfl_xor(x, 2);
        x += __shfl_xor(x, 4);
        x += __shfl_xor(x, 8);
        if (ln == 0) red[wave][16 * h + lg + 4 * q] = x;
      }
    __syncthreads();
    if (threadIdx.x < kMaxL) {
      const int c = threadIdx.x;
      float v = 0.f;
      if (c < 16 * NH) v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      colsq[blockIdx.x * kMaxL + c] = c < l ? v : 0.f;
    }
  }
}

// Few right-hand sides (l <= 8): the product with the step on the vector units.
// On gfx950 a wave's FP64 FMA and an FP64 matrix instruction retire the same
// number of multiply-adds per cycle on the same pipe, so for l <= 8 the vector
// form does l multiply-adds per kernel entry where the 16-column matrix tile
// does 16. A lane accumulates, for each of its four row tiles, the columns
// j = 4 st + lane / 16 of the block; the four lanes of a row then add their
// partial sums in a fixed order (every lane ends with the same total).
template <int KERN, int DV, int DP, int NV>
__global__ __launch_bounds__(256) void k_fused_fp64v(Layout L, Params P,
                                                     const float* __restrict__ X,
                                                     const double* __restrict__ delta,
                                                     const Ctl* __restrict__ ctl, int block,
                                                     float* __restrict__ R,
                                                     float* __restrict__ rowsq,
                                                     float* __restrict__ colsq, int want_rowsq,
                                                     int want_colsq) {
  constexpr int NQ = (NV + 3) / 4;  // output columns per lane
  __shared__ double sx[kCols64][DP];
  __shared__ double sn[kCols64];
  __shared__ double sd[kCols64][NV];
  __shared__ float red[4][kMaxL];
  __shared__ double etab[kExpTab];  // s * 2^(j/256) for the exponential
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  scaled_exp_table(etab, P.s);  // visible after the first barrier of the chunk loop
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int d = L.d, l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 64;

  double xi[4][DV], ni[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) row_feat<DV>(X, row0 + 16 * t + ln, L.n, d, P, ctl, xi[t], &ni[t]);
  double acc[4][NV];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[t][c] = 0.0;

  for (int c0 = 0; c0 < len; c0 += kCols64) {
    __syncthreads();
    stage_cols64<DV, DP>(X, start, c0, len, d, P, ctl, sx, sn);
    for (int e = threadIdx.x; e < kCols64 * NV; e += 256) {
      const int jj = e / NV, c = e % NV;
      sd[jj][c] = (c0 + jj < len) ? delta[(size_t)(c0 + jj) * kMaxL + c] : 0.0;
    }
    __syncthreads();
    const int steps = std::min(kCols64, len - c0 + 3) / 4;
    for (int st = 0; st < steps; ++st) {
      const int jj = 4 * st + lg;
      double a[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) a[c] = sd[jj][c];
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[jj][k];
      const double nc = sn[jj];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double r2 = dist2n64<DV>(xi[t], ni[t], xc, nc);
        if constexpr (KERN != 0) r2 = fmax(r2, 0.0);
        const double kv = kernel_fp64<KERN>(r2, etab);
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[t][c] = fma(kv, a[c], acc[t][c]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      acc[t][c] += __shfl_xor(acc[t][c], 16);
      acc[t][c] += __shfl_xor(acc[t][c], 32);
    }

  // lane writes columns c = lane / 16 + 4 q of its row
  float csum[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) csum[q] = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t row = row0 + 16 * t + ln;
    const bool live = row < L.n;
    const bool in_i = row >= start && row < start + len;
    float rs = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = lg + 4 * q;
      double v = 0.0;
#pragma unroll
      for (int cc = 4 * q; cc < 4 * q + 4 && cc < NV; ++cc)
        if (cc == c) v = acc[t][cc];
      if (live && c < l) {
        const float r = in_i ? 0.f : (float)((double)R[row * l + c] - v);
        R[row * l + c] = r;
        rs = fmaf(r, r, rs);
        csum[q] = fmaf(r, r, csum[q]);
      }
    }
    if (want_rowsq) {
      rs += __shfl_xor(rs, 16);
      rs += __shfl_xor(rs, 32);
      if (lg == 0 && row < L.n_pad) rowsq[row] = live ? rs : 0.f;
    }
  }
  if (want_colsq) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float x = csum[q];
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 8);
      if (ln == 0 && lg + 4 * q < NV) red[wave][lg + 4 * q] = x;
    }
    __syncthreads();
    if (threadIdx.x < kMaxL) {
      const int c = threadIdx.x;
      float v = 0.f;
      if (c < NV) v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      colsq[blockIdx.x * kMaxL + c] = c < l ? v : 0.f;
    }
  }
}

template <int KERN, int NV>
hipError_t launch_nv(const Layout& L, const Dev& D, const Params& P, const float* X, int32_t block,
                     float* R, bool wr, bool wc, hipStream_t st) {
  const dim3 g(L.nwg), t(256);
#define AP_F64V(DV, DP)                                                                          \
  hipLaunchKernelGGL((k_fused_fp64v<KERN, DV, DP, NV>), g, t, 0, st, L, P, X, D.delta, D.ctl,   \
                     block, R, D.rowsq, D.colsq, (int)wr, (int)wc)
  if (L.d == 3) {
    AP_F64V(3, 4);
  } else {
    switch (L.dp) {
      case 4: AP_F64V(4, 4); break;
      case 8: AP_F64V(8, 8); break;
      case 12: AP_F64V(12, 12); break;
      case 16: AP_F64V(16, 16); break;
      case 20: AP_F64V(20, 20); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef AP_F64V
  return hipGetLastError();
}

template <int KERN, int NH>
hipError_t launch_nh(const Layout& L, const Dev& D, const Params& P, const float* X, int32_t block,
                     float* R, bool wr, bool wc, hipStream_t st) {
  const dim3 g(L.nwg), t(256);
#define AP_F64(DV, DP)                                                                           \
  hipLaunchKernelGGL((k_fused_fp64<KERN, DV, DP, NH>), g, t, 0, st, L, P, X, D.delta, D.ctl, block, \
                     R, D.rowsq, D.colsq, (int)wr, (int)wc)
  if (L.d == 3) {
    AP_F64(3, 4);
  } else {
    switch (L.dp) {
      case 4: AP_F64(4, 4); break;
      case 8: AP_F64(8, 8); break;
      case 12: AP_F64(12, 12); break;
      case 16: AP_F64(16, 16); break;
      case 20: AP_F64(20, 20); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef AP_F64
  return hipGetLastError();
}

template <int KERN>
hipError_t launch_k(const Layout& L, const Dev& D, const Params& P, const float* X, int32_t block,
                    float* R, bool wr, bool wc, hipStream_t st) {
  if (L.l <= 1) return launch_nv<KERN, 1>(L, D, P, X, block, R, wr, wc, st);
  if (L.l <= 2) return launch_nv<KERN, 2>(L, D, P, X, block, R, wr, wc, st);
  if (L.l <= 4) return launch_nv<KERN, 4>(L, D, P, X, block, R, wr, wc, st);
  if (L.l <= 8) return launch_nv<KERN, 8>(L, D, P, X, block, R, wr, wc, st);
  if (L.l <= 16) return launch_nh<KERN, 1>(L, D, P, X, block, R, wr, wc, st);
  return launch_nh<KERN, 2>(L, D, P, X, block, R, wr, wc, st);
}

}  // namespace

hipError_t launch_fused_update64(const Layout& L, const Dev& D, const Params& P, const float* X,
                                 int32_t block, float* R, bool want_rowsq, bool want_colsq,
                                 hipStream_t st) {
  switch (L.kernel) {
    case 0: return launch_k<0>(L, D, P, X, block, R, want_rowsq, want_colsq, st);
    case 1: return launch_k<1>(L, D, P, X, block, R, want_rowsq, want_colsq, st);
    default: return launch_k<2>(L, D, P, X, block, R, want_rowsq, want_colsq, st);
  }
}

}  // namespace ap
