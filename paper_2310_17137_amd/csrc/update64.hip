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
// block's columns are staged through LDS 64 at a time (features, norms and
// step), copied asynchronously into one of two buffers while the other is
// computed; per step of 4 columns a lane evaluates one kernel value per row
// tile (row lane % 16, column lane / 16) and the matrix cores accumulate
// acc[c][i] += delta^T[c][j] K^T[j][i] for 16 right-hand sides per half.
//
// The squared distance comes from the norm expansion of the centred features
// u = (x - mu) / ell (prepared once per factorization with their norms):
// |u_i|^2 + |u_j|^2 - 2 u_i.u_j, with the row held as -2 u_i and the column as
// u_j with its norm, d + 1 FP64 operations where differencing takes 2d. The
// cancellation costs an absolute error near 1e-13 in r^2 (|u|^2 is at most a
// few hundred), far below the FP32 rounding of the stored residual; the FP64
// references (true residual, posterior mean, MLL gradient) keep exact
// differencing.
#include <algorithm>
#include <type_traits>

#include "ap_internal.h"
#include "kmap64.h"

namespace ap {
namespace {

typedef __attribute__((ext_vector_type(4))) double f64x4;
constexpr int kCols64 = 64;

// Asynchronous staging of one step of kCols64 block columns (c0 .. c0 + 63 of
// block start) for the FP64 tile kernels: the columns' centred features u_j
// (kCols64 x DP doubles), their norms |u_j|^2 and the first NS columns of the
// FP64 step's rows are copied from global memory straight into LDS with
// global_load_lds (each lane moves 16 or 4 bytes to base + lane * size; a
// wave-load moves 1 KiB or 256 B). Columns past the block's end carry the next
// points' features (or the zero padding rows) and a zero step, so they add
// exact zeros. A step can reach 63 rows past n while the features are padded to
// n_pad >= n + 32 rows, so the feature and norm sources are clamped to the
// last padding row (zeros). The caller waits (s_waitcnt) and crosses a barrier
// before reading.
template <int DP, int NS, int NW>
__device__ __forceinline__ void stage_async64(const double* __restrict__ xu,
                                              const double* __restrict__ xun,
                                              const double* __restrict__ delta, int64_t n_pad,
                                              int64_t start, int c0, double* sx, double* sn,
                                              double* sd) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t cb = start + c0;
  const double* d0 = delta + (size_t)c0 * kMaxL;
  if constexpr (NS >= 2) {  // step rows in 16-byte pieces (two doubles), QR per row
    constexpr int QR = NS / 2, NP = kCols64 * QR;
    for (int q = wave; 64 * q < NP; q += NW) {
      const int pc = 64 * q + lane;
      if (pc < NP)
        __builtin_amdgcn_global_load_lds(d0 + (pc / QR) * kMaxL + 2 * (pc % QR), sd + 128 * q, 16,
                                         0, 0);
    }
  } else {  // one double per row: two 4-byte pieces each, two wave-loads
    for (int q = wave; q < 2; q += NW) {
      const int pc = 64 * q + lane;  // dword pc of the 64 doubles
      __builtin_amdgcn_global_load_lds((const uint32_t*)(d0 + (pc / 2) * kMaxL) + pc % 2,
                                       sd + 32 * q, 4, 0, 0);
    }
  }
  const int64_t xlast = n_pad * DP - 2;  // first double of the last 16-byte piece
  for (int q = wave; q < kCols64 * DP / 128; q += NW)
    __builtin_amdgcn_global_load_lds(xu + std::min(cb * DP + 128 * q + 2 * lane, xlast),
                                     sx + 128 * q, 16, 0, 0);
  const int64_t nlast = 2 * n_pad - 1;  // last dword of the norms
  for (int q = wave; q < 2; q += NW)  // 64 norms as 128 dwords: 4-byte copies keep odd cb aligned
    __builtin_amdgcn_global_load_lds((const uint32_t*)xun + std::min(2 * cb + 64 * q + lane, nlast),
                                     sn + 32 * q, 4, 0, 0);
}

template <int DV>
__device__ __forceinline__ double dist2n64(const double* m2, double nu, const double* uc, double nj) {
  double a = nu + nj;  // row held as m2 = -2 u_i, column as u_j
#pragma unroll
  for (int k = 0; k < DV; ++k) a = fma(m2[k], uc[k], a);
  return a;
}

template <int KERN, int DV, int DP, int NH>
__global__ __launch_bounds__(256) void k_fused_fp64(
    Layout L, Params P, const double* __restrict__ xu, const double* __restrict__ xun,
    const double* __restrict__ delta, const Ctl* __restrict__ ctl, int block,
    float* __restrict__ R, float* __restrict__ rowsq, float* __restrict__ colsq, int want_rowsq,
    int want_colsq) {
  constexpr int NW = 4;
  __shared__ __attribute__((aligned(16))) double sx[2][kCols64][DP];
  __shared__ __attribute__((aligned(16))) double sn[2][kCols64];
  __shared__ __attribute__((aligned(16))) double sd[2][kCols64][16 * NH];
  __shared__ float red[4][kMaxL];
  __shared__ double etab[kExpTab];  // s * 2^(j/256) for the exponential
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  scaled_exp_table(etab, P.s);  // visible after the first barrier
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 64;
  const int nst = (len + kCols64 - 1) / kCols64;  // steps of kCols64 columns

  stage_async64<DP, 16 * NH, NW>(xu, xun, delta, L.n_pad, start, 0, &sx[0][0][0], sn[0],
                                 &sd[0][0][0]);
  double xi[4][DV], ni[4];  // -2 u_i and |u_i|^2
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int k = 0; k < DV; ++k) xi[t][k] = -2.0 * xu[(row0 + 16 * t + ln) * DP + k];
    ni[t] = xun[row0 + 16 * t + ln];
  }
  f64x4 acc[4][NH];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int h = 0; h < NH; ++h) acc[t][h] = f64x4{0.0, 0.0, 0.0, 0.0};
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // One step from buffer B (a compile-time constant), the next step's copies
  // going into the other (last read before the previous barrier).
  auto step = [&](auto buf, int c0) {
    constexpr int B = decltype(buf)::value;
    if (c0 + kCols64 < len)
      stage_async64<DP, 16 * NH, NW>(xu, xun, delta, L.n_pad, start, c0 + kCols64,
                                     &sx[B ^ 1][0][0], sn[B ^ 1], &sd[B ^ 1][0][0]);
    const int steps = std::min(kCols64, len - c0 + 3) / 4;
    for (int st = 0; st < steps; ++st) {
      const int jj = 4 * st + lg;
      double a[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) a[h] = sd[B][jj][16 * h + ln];
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[B][jj][k];
      const double nc = sn[B][jj];
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
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  for (int s2 = 0; s2 < nst; s2 += 2) {
    step(std::integral_constant<int, 0>{}, s2 * kCols64);
    if (s2 + 1 < nst) step(std::integral_constant<int, 1>{}, (s2 + 1) * kCols64);
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
__global__ __launch_bounds__(256) void k_fused_fp64v(
    Layout L, Params P, const double* __restrict__ xu, const double* __restrict__ xun,
    const double* __restrict__ delta, const Ctl* __restrict__ ctl, int block,
    float* __restrict__ R, float* __restrict__ rowsq, float* __restrict__ colsq, int want_rowsq,
    int want_colsq) {
  constexpr int NW = 4;
  constexpr int NQ = (NV + 3) / 4;  // output columns per lane
  __shared__ __attribute__((aligned(16))) double sx[2][kCols64][DP];
  __shared__ __attribute__((aligned(16))) double sn[2][kCols64];
  __shared__ __attribute__((aligned(16))) double sd[2][kCols64][NV];
  __shared__ float red[4][kMaxL];
  __shared__ double etab[kExpTab];  // s * 2^(j/256) for the exponential
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  scaled_exp_table(etab, P.s);  // visible after the first barrier
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 64;
  const int nst = (len + kCols64 - 1) / kCols64;

  stage_async64<DP, NV, NW>(xu, xun, delta, L.n_pad, start, 0, &sx[0][0][0], sn[0], &sd[0][0][0]);
  double xi[4][DV], ni[4];  // -2 u_i and |u_i|^2
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int k = 0; k < DV; ++k) xi[t][k] = -2.0 * xu[(row0 + 16 * t + ln) * DP + k];
    ni[t] = xun[row0 + 16 * t + ln];
  }
  double acc[4][NV];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[t][c] = 0.0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  auto step = [&](auto buf, int c0) {
    constexpr int B = decltype(buf)::value;
    if (c0 + kCols64 < len)
      stage_async64<DP, NV, NW>(xu, xun, delta, L.n_pad, start, c0 + kCols64, &sx[B ^ 1][0][0],
                                sn[B ^ 1], &sd[B ^ 1][0][0]);
    const int steps = std::min(kCols64, len - c0 + 3) / 4;
    for (int st = 0; st < steps; ++st) {
      const int jj = 4 * st + lg;
      double a[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) a[c] = sd[B][jj][c];
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[B][jj][k];
      const double nc = sn[B][jj];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double r2 = dist2n64<DV>(xi[t], ni[t], xc, nc);
        if constexpr (KERN != 0) r2 = fmax(r2, 0.0);
        const double kv = kernel_fp64<KERN>(r2, etab);
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[t][c] = fma(kv, a[c], acc[t][c]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  for (int s2 = 0; s2 < nst; s2 += 2) {
    step(std::integral_constant<int, 0>{}, s2 * kCols64);
    if (s2 + 1 < nst) step(std::integral_constant<int, 1>{}, (s2 + 1) * kCols64);
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
  hipLaunchKernelGGL((k_fused_fp64v<KERN, DV, DP, NV>), g, t, 0, st, L, P, D.xu, D.xun,      \
                     D.delta, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc)
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
  hipLaunchKernelGGL((k_fused_fp64<KERN, DV, DP, NH>), g, t, 0, st, L, P, D.xu, D.xun, D.delta, \
                     D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc)
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
