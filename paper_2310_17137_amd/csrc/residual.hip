// FP64 true residual R = B - K^ W over all n^2 kernel entries (Lemma
// residual_equality: the maintained residual equals this in exact arithmetic,
// so recomputing it removes the drift of the reduced-precision update).
// Exact differencing of the FP32 inputs widened to FP64, FP64 kernel map, FP64
// accumulation in a fixed column order. One lane per row; the columns' features
// and weights are staged through LDS and read by all lanes at once.
#include <algorithm>

#include "ap_internal.h"

namespace ap {
namespace {

constexpr int kCols = 64;  // columns staged per step

template <int KERN, int LB>
__global__ __launch_bounds__(kResRows) void k_residual(Layout L, Params P,
                                                       const float* __restrict__ X,
                                                       const float* __restrict__ B,
                                                       const double* __restrict__ W,
                                                       float* __restrict__ Rout,
                                                       float* __restrict__ rowsq,
                                                       double* __restrict__ part) {
  __shared__ double sx[kCols][kMaxD];
  __shared__ double sw[kCols][LB];
  __shared__ double sq[LB][kResRows];
  const int d = L.d, l = L.l;
  const int64_t i = (int64_t)blockIdx.x * kResRows + threadIdx.x;
  const bool live = i < L.n;
  double inv_ell[kMaxD], xi[kMaxD];
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) {
    inv_ell[k] = k < d ? 1.0 / P.ell[k] : 0.0;
    xi[k] = (live && k < d) ? (double)X[i * d + k] : 0.0;
  }
  double acc[LB];
#pragma unroll
  for (int c = 0; c < LB; ++c) acc[c] = 0.0;
  for (int64_t j0 = 0; j0 < L.n; j0 += kCols) {
    const int cols = (int)std::min<int64_t>(kCols, L.n - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < kCols * kMaxD; e += kResRows) {
      int jj = e / kMaxD, k = e % kMaxD;
      sx[jj][k] = (jj < cols && k < d) ? (double)X[(j0 + jj) * d + k] : 0.0;
    }
    for (int e = threadIdx.x; e < kCols * LB; e += kResRows) {
      int jj = e / LB, c = e % LB;
      sw[jj][c] = (jj < cols && c < l) ? W[(j0 + jj) * l + c] : 0.0;
    }
    __syncthreads();
    for (int jj = 0; jj < cols; ++jj) {
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxD; ++k) {
        if (k < d) {
          double t = (xi[k] - sx[jj][k]) * inv_ell[k];
          r2 = fma(t, t, r2);
        }
      }
      double kv;
      if constexpr (KERN == 0) {
        kv = P.s * exp(-0.5 * r2);
      } else if constexpr (KERN == 1) {
        double t = 1.7320508075688772 * sqrt(r2);
        kv = P.s * (1.0 + t) * exp(-t);
      } else {
        double r = sqrt(r2), t = 2.23606797749979 * r;
        kv = P.s * (1.0 + t + (5.0 / 3.0) * r2) * exp(-t);
      }
      if (j0 + jj == i) kv += P.noise;
#pragma unroll
      for (int c = 0; c < LB; ++c) acc[c] = fma(kv, sw[jj][c], acc[c]);
    }
  }
  double rs = 0.0;
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    double r = 0.0;
    if (live && c < l) {
      r = (double)B[i * l + c] - acc[c];
      Rout[i * l + c] = (float)r;
      rs = fma(r, r, rs);
    }
    sq[c][threadIdx.x] = r * r;
  }
  if (rowsq && live) rowsq[i] = (float)rs;
  __syncthreads();
  for (int s = kResRows / 2; s > 0; s >>= 1) {
    for (int c = 0; c < LB; ++c)
      if (threadIdx.x < s) sq[c][threadIdx.x] += sq[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < kMaxL)
    part[(size_t)blockIdx.x * kMaxL + threadIdx.x] = threadIdx.x < LB ? sq[threadIdx.x][0] : 0.0;
}

__global__ __launch_bounds__(256) void k_residual_final(Layout L, const double* __restrict__ part,
                                                        Ctl* ctl) {
  __shared__ double red[256];
  __shared__ double ratio[kMaxL];
  for (int c = 0; c < L.l; ++c) {
    double acc = 0.0;
    for (int g = threadIdx.x; g < L.nwg_res; g += 256) acc += part[(size_t)g * kMaxL + c];
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

template <int KERN>
void launch_res_k(const Layout& L, const Dev& D, const Params& P, const float* X, const float* B,
                  const double* W, float* Rout, float* rowsq, hipStream_t st) {
  const dim3 g(L.nwg_res), t(kResRows);
  if (L.l <= 1)
    hipLaunchKernelGGL((k_residual<KERN, 1>), g, t, 0, st, L, P, X, B, W, Rout, rowsq, D.respart);
  else if (L.l <= 4)
    hipLaunchKernelGGL((k_residual<KERN, 4>), g, t, 0, st, L, P, X, B, W, Rout, rowsq, D.respart);
  else if (L.l <= 8)
    hipLaunchKernelGGL((k_residual<KERN, 8>), g, t, 0, st, L, P, X, B, W, Rout, rowsq, D.respart);
  else if (L.l <= 16)
    hipLaunchKernelGGL((k_residual<KERN, 16>), g, t, 0, st, L, P, X, B, W, Rout, rowsq, D.respart);
  else
    hipLaunchKernelGGL((k_residual<KERN, 32>), g, t, 0, st, L, P, X, B, W, Rout, rowsq, D.respart);
}

}  // namespace

hipError_t launch_residual(const Layout& L, const Dev& D, const Params& P, const float* X,
                           const float* B, const double* W, float* Rout, bool in_place,
                           hipStream_t st) {
  // refining in place keeps the greedy rule's row norms in step with R
  float* rowsq = in_place ? D.rowsq : nullptr;
  switch (L.kernel) {
    case 0: launch_res_k<0>(L, D, P, X, B, W, Rout, rowsq, st); break;
    case 1: launch_res_k<1>(L, D, P, X, B, W, Rout, rowsq, st); break;
    default: launch_res_k<2>(L, D, P, X, B, W, Rout, rowsq, st); break;
  }
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, L, D.respart, D.ctl);
  return hipGetLastError();
}

}  // namespace ap
