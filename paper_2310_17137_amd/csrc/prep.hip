// Workspace layout, feature preparation, Algorithm 1's initialization, block
// selection and the epoch-end residual check.
#include <algorithm>
#include <cmath>

#include "ap_internal.h"

namespace ap {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool make_layout(int64_t n, int32_t d, int32_t l, int32_t b, int32_t kernel, int32_t order,
                 int32_t tile, Layout* L) {
  if (n < 1 || d < 1 || d > kMaxD || l < 1 || l > kMaxL || b < 1 || b > 4096 || b > n ||
      n >= (int64_t(1) << 31))
    return false;
  Layout o{};
  o.n = n;
  o.d = d;
  o.l = l;
  o.b = b;
  o.m = (int32_t)((n + b - 1) / b);
  o.b_pad = (b + kT - 1) / kT * kT;
  o.last_len = (int32_t)(n - (int64_t)(o.m - 1) * b);
  o.kernel = kernel;
  o.order = order;
  o.tile = tile;
  o.ks = (3 * d + 6 + 15) / 16;
  o.dp = (d + 3) / 4 * 4;
  o.n_pad = (n + 32 + kRowsWG - 1) / kRowsWG * kRowsWG;
  o.nwg = (int32_t)(o.n_pad / kRowsWG);
  // the true residual's per-workgroup partials: at most one per 64 rows (its
  // workgroups cover 64 or 256 rows by n)
  o.nwg_res = (int32_t)((n + 63) / 64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  o.off_ctl = take(sizeof(Ctl));
  o.off_xs = take(tile == 0 || tile == 2 ? (size_t)o.n_pad * o.dp * sizeof(double) : 0);
  o.off_xn = take(tile == 0 || tile == 2 ? (size_t)o.n_pad * sizeof(double) : 0);
  // every mode: a handle may move to FP64 tiles (ap_set_tile, the solve's escalation)
  o.off_xu = take((size_t)o.n_pad * o.dp * sizeof(double));
  o.off_xun = take((size_t)o.n_pad * sizeof(double));
  o.off_xrow = take(tile == 1 ? (size_t)o.n_pad * 16 * o.ks * 2 : 0);
  o.off_xcol = take(tile == 1 ? (size_t)o.n_pad * 16 * o.ks * 2 : 0);
  o.off_kinv = take((size_t)o.m * o.b_pad * o.b_pad * sizeof(double));
  o.off_dinv = take((size_t)o.m * o.b_pad * kT * sizeof(double));
  o.off_panel = take((size_t)o.m * o.b_pad * kT * sizeof(double));
  o.off_delta = take((size_t)o.b_pad * kMaxL * sizeof(double));
  o.off_bspart = take((size_t)kBsSplit * o.b_pad * kMaxL * sizeof(double));
  o.off_dtile = take((size_t)o.b_pad * 2 * kMaxL * sizeof(float));
  o.off_rowsq = take((size_t)o.n_pad * sizeof(float));
  o.off_colsq = take((size_t)o.nwg * kMaxL * sizeof(float));
  o.off_blocknorm = take((size_t)o.m * sizeof(double));
  o.off_respart = take((size_t)std::max(o.nwg_res, 1024) * kMaxL * sizeof(double));
  o.off_mupart = take((size_t)256 * kMaxD * sizeof(double));
  o.off_desc = take(sizeof(Desc));
  o.nwg_mll = (int32_t)((n + 63) / 64);
  o.off_gpart = take((size_t)o.nwg_mll * (kMaxD + 2) * sizeof(double));
  o.total = off;
  *L = o;
  return true;
}

Dev bind(const Layout& L, void* ws) {
  char* base = (char*)ws;
  Dev D;
  D.ctl = (Ctl*)(base + L.off_ctl);
  D.xv = (double*)(base + L.off_xs);
  D.xn = (double*)(base + L.off_xn);
  D.xu = (double*)(base + L.off_xu);
  D.xun = (double*)(base + L.off_xun);
  D.xrow = (uint16_t*)(base + L.off_xrow);
  D.xcol = (uint16_t*)(base + L.off_xcol);
  D.kinv = (double*)(base + L.off_kinv);
  D.dinv = (double*)(base + L.off_dinv);
  D.panel = (double*)(base + L.off_panel);
  D.delta = (double*)(base + L.off_delta);
  D.bspart = (double*)(base + L.off_bspart);
  D.dtile = (void*)(base + L.off_dtile);
  D.rowsq = (float*)(base + L.off_rowsq);
  D.colsq = (float*)(base + L.off_colsq);
  D.blocknorm = (double*)(base + L.off_blocknorm);
  D.respart = (double*)(base + L.off_respart);
  D.mupart = (double*)(base + L.off_mupart);
  D.gpart = (double*)(base + L.off_gpart);
  return D;
}

namespace {

// Round to nearest even BF16 (finite inputs).
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline double feat_scale(int kernel) {
  if (kernel == 0) return sqrt(0.5 * kLog2e);
  if (kernel == 1) return 1.7320508075688772 * kLog2e;
  return 2.23606797749979 * kLog2e;
}

// Column sums of X in FP64: 256 workgroups, one strided slice each.
__global__ __launch_bounds__(256) void k_mu_partial(Layout L, const float* __restrict__ X,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  for (int k = 0; k < L.d; ++k) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < L.n; i += 256 * 256)
      acc += (double)X[i * L.d + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * kMaxD + k] = red[0];
    __syncthreads();
  }
}

__global__ void k_mu_final(Layout L, const double* __restrict__ part, Ctl* ctl) {
  int k = threadIdx.x;
  if (k < L.d) {
    double acc = 0.0;
    for (int g = 0; g < 256; ++g) acc += part[g * kMaxD + k];
    ctl->mu[k] = acc / (double)L.n;
  }
  if (k == 0) {
    ctl->fail = ~0ull;
    ctl->status = 0;
    ctl->sel = 0;
    ctl->epoch = 0;
    ctl->rho = 0.0;
    ctl->rho_true = 0.0;
    ctl->cursor = 0;
    ctl->state = 0;
    ctl->run = 1;
    ctl->next_refine = 0;
    // random order: the first block is draw 0
    ctl->draws = L.order == 2 ? 1ull : 0ull;
    if (L.order == 2) ctl->sel = random_block(L.seed, 0ull, L.m);
  }
}

// Prepared copies of the features (one thread per row). Every mode: the FP64
// tiles' u = (x - mu) / ell and |u|^2 (summed in feature order with FMAs), the
// values the FP64-tile update stages. Then v = u * c by mode. FP32 and split
// paths: xv[i] = v in FP64, differenced and squared in FP64 by
// the fused update, and xn[i] = |v|^2 summed in feature order with FMAs (the
// order of the fused update's own norms). BF16 path: v = vh + vl (two BF16 terms), |v|^2 = nh + nm + nl
// (three BF16 terms), and the row / column operands
//   row: [vh, vh, vl, -nh, -nm, -nl, 1, 1, 1, 0...]
//   col: [2vh, 2vl, 2vh, 1, 1, 1, -nh, -nm, -nl, 0...]
// whose dot product is 2 v_i.v_j - |v_i|^2 - |v_j|^2 = -|v_i - v_j|^2 (the
// vl_i.vl_j term dropped). Padding rows (i >= n) are zero.
__global__ __launch_bounds__(256) void k_prep(Layout L, Params P, const float* __restrict__ X,
                                              const Ctl* __restrict__ ctl, double* __restrict__ xv,
                                              double* __restrict__ xn, double* __restrict__ xu,
                                              double* __restrict__ xun,
                                              uint16_t* __restrict__ xrow,
                                              uint16_t* __restrict__ xcol) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= L.n_pad) return;
  const double c = feat_scale(L.kernel);
  const int d = L.d;
  {
    double a = 0.0;
    for (int k = 0; k < L.dp; ++k) {
      double u = 0.0;
      if (i < L.n && k < d) u = ((double)X[i * d + k] - ctl->mu[k]) / P.ell[k];
      xu[i * L.dp + k] = u;
      a = fma(u, u, a);
    }
    xun[i] = a;
  }
  if (L.tile == 0 || L.tile == 2) {
    double a = 0.0;
    for (int k = 0; k < L.dp; ++k) {
      double v = 0.0;
      if (i < L.n && k < d) v = ((double)X[i * d + k] - ctl->mu[k]) / P.ell[k] * c;
      xv[i * L.dp + k] = v;
      a = fma(v, v, a);
    }
    xn[i] = a;
    return;
  }
  if (L.tile != 1) return;  // the FP64-tile path stages xu
  const int kf = 16 * L.ks;
  uint16_t* r = xrow + i * kf;
  uint16_t* q = xcol + i * kf;
  for (int k = 0; k < kf; ++k) {
    r[k] = 0;
    q[k] = 0;
  }
  if (i >= L.n) return;
  const uint16_t one = to_bf16(1.0f);
  double nrm = 0.0;
  for (int k = 0; k < d; ++k) {
    double v = ((double)X[i * d + k] - ctl->mu[k]) / P.ell[k] * c;
    uint16_t hi = to_bf16((float)v);
    double vh = (double)from_bf16(hi);
    uint16_t lo = to_bf16((float)(v - vh));
    double vl = (double)from_bf16(lo);
    double vv = vh + vl;
    nrm += vv * vv;
    uint16_t hi2 = to_bf16(2.0f * from_bf16(hi));
    uint16_t lo2 = to_bf16(2.0f * from_bf16(lo));
    r[k] = hi;
    r[d + k] = hi;
    r[2 * d + k] = lo;
    q[k] = hi2;
    q[d + k] = lo2;
    q[2 * d + k] = hi2;
  }
  uint16_t nh = to_bf16((float)nrm);
  double rem = nrm - (double)from_bf16(nh);
  uint16_t nm = to_bf16((float)rem);
  rem -= (double)from_bf16(nm);
  uint16_t nl = to_bf16((float)rem);
  const int o = 3 * d;
  r[o + 0] = nh ^ 0x8000;
  r[o + 1] = nm ^ 0x8000;
  r[o + 2] = nl ^ 0x8000;
  r[o + 3] = one;
  r[o + 4] = one;
  r[o + 5] = one;
  q[o + 0] = one;
  q[o + 1] = one;
  q[o + 2] = one;
  q[o + 3] = nh ^ 0x8000;
  q[o + 4] = nm ^ 0x8000;
  q[o + 5] = nl ^ 0x8000;
}

// W = 0, R = B (Algorithm 1 initialization), per-row sums of squares of B, and
// per-workgroup FP64 column partials of ||B_c||^2. With R == nullptr only the
// column partials are formed (W, R and rowsq untouched).
__global__ __launch_bounds__(256) void k_reset(Layout L, const float* __restrict__ B,
                                               double* __restrict__ W, float* __restrict__ R,
                                               float* __restrict__ rowsq,
                                               double* __restrict__ part, int keep_w) {
  __shared__ double red[256 * 2];
  const int l = L.l;
  const bool write = R != nullptr;
  double col[kMaxL];
  for (int c = 0; c < kMaxL; ++c) col[c] = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < L.n_pad; i += (int64_t)gridDim.x * 256) {
    float rs = 0.f;
    if (i < L.n) {
      for (int c = 0; c < l; ++c) {
        float v = B[i * l + c];
        if (write) {
          R[i * l + c] = v;
          if (!keep_w) W[i * l + c] = 0.0;
        }
        rs = fmaf(v, v, rs);
        col[c] += (double)v * (double)v;
      }
    }
    if (write) rowsq[i] = rs;
  }
  for (int c = 0; c < l; ++c) {
    red[threadIdx.x] = col[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * kMaxL + c] = red[0];
    __syncthreads();
  }
}

__global__ void k_reset_final(Layout L, const double* __restrict__ part, int groups, Ctl* ctl) {
  int c = threadIdx.x;
  if (c < L.l) {
    double acc = 0.0;
    for (int g = 0; g < groups; ++g) acc += part[g * kMaxL + c];
    ctl->bnorm2[c] = acc;
  }
  if (c == 0) {
    ctl->status = 0;
    ctl->sel = 0;
    ctl->epoch = 0;
    ctl->rho = 1.0;
    ctl->cursor = 0;
    ctl->state = 0;
    ctl->run = 1;
    ctl->next_refine = 0;
    // random order: the first block is draw 0
    ctl->draws = L.order == 2 ? 1ull : 0ull;
    if (L.order == 2) ctl->sel = random_block(L.seed, 0ull, L.m);
  }
}

// ||R_I||_F^2 for every block from the per-row sums of squares (one workgroup
// per block, fixed reduction order).
__device__ __forceinline__ void block_norm_body(const Layout& L, const float* __restrict__ rowsq,
                                                double* __restrict__ out, int64_t j) {
  __shared__ double red[256];
  const int64_t s = j * L.b;
  const int64_t e = std::min<int64_t>(s + L.b, L.n);
  double acc = 0.0;
  for (int64_t i = s + threadIdx.x; i < e; i += 256) acc += (double)rowsq[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

__global__ __launch_bounds__(256) void k_block_norms(Layout L, const float* __restrict__ rowsq,
                                                     double* __restrict__ out) {
  block_norm_body(L, rowsq, out, blockIdx.x);
}

// Modified Gauss-Southwell rule: argmax over blocks, ties to the lowest index.
// A NaN norm is never selected. If no block has a norm that compares (every
// one NaN), block 0 is taken and the status word marks the residual as not
// finite, so the selection is always a valid block and the host sees the
// failure at the epoch-end check.
__device__ __forceinline__ void argmax_body(const Layout& L, const double* __restrict__ nrm,
                                            Ctl* ctl) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int idx = -1;
  for (int j = threadIdx.x; j < L.m; j += 256) {
    double v = nrm[j];
    if (v > best) {
      best = v;
      idx = j;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double v2 = bv[threadIdx.x + s];
      int i2 = bi[threadIdx.x + s];
      if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (bi[0] >= 0 && bi[0] < L.m) {
      ctl->sel = bi[0];
    } else {
      ctl->sel = 0;
      ctl->status = -3;
    }
  }
}

__global__ __launch_bounds__(256) void k_argmax(Layout L, const double* __restrict__ nrm,
                                                Ctl* ctl) {
  argmax_body(L, nrm, ctl);
}

// Grouped selection of a batch step for the greedy problems: one workgroup per
// block of each problem, then one per problem for the argmax.
__global__ __launch_bounds__(256) void g_block_norms(Group g) {
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  const Layout L = ds->L;
  block_norm_body(L, ds->D.rowsq, ds->D.blocknorm, wg);
}

__global__ __launch_bounds__(256) void g_argmax(Group g) {
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  const Layout L = ds->L;
  argmax_body(L, ds->D.blocknorm, ds->D.ctl);
}

// Random order: the block of the next update, draw ctl->draws of the
// problem's sequence. In a batch step only a problem whose update ran draws,
// so its sequence does not depend on when it was held.
__device__ __forceinline__ void random_sel_body(const Layout& L, Ctl* ctl) {
  if (threadIdx.x == 0) {
    const unsigned long long u = ctl->draws;
    ctl->sel = random_block(L.seed, u, L.m);
    ctl->draws = u + 1ull;
  }
}

__global__ void k_random_sel(Layout L, Ctl* ctl) { random_sel_body(L, ctl); }

__global__ void g_random_sel(Group g) {
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  Ctl* ctl = ds->D.ctl;
  if (ctl->run) random_sel_body(ds->L, ctl);
}

// Epoch-end check (Section 5, "Alternating Projection Details"): column norms
// of R from the fused update's per-workgroup partials, in a fixed order, then
// rho = mean_c ||r_c|| / ||b_c||.
__device__ __forceinline__ void epoch_check_body(const Layout& L, const float* __restrict__ colsq,
                                                 Ctl* ctl) {
  __shared__ double red[256];
  __shared__ double ratio[kMaxL];
  for (int c = 0; c < L.l; ++c) {
    double acc = 0.0;
    for (int g = threadIdx.x; g < L.nwg; g += 256) acc += (double)colsq[g * kMaxL + c];
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
      ctl->colrel[c] = r;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int c = 0; c < L.l; ++c) acc += ratio[c];
    double rho = acc / L.l;
    ctl->rho = rho;
    ctl->epoch += 1;
    if (!isfinite(rho)) ctl->status = -3;
  }
}

__global__ __launch_bounds__(256) void k_epoch_check(Layout L, const float* __restrict__ colsq,
                                                     Ctl* ctl) {
  epoch_check_body(L, colsq, ctl);
}

// Batch step epilogue, one workgroup per problem of the group: a problem that
// updated in this step advances its cursor; after the last block of an epoch
// the epoch-end check runs and the problem is held when the host has to act:
// the ratio is not finite, it is below the tolerance (with at least
// min_epochs epochs), max_epochs is reached, or an FP64 true residual is due
// every refine_every epochs. The run flag of the next step is latched here, so
// a problem is either updated through a whole step or not at all.
__global__ __launch_bounds__(256) void g_advance(Group g) {
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  Ctl* ctl = ds->D.ctl;
  const Layout L = ds->L;
  const int ran = ctl->run;
  const int cur = ctl->cursor + 1;
  __syncthreads();  // every thread holds run and cursor before thread 0 rewrites them
  if (ran) {
    if (cur == L.m) {
      epoch_check_body(L, ds->D.colsq, ctl);
      __syncthreads();
      if (threadIdx.x == 0) {
        const int ep = ctl->epoch;
        const double rho = ctl->rho;
        int state = 0;
        if (ctl->status != 0 || !isfinite(rho))
          state = 4;
        else if (rho < ds->tol && ep >= ds->min_epochs)
          state = 2;
        else if (ep >= ds->max_epochs)
          state = 3;
        else if (ctl->next_refine > 0 ? ep >= ctl->next_refine
                                       : ds->refine_every > 0 && ep % ds->refine_every == 0)
          state = 1;
        ctl->cursor = 0;
        ctl->state = state;
      }
    } else if (threadIdx.x == 0) {
      ctl->cursor = cur;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    ctl->run = ctl->state == 0 ? 1 : 0;
  }
}

// The host has acted on a held problem: it updates again from the next step,
// with the next true-residual hold at epoch next_refine (0: the schedule).
__global__ void k_release(Ctl* ctl, int next_refine) {
  if (threadIdx.x == 0) {
    ctl->state = 0;
    ctl->status = 0;
    ctl->run = 1;
    ctl->next_refine = next_refine;
  }
}

}  // namespace

hipError_t launch_prep(const Layout& L, const Dev& D, const Params& P, const float* X,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_mu_partial, dim3(256), dim3(256), 0, st, L, X, D.mupart);
  hipLaunchKernelGGL(k_mu_final, dim3(1), dim3(64), 0, st, L, D.mupart, D.ctl);
  unsigned g = (unsigned)((L.n_pad + 255) / 256);
  hipLaunchKernelGGL(k_prep, dim3(g), dim3(256), 0, st, L, P, X, D.ctl, D.xv, D.xn, D.xu, D.xun,
                     D.xrow, D.xcol);
  return hipGetLastError();
}

hipError_t launch_reset(const Layout& L, const Dev& D, const float* B, double* W, float* R,
                        bool keep_w, hipStream_t st) {
  const int groups = kResetGroups;
  hipLaunchKernelGGL(k_reset, dim3(groups), dim3(256), 0, st, L, B, W, R, D.rowsq, D.respart,
                     (int)keep_w);
  hipLaunchKernelGGL(k_reset_final, dim3(1), dim3(64), 0, st, L, D.respart, groups, D.ctl);
  if (L.order == 1) return launch_select(L, D, st);
  return hipGetLastError();
}

hipError_t launch_bnorm(const Layout& L, const Dev& D, const float* B, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(kResetGroups), dim3(256), 0, st, L, B, nullptr, nullptr,
                     nullptr, D.respart, 0);
  hipLaunchKernelGGL(k_reset_final, dim3(1), dim3(64), 0, st, L, D.respart, kResetGroups, D.ctl);
  return hipGetLastError();
}

hipError_t launch_select(const Layout& L, const Dev& D, hipStream_t st) {
  hipLaunchKernelGGL(k_block_norms, dim3(L.m), dim3(256), 0, st, L, D.rowsq, D.blocknorm);
  hipLaunchKernelGGL(k_argmax, dim3(1), dim3(256), 0, st, L, D.blocknorm, D.ctl);
  return hipGetLastError();
}

hipError_t launch_random_select(const Layout& L, const Dev& D, hipStream_t st) {
  hipLaunchKernelGGL(k_random_sel, dim3(1), dim3(64), 0, st, L, D.ctl);
  return hipGetLastError();
}

hipError_t launch_group_random(const Group& g, hipStream_t st) {
  hipLaunchKernelGGL(g_random_sel, dim3(g.count), dim3(64), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_group_select(const Group& gn, const Group& ga, hipStream_t st) {
  hipLaunchKernelGGL(g_block_norms, dim3(gn.wg0[gn.count]), dim3(256), 0, st, gn);
  hipLaunchKernelGGL(g_argmax, dim3(ga.count), dim3(256), 0, st, ga);
  return hipGetLastError();
}

hipError_t launch_group_advance(const Group& g, hipStream_t st) {
  hipLaunchKernelGGL(g_advance, dim3(g.count), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_release(const Dev& D, int32_t next_refine, hipStream_t st) {
  hipLaunchKernelGGL(k_release, dim3(1), dim3(64), 0, st, D.ctl, next_refine);
  return hipGetLastError();
}

hipError_t launch_epoch_check(const Layout& L, const Dev& D, hipStream_t st) {
  hipLaunchKernelGGL(k_epoch_check, dim3(1), dim3(256), 0, st, L, D.colsq, D.ctl);
  return hipGetLastError();
}

}  // namespace ap
