// FP64 block solve of Algorithm 1's weight update (eq. text_update_of_w):
//   delta = K^_{I,I}^{-1} R_I,  W_I += delta,
// with the cached inverse, so the solve is one FP64 product of a b x b matrix
// with the b x l block of the residual. The step is also written, times the
// outputscale, in the operand layout of the fused residual update: FP32, one
// BF16 term, or three BF16 terms (h + m + l) for the split path.
#include <algorithm>

#include "ap_internal.h"

namespace ap {
namespace {

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Partial products over one of kBsSplit slices of the block columns q.
// Workgroup: 64 output rows (one per lane) x LB >= l columns; the 4 waves take
// interleaved quarters of the slice. The inverse is read along rows of its
// symmetric storage, K^-1[q][i] = K^-1[i][q], so the 64 lanes of a wave read
// 512 contiguous bytes per q; R_I is staged once per slice in LDS as FP64.
constexpr int kSlice = 4096 / kBsSplit;  // largest slice (b_pad <= 4096)
template <int LB>
constexpr int bs_smem() {
  return kSlice * LB > 4 * 64 * LB ? kSlice * LB : 4 * 64 * LB;
}

template <int LB>
__device__ __forceinline__ void bs_partial_body(const Layout& L, const double* __restrict__ kinv,
                                                int blk, const float* __restrict__ R,
                                                double* __restrict__ part, int wg,
                                                double* smem) {
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int l = L.l;
  const int ntile = L.b_pad / 64;
  const int it = wg % ntile, sp = wg / ntile;
  const int slice = L.b_pad / kBsSplit;  // multiple of 4
  const int q0 = sp * slice;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = it * 64 + lane;
  const double* K = kinv + (size_t)blk * L.b_pad * L.b_pad;
  for (int e = threadIdx.x; e < slice * LB; e += 256) {
    int qq = e / LB, c = e % LB;
    int q = q0 + qq;
    smem[e] = (q < len && c < l) ? (double)R[(start + q) * l + c] : 0.0;
  }
  __syncthreads();
  double acc[LB];
#pragma unroll
  for (int c = 0; c < LB; ++c) acc[c] = 0.0;
  // The wave's rows q of the inverse in batches of kBsAhead: the batch's loads
  // are issued together (one at a time, each would wait out the memory latency)
  // and the sum keeps its q order. The empty asm keeps each q's LDS reads after
  // the previous q's, so the batch does not hold every staged row in registers.
  constexpr int kBsAhead = 8;
  for (int qb = wave; qb < slice; qb += 4 * kBsAhead) {
    double kv[kBsAhead];
#pragma unroll
    for (int j = 0; j < kBsAhead; ++j) {
      const int qq = qb + 4 * j;
      kv[j] = qq < slice ? K[(size_t)(q0 + qq) * L.b_pad + i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kBsAhead; ++j) {
      const int qq = qb + 4 * j;
      if (qq < slice) {
        asm volatile("" ::: "memory");
        const double* rq = smem + qq * LB;
#pragma unroll
        for (int c = 0; c < LB; ++c) acc[c] = fma(kv[j], rq[c], acc[c]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < LB; ++c) smem[(wave * 64 + lane) * LB + c] = acc[c];
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * kMaxL; e += 256) {
    int r = e / kMaxL, c = e % kMaxL;
    double v = 0.0;
    if (c < LB)
      v = ((smem[(0 * 64 + r) * LB + c] + smem[(1 * 64 + r) * LB + c]) +
           smem[(2 * 64 + r) * LB + c]) + smem[(3 * 64 + r) * LB + c];
    part[((size_t)sp * L.b_pad + it * 64 + r) * kMaxL + c] = v;
  }
}

template <int LB>
__global__ __launch_bounds__(256) void k_bs_partial(Layout L, const double* __restrict__ kinv,
                                                    const Ctl* __restrict__ ctl, int block,
                                                    const float* __restrict__ R,
                                                    double* __restrict__ part) {
  __shared__ double smem[bs_smem<LB>()];
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  bs_partial_body<LB>(L, kinv, blk, R, part, (int)blockIdx.x, smem);
}

// Sum the slices in a fixed order, update W_I, keep delta in FP64 and write
// s * delta in the fused update's operand layout (element e = i * 32 + c).
__device__ __forceinline__ void bs_finish_body(const Layout& L, int blk, int tile, double s,
                                               const double* __restrict__ part,
                                               double* __restrict__ W,
                                               double* __restrict__ delta, void* dtile, int e) {
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  if (e >= L.b_pad * kMaxL) return;
  const int i = e / kMaxL, c = e % kMaxL;
  double v = 0.0;
  if (i < len && c < L.l) {
    for (int sp = 0; sp < kBsSplit; ++sp) v += part[((size_t)sp * L.b_pad + i) * kMaxL + c];
    W[(start + i) * L.l + c] += v;
  }
  delta[i * kMaxL + c] = v;
  if (tile == 3) return;  // the FP64-tile update reads delta itself
  if (tile == 0) {
    ((float*)dtile)[i * kMaxL + c] = (float)(s * v);
    return;
  }
  // BF16 operand layout: bcol i of chunk ch sits in k-step st = w / 16 at
  // lane g * 32 + c, element el, where w = i % 32 = 16 st + 4 g + (el % 4) + 8 (el / 4)
  const int ch = i / 32, w = i % 32, st = w / 16, w2 = w % 16;
  const int g = (w2 % 8) / 4, el = (w2 / 8) * 4 + w2 % 4;
  const int lane = g * 32 + c;
  const size_t at = (((size_t)ch * 2 + st) * 64 + lane) * 8 + el;
  uint16_t* out = (uint16_t*)dtile;
  if (tile == 1) {
    out[at] = bf16_rne((float)(s * v));
    return;
  }
  // split path: s * delta = h + m + l, three BF16 terms (24 significant bits)
  const size_t term = (size_t)L.b_pad * kMaxL;
  const double sv = s * v;
  const uint16_t h = bf16_rne((float)sv);
  const double r1 = sv - (double)bf16_to_f32(h);
  const uint16_t m = bf16_rne((float)r1);
  const double r2 = r1 - (double)bf16_to_f32(m);
  out[at] = h;
  out[term + at] = m;
  out[2 * term + at] = bf16_rne((float)r2);
}

__global__ __launch_bounds__(256) void k_bs_finish(Layout L, const Ctl* __restrict__ ctl,
                                                   int block, double s,
                                                   const double* __restrict__ part,
                                                   double* __restrict__ W,
                                                   double* __restrict__ delta, void* dtile) {
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  bs_finish_body(L, blk, L.tile, s, part, W, delta, dtile, (int)blockIdx.x * 256 + threadIdx.x);
}

// Grouped forms for a batch step: every workgroup finds its problem in the
// group and runs the same bodies on that problem's block.
__device__ __forceinline__ int batch_code(const Layout& L) {
  return L.order != 0 ? kBlockBatchSel : kBlockBatchCyclic;
}

__global__ __launch_bounds__(256) void g_bs_partial(Group g) {
  __shared__ double smem[bs_smem<kMaxL>()];
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  const Layout L = ds->L;
  const int blk = resolve_block(batch_code(L), ds->D.ctl, L.m);
  if (blk < 0) return;
  const double* kinv = ds->D.kinv;
  double* part = ds->D.bspart;
  const float* R = g.R[p];
  if (L.l <= 1)
    bs_partial_body<1>(L, kinv, blk, R, part, wg, smem);
  else if (L.l <= 4)
    bs_partial_body<4>(L, kinv, blk, R, part, wg, smem);
  else if (L.l <= 8)
    bs_partial_body<8>(L, kinv, blk, R, part, wg, smem);
  else if (L.l <= 16)
    bs_partial_body<16>(L, kinv, blk, R, part, wg, smem);
  else
    bs_partial_body<32>(L, kinv, blk, R, part, wg, smem);
}

__global__ __launch_bounds__(256) void g_bs_finish(Group g) {
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  const Layout L = ds->L;
  const int blk = resolve_block(batch_code(L), ds->D.ctl, L.m);
  if (blk < 0) return;
  bs_finish_body(L, blk, g.tile[p], ds->P.s, ds->D.bspart, g.W[p], ds->D.delta, ds->D.dtile,
                 wg * 256 + threadIdx.x);
}

}  // namespace

hipError_t launch_block_solve(const Layout& L, const Dev& D, const Params& P, int32_t block,
                              const float* R, double* W, hipStream_t st) {
  const int ntile = L.b_pad / 64;
  const dim3 g(ntile * kBsSplit), t(256);
  if (L.l <= 1)
    hipLaunchKernelGGL(k_bs_partial<1>, g, t, 0, st, L, D.kinv, D.ctl, block, R, D.bspart);
  else if (L.l <= 4)
    hipLaunchKernelGGL(k_bs_partial<4>, g, t, 0, st, L, D.kinv, D.ctl, block, R, D.bspart);
  else if (L.l <= 8)
    hipLaunchKernelGGL(k_bs_partial<8>, g, t, 0, st, L, D.kinv, D.ctl, block, R, D.bspart);
  else if (L.l <= 16)
    hipLaunchKernelGGL(k_bs_partial<16>, g, t, 0, st, L, D.kinv, D.ctl, block, R, D.bspart);
  else
    hipLaunchKernelGGL(k_bs_partial<32>, g, t, 0, st, L, D.kinv, D.ctl, block, R, D.bspart);
  const int tot = L.b_pad * kMaxL;
  hipLaunchKernelGGL(k_bs_finish, dim3((tot + 255) / 256), dim3(256), 0, st, L, D.ctl, block,
                     P.s, D.bspart, W, D.delta, D.dtile);
  return hipGetLastError();
}

// gp: workgroups (b_pad / 64) kBsSplit per problem; gf: (32 b_pad) / 256.
hipError_t launch_group_solve(const Group& gp, const Group& gf, hipStream_t st) {
  hipLaunchKernelGGL(g_bs_partial, dim3(gp.wg0[gp.count]), dim3(256), 0, st, gp);
  hipLaunchKernelGGL(g_bs_finish, dim3(gf.wg0[gf.count]), dim3(256), 0, st, gf);
  return hipGetLastError();
}

}  // namespace ap
