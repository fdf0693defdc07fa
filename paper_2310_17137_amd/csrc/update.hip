// Fused residual update of Algorithm 1 (eq. text_update_of_r):
//   R <- R - K^_{:,I} delta,   delta = K^_{I,I}^{-1} R_I,
// with K^_{:,I} evaluated tile by tile from the features and never stored.
// On the rows of I the update is exactly zero (K^_{I,I} K^_{I,I}^{-1} R_I = R_I),
// and those rows are written as 0. In the same pass the kernel reduces the new
// residual's per-row sums of squares (the block norms of the modified
// Gauss-Southwell rule, eq. approximate_gauss_southwell) and per-workgroup
// column sums of squares (the epoch-end stopping test).
//
// Every kernel here gives a workgroup 256 data rows and walks the block in
// chunks of 32 columns, adding each chunk's FP32 sums into FP64 accumulators.
// The tile modes differ in how a chunk's kernel values are formed and applied:
//  - FP32 tiles (k_fused_fp32, k_fused_fp32h, k_fused_fp32v): FP64 squared
//    distances on the vector units, the map in FP32, and the product with the
//    step on the FP32 matrix cores (32 or 16 right-hand sides) or, for l <= 8,
//    as vector FMAs;
//  - split tiles (k_fused_split): the same FP32 kernel values, with the tile
//    and the step each split into three BF16 terms for six BF16 products;
//  - BF16 tiles (k_fused_bf16): two 32 x 32 MFMA products per row tile,
//    S^T = X_chunk X_rows^T (x.x' on the BF16 matrix cores, then the map in
//    registers) and acc += delta_chunk^T K_tile^T. The transposed tile makes the
//    first product's accumulator layout (lane = data row, 16 chunk columns) the
//    second product's B operand, so the kernel values never leave registers.
#include <algorithm>
#include <type_traits>

#include "ap_internal.h"

namespace ap {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(16))) double f64x16;

constexpr float kInvLog2e = (float)(1.0 / kLog2e);                   // ln 2
constexpr float kInv3Log2e2 = (float)(1.0 / (3.0 * kLog2e * kLog2e));  // 1 / (3 log2(e)^2)

// Kernel map of the BF16 tiles on a = -|v_i - v_j|^2 as the matrix cores return
// it (FP32); only its magnitude enters the Matern maps.
template <int KERN>
__device__ __forceinline__ float kmap_neg(float a) {  // a = -|dv|^2
  if constexpr (KERN == 0) {
    return __builtin_amdgcn_exp2f(a);
  } else {
    float t = __builtin_amdgcn_sqrtf(fabsf(a));
    float e = __builtin_amdgcn_exp2f(-t);
    if constexpr (KERN == 1) return fmaf(t, kInvLog2e, 1.0f) * e;
    return fmaf(t, fmaf(t, kInv3Log2e2, kInvLog2e), 1.0f) * e;
  }
}

// Kernel map of the FP32 and split tiles: k/s from the FP64 squared distance a
// of the prepared features, in FP32 to within about 2 ulp for RBF and a few ulp
// for the Matern maps (half an ulp on average). The exponential runs
// on the FP32 unit from a_hi = fl32(a); the argument's rounding a_lo = a - a_hi
// enters to first order, 2^-(a_hi + a_lo) = 2^-a_hi (1 - a_lo ln 2). The
// Matern maps take t = sqrt(a) as t_hi = sqrt(a_hi) plus the correction
// k'(t_hi) (a - t_hi^2) / (2 t_hi), in which t_hi cancels:
//   Matern-3/2: k/s = (1 + t ln2) 2^-t,              k' = -t ln2^2 2^-t,
//   Matern-5/2: k/s = (1 + t ln2 + t^2 ln2^2/3) 2^-t, k' = -(t ln2^2/3)(1 + t ln2) 2^-t,
// so no division is needed and a = 0 (the diagonal, duplicate points) is exact.
template <int KERN>
__device__ __forceinline__ float kmap_acc(double a) {
  const float ah = (float)a;
  if constexpr (KERN == 0) {
    const float al = (float)(a - (double)ah);
    const float e = __builtin_amdgcn_exp2f(-ah);
    return fmaf(e, al * -kInvLog2e, e);
  } else {
    const float th = __builtin_amdgcn_sqrtf(fmaxf(ah, 0.0f));
    const double thd = (double)th;
    const float ea = (float)fma(-thd, thd, a);  // a - t_hi^2, exact in FP64
    const float e = __builtin_amdgcn_exp2f(-th);
    // k/s = 2^-t_hi (p(t_hi) + (a - t_hi^2) c(t_hi)), the correction's factor
    // c(t) = k'(t) / (2 t 2^-t) carrying its constants
    constexpr double kHalfLn2Sq = 0.5 / (kLog2e * kLog2e);
    if constexpr (KERN == 1) {
      const float p = fmaf(th, kInvLog2e, 1.0f);
      return fmaf(ea, (float)-kHalfLn2Sq, p) * e;
    } else {
      constexpr float kC0 = (float)(-kHalfLn2Sq / 3.0);
      constexpr float kC1 = (float)(-kHalfLn2Sq / (3.0 * kLog2e));
      const float p = fmaf(th, fmaf(th, kInv3Log2e2, kInvLog2e), 1.0f);
      return fmaf(ea, fmaf(th, kC1, kC0), p) * e;
    }
  }
}

// FP64 squared distance of a row's prepared features v_i (norm ni) to a staged
// column's v_j (norm nj), through the norm expansion |v_i|^2 + |v_j|^2 -
// 2 v_i.v_j with the row held as m2 = -2 v_i: d + 1 FP64 operations instead
// of 2d. The features are centred and scaled, so |v|^2 stays within a few
// hundred and the cancellation leaves an absolute error near 1e-13, far below
// the FP32 map's rounding; the Matern maps clamp the result at 0.
template <int DV>
__device__ __forceinline__ double dist2n(const double* m2, double ni, const double* xc, double nj) {
  double a = ni + nj;
#pragma unroll
  for (int k = 0; k < DV; ++k) a = fma(m2[k], xc[k], a);
  return a;
}

// The same by exact differencing (2d FP64 operations; the split tiles use it:
// there the expansion's extra registers cost more than its two operations).
template <int DV>
__device__ __forceinline__ double dist2(const double* xr, const double* xc) {
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < DV; ++k) {
    const double df = xr[k] - xc[k];
    a = fma(df, df, a);
  }
  return a;
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p) {
  uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ bf16x8 pack8(const f32x16& v, int base) {
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    f32x2 f = {v[base + e], v[base + e + 1]};
    bf16x2 h = __builtin_convertvector(f, bf16x2);
    r[e] = h[0];
    r[e + 1] = h[1];
  }
  return r;
}

// Epilogue of the 32-row tile kernels (RT row tiles per wave, NW waves).
// acc[t][v] holds, for data row row0 + 32 t + lane % 32, the update of column
// m = 8 (v / 4) + 4 (lane / 32) + v % 4.
template <int RT, int NW, typename Acc>
__device__ __forceinline__ void epilogue(const Layout& L, int64_t row0, int64_t start, int len,
                                         const Acc acc[RT], float* __restrict__ R,
                                         float* __restrict__ rowsq, float* __restrict__ colsq,
                                         bool want_rowsq, bool want_colsq, int wg) {
  __shared__ float red[NW][kMaxL];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int nl = lane % 32, g = lane / 32;
  const int l = L.l;
  float csum[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) csum[v] = 0.f;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = row0 + 32 * t + nl;
    const bool in_i = row >= start && row < start + len;
    const bool live = row < L.n;
    float rs = 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = 8 * (v / 4) + 4 * g + (v % 4);
      if (live && m < l) {
        float r = in_i ? 0.f : (float)(R[row * l + m] - acc[t][v]);
        R[row * l + m] = r;
        rs = fmaf(r, r, rs);
        csum[v] = fmaf(r, r, csum[v]);
      }
    }
    if (want_rowsq) {
      rs += __shfl_xor(rs, 32);
      if (g == 0 && row < L.n_pad) rowsq[row] = live ? rs : 0.f;
    }
  }
  if (want_colsq) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float x = csum[v];
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 8);
      x += __shfl_xor(x, 16);
      csum[v] = x;
    }
    if (nl == 0) {
#pragma unroll
      for (int v = 0; v < 16; ++v) red[wave][8 * (v / 4) + 4 * g + (v % 4)] = csum[v];
    }
    __syncthreads();
    if (threadIdx.x < kMaxL) {
      const int m = threadIdx.x;
      float s = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[w][m];
      colsq[(size_t)wg * kMaxL + m] = m < l ? s : 0.f;
    }
  }
}

// BF16 tiles: KS K-steps of 16 prepared feature slots (3d + 6 <= 16 KS).
template <int KERN, int KS>
__global__ __launch_bounds__(256) void k_fused_bf16(Layout L, const uint16_t* __restrict__ xrow,
                                                    const uint16_t* __restrict__ xcol,
                                                    const uint16_t* __restrict__ dtile,
                                                    const Ctl* __restrict__ ctl, int block,
                                                    float* __restrict__ R,
                                                    float* __restrict__ rowsq,
                                                    float* __restrict__ colsq, int want_rowsq,
                                                    int want_colsq) {
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int nch = (len + kChunk - 1) / kChunk;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int nl = lane % 32, g = lane / 32;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 64;
  constexpr int KF = 16 * KS;

  bf16x8 brow[2][KS];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      brow[t][ks] = load_bf16x8(xrow + (row0 + 32 * t + nl) * KF + 16 * ks + 8 * g);

  f32x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;

  for (int ch = 0; ch < nch; ++ch) {
    const int64_t cb = start + (int64_t)ch * kChunk;
    bf16x8 acol[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) acol[ks] = load_bf16x8(xcol + (cb + nl) * KF + 16 * ks + 8 * g);
    const bf16x8 d0 = load_bf16x8(dtile + (((size_t)ch * 2 + 0) * 64 + lane) * 8);
    const bf16x8 d1 = load_bf16x8(dtile + (((size_t)ch * 2 + 1) * 64 + lane) * 8);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x16 s;
#pragma unroll
      for (int v = 0; v < 16; ++v) s[v] = 0.f;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        s = __builtin_amdgcn_mfma_f32_32x32x16_bf16(acol[ks], brow[t][ks], s, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) s[v] = kmap_neg<KERN>(s[v]);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(d0, pack8(s, 0), acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(d1, pack8(s, 8), acc[t], 0, 0, 0);
    }
  }
  epilogue<2, 4>(L, row0, start, len, acc, R, rowsq, colsq, want_rowsq, want_colsq, (int)blockIdx.x);
}

// Asynchronous staging of one chunk (block columns cb .. cb + 31) for the FP32
// tile kernels: the columns' prepared features v_j (kChunk x DP doubles), their
// norms |v_j|^2 and the first NS columns of the step's rows (kChunk x NS
// floats) are copied from global memory straight into LDS with global_load_lds
// (each lane moves 16 or 4 bytes to base + lane * size; no registers are
// held). A wave-load moves 1 KiB; the waves take them in turn. The caller
// waits for the copies (s_waitcnt) and crosses a barrier before reading.
template <int DP, int NS, int NW>
__device__ __forceinline__ void stage_async(const double* __restrict__ xv,
                                            const double* __restrict__ xn,
                                            const float* __restrict__ dtile, int64_t start,
                                            int ch, double* sx, double* sn, float* sd) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t cb = start + (int64_t)ch * kChunk;
  const float* d0 = dtile + (int64_t)ch * kChunk * kMaxL;
  if constexpr (NS >= 4) {  // step rows in 16-byte pieces, QR per row
    constexpr int QR = NS / 4, NP = kChunk * QR;
    for (int q = wave; 64 * q < NP; q += NW) {
      const int pc = 64 * q + lane;
      if (pc < NP)
        __builtin_amdgcn_global_load_lds(d0 + (pc / QR) * kMaxL + 4 * (pc % QR), sd + 256 * q, 16,
                                         0, 0);
    }
  } else {  // one or two values per row: 4-byte pieces, one wave-load
    if (wave == 0 && lane < kChunk * NS)
      __builtin_amdgcn_global_load_lds(d0 + (lane / NS) * kMaxL + lane % NS, sd, 4, 0, 0);
  }
  for (int q = wave; q < kChunk * DP / 128; q += NW)
    __builtin_amdgcn_global_load_lds(xv + cb * DP + 128 * q + 2 * lane, sx + 128 * q, 16, 0, 0);
  if (wave == NW - 1)  // 32 norms as 64 dwords: 4-byte copies keep odd cb aligned
    __builtin_amdgcn_global_load_lds((const uint32_t*)(xn + cb) + lane, sn, 4, 0, 0);
}

// FP32 tiles: the prepared features in FP64, the squared distance in FP64, the
// kernel map in FP32 (kmap_acc, within a few ulp), and the product with the
// step on v_mfma_f32_32x32x2f32 (one kernel value per lane per step). Each
// chunk's column features, norms and step rows are staged in LDS, double-
// buffered: chunk c + 1 is copied into one buffer while chunk c is computed
// from the other, with one barrier per chunk. The rows are held as -2 v_i and
// the columns as v_j: the products equal v_i . (-2 v_j) exactly.
template <int KERN, int DV, int DP, int RT>
__global__ __launch_bounds__(kRowsWG / (32 * RT) * 64) void k_fused_fp32(
    Layout L, const double* __restrict__ xv, const double* __restrict__ xn,
    const float* __restrict__ dtile, const Ctl* __restrict__ ctl, int block,
    float* __restrict__ R, float* __restrict__ rowsq, float* __restrict__ colsq, int want_rowsq,
    int want_colsq) {
  constexpr int NW = kRowsWG / (32 * RT);  // waves of the workgroup
  __shared__ __attribute__((aligned(16))) double sx[2][kChunk][DP];
  __shared__ __attribute__((aligned(16))) double sn[2][kChunk];
  __shared__ __attribute__((aligned(16))) float sd[2][kChunk][kMaxL];
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int nch = (len + kChunk - 1) / kChunk;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int nl = lane % 32, g = lane / 32;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 32 * RT;

  stage_async<DP, kMaxL, NW>(xv, xn, dtile, start, 0, &sx[0][0][0], sn[0], &sd[0][0][0]);
  double xr[RT][DV], nr[RT];  // -2 v_i and |v_i|^2
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int k = 0; k < DV; ++k) xr[t][k] = -2.0 * xv[(row0 + 32 * t + nl) * DP + k];
    nr[t] = xn[row0 + 32 * t + nl];
  }
  // The products of a pair of chunks (64 columns) accumulate in FP32 on the
  // matrix cores; the pair sums then accumulate in FP64, so the rounding of the
  // long sum over the block stays at the level of 64 products. (Pairs rather
  // than single chunks halve the FP64 additions and their conversions.)
  f64x16 acc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // One chunk from buffer B (a compile-time constant, so that the LDS reads
  // keep immediate offsets), the next chunk's copies going into the other.
  f32x16 part[RT];  // FP32 sums of the current chunk pair (even ch, then ch + 1)
  auto chunk = [&](auto buf, int ch) {
    constexpr int B = decltype(buf)::value;
    // the other buffer was last read before the previous barrier
    if (ch + 1 < nch)
      stage_async<DP, kMaxL, NW>(xv, xn, dtile, start, ch + 1, &sx[B ^ 1][0][0], sn[B ^ 1],
                                 &sd[B ^ 1][0][0]);
    if constexpr (B == 0) {  // even chunks (buffer 0) open a pair
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) part[t][v] = 0.f;
    }
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int cc = 2 * st + g;  // this lane's chunk column
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[B][cc][k];
      const double nc = sn[B][cc];
      const float dv = sd[B][cc][nl];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const float kv = kmap_acc<KERN>(dist2n<DV>(xr[t], nr[t], xc, nc));
        part[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(dv, kv, part[t], 0, 0, 0);
      }
    }
    if (B == 1 || ch + 1 >= nch) {  // odd chunks, and a last even one, close it
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][v] += (double)part[t][v];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  for (int ch = 0; ch < nch; ch += 2) {
    chunk(std::integral_constant<int, 0>{}, ch);
    if (ch + 1 < nch) chunk(std::integral_constant<int, 1>{}, ch + 1);
  }
  epilogue<RT, NW>(L, row0, start, len, acc, R, rowsq, colsq, want_rowsq, want_colsq,
                   (int)blockIdx.x);
}

// FP32 tiles with 8 < l <= 16: the product on v_mfma_f32_16x16x4f32, whose 16
// right-hand sides cover l where the 32-row tile of k_fused_fp32 would leave half
// its multiply-adds idle (and the FP32 matrix instructions do not overlap the
// vector work of the kernel map, so idle matrix cycles are lost cycles). A wave
// owns RT 16-row tiles (the workgroup's 256 rows over 256 / (16 RT) waves); per
// step of 4 chunk columns a lane evaluates one kernel value per row tile (row
// lane % 16, column lane / 16) and the matrix cores accumulate
// part[r][i] += delta^T[r][j] K^T[j][i]. FP32 sums per chunk, FP64 across chunks.
template <int KERN, int DV, int DP, int RT>
__global__ __launch_bounds__(kRowsWG / (16 * RT) * 64) void k_fused_fp32h(
    Layout L, const double* __restrict__ xv, const double* __restrict__ xn,
    const float* __restrict__ dtile, const Ctl* __restrict__ ctl, int block,
    float* __restrict__ R, float* __restrict__ rowsq, float* __restrict__ colsq, int want_rowsq,
    int want_colsq) {
  constexpr int NH = 16;                     // right-hand sides of the tile
  constexpr int NW = kRowsWG / (16 * RT);    // waves of the workgroup
  __shared__ __attribute__((aligned(16))) double sx[2][kChunk][DP];
  __shared__ __attribute__((aligned(16))) double sn[2][kChunk];
  __shared__ __attribute__((aligned(16))) float sd[2][kChunk][NH];
  __shared__ float red[NW][NH];
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int nch = (len + kChunk - 1) / kChunk;
  const int l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int ln = lane % 16, lg = lane / 16;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * 16 * RT;

  stage_async<DP, NH, NW>(xv, xn, dtile, start, 0, &sx[0][0][0], sn[0], &sd[0][0][0]);
  double xr[RT][DV], nr[RT];  // -2 v_i and |v_i|^2
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int k = 0; k < DV; ++k) xr[t][k] = -2.0 * xv[(row0 + 16 * t + ln) * DP + k];
    nr[t] = xn[row0 + 16 * t + ln];
  }
  double acc[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = 0.0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // One chunk from buffer B (a compile-time constant), the next chunk's copies
  // going into the other, as in k_fused_fp32.
  auto chunk = [&](auto buf, int ch) {
    constexpr int B = decltype(buf)::value;
    if (ch + 1 < nch)
      stage_async<DP, NH, NW>(xv, xn, dtile, start, ch + 1, &sx[B ^ 1][0][0], sn[B ^ 1],
                              &sd[B ^ 1][0][0]);
    f32x4 part[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) part[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < kChunk / 4; ++st) {
      const int jj = 4 * st + lg;  // this lane's chunk column
      double xc[DV];
#pragma unroll
      for (int k = 0; k < DV; ++k) xc[k] = sx[B][jj][k];
      const double nc = sn[B][jj];
      const float dv = sd[B][jj][ln];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const float kv = kmap_acc<KERN>(dist2n<DV>(xr[t], nr[t], xc, nc));
        part[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(dv, kv, part[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[t][q] += (double)part[t][q];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  for (int ch = 0; ch < nch; ch += 2) {
    chunk(std::integral_constant<int, 0>{}, ch);
    if (ch + 1 < nch) chunk(std::integral_constant<int, 1>{}, ch + 1);
  }

  // lane holds acc[t][q]: row row0 + 16 t + lane % 16, right-hand side c = 4 (lane / 16) + q
  float csum[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t row = row0 + 16 * t + ln;
    const bool live = row < L.n;
    const bool in_i = row >= start && row < start + len;
    float rs = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * lg + q;
      if (live && c < l) {
        const float r = in_i ? 0.f : (float)((double)R[row * l + c] - acc[t][q]);
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
    for (int q = 0; q < 4; ++q) {
      float x = csum[q];
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 8);
      if (ln == 0) red[wave][4 * lg + q] = x;
    }
    __syncthreads();
    if (threadIdx.x < kMaxL) {
      const int c = threadIdx.x;
      float v = 0.f;
      if (c < NH) {
#pragma unroll
        for (int w = 0; w < NW; ++w) v += red[w][c];
      }
      colsq[(size_t)blockIdx.x * kMaxL + c] = c < l ? v : 0.f;
    }
  }
}

// FP32 tiles with few right-hand sides (l <= 8): the product with the step on
// the vector units, since the 32-column matrix tile would do 32 multiply-adds
// per kernel entry where l are needed. One thread per row (256 rows per
// workgroup, the same partials as the tile kernels); the chunk's column
// features and step are staged in LDS and read by all lanes at once. Each
// chunk's l sums accumulate in FP32 and the chunk sums in FP64, as in the
// 16-row matrix-core kernel.
template <int KERN, int DV, int DP, int NV>
__global__ __launch_bounds__(256) void k_fused_fp32v(
    Layout L, const double* __restrict__ xv, const double* __restrict__ xn,
    const float* __restrict__ dtile, const Ctl* __restrict__ ctl, int block,
    float* __restrict__ R, float* __restrict__ rowsq, float* __restrict__ colsq, int want_rowsq,
    int want_colsq) {
  constexpr int NW = 4;
  __shared__ __attribute__((aligned(16))) double sx[2][kChunk][DP];
  __shared__ __attribute__((aligned(16))) double sn[2][kChunk];
  __shared__ __attribute__((aligned(16))) float sd[2][kChunk][NV];
  __shared__ float red[4][NV];
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int nch = (len + kChunk - 1) / kChunk;
  const int l = L.l;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t row = (int64_t)blockIdx.x * kRowsWG + threadIdx.x;

  stage_async<DP, NV, NW>(xv, xn, dtile, start, 0, &sx[0][0][0], sn[0], &sd[0][0][0]);
  double xr[DV];  // -2 v_i
#pragma unroll
  for (int k = 0; k < DV; ++k) xr[k] = -2.0 * xv[row * DP + k];
  const double nr = xn[row];
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = 0.0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // double-buffered chunks, as in k_fused_fp32
  auto chunk = [&](auto buf, int ch) {
    constexpr int B = decltype(buf)::value;
    if (ch + 1 < nch)
      stage_async<DP, NV, NW>(xv, xn, dtile, start, ch + 1, &sx[B ^ 1][0][0], sn[B ^ 1],
                              &sd[B ^ 1][0][0]);
    float part[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) part[c] = 0.f;
#pragma unroll 4
    for (int j = 0; j < kChunk; ++j) {
      const float kv = kmap_acc<KERN>(dist2n<DV>(xr, nr, sx[B][j], sn[B][j]));
#pragma unroll
      for (int c = 0; c < NV; ++c) part[c] = fmaf(kv, sd[B][j][c], part[c]);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] += (double)part[c];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  for (int ch = 0; ch < nch; ch += 2) {
    chunk(std::integral_constant<int, 0>{}, ch);
    if (ch + 1 < nch) chunk(std::integral_constant<int, 1>{}, ch + 1);
  }

  const bool live = row < L.n;
  const bool in_i = row >= start && row < start + len;
  float rs = 0.f, csq[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    csq[c] = 0.f;
    if (live && c < l) {
      const float r = in_i ? 0.f : (float)((double)R[row * l + c] - acc[c]);
      R[row * l + c] = r;
      rs = fmaf(r, r, rs);
      csq[c] = r * r;
    }
  }
  if (want_rowsq && row < L.n_pad) rowsq[row] = live ? rs : 0.f;
  if (want_colsq) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      float x = csq[c];
      x += __shfl_xor(x, 1);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 8);
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      if (lane == 0) red[wave][c] = x;
    }
    __syncthreads();
    if (threadIdx.x < kMaxL) {
      const int c = threadIdx.x;
      float v = 0.f;
      if (c < NV) v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      colsq[(size_t)blockIdx.x * kMaxL + c] = c < l ? v : 0.f;
    }
  }
}

// Split path: FP32 kernel tiles (FP64 squared distance of the FP64 prepared
// features by differencing, kmap_acc) and the product on BF16 matrix cores. The tile K = kh + km + kl and the
// step d = dh + dm + dl are each held as three BF16 terms (24 significant bits),
// and the six partial products with term orders summing to at most 2,
//   dl kh + dh kl + dm km + dm kh + dh km + dh kh   (small to large),
// are accumulated in FP32 per chunk and in FP64 across chunks: the product has
// FP32-grade accuracy at BF16 matrix-core rates. The K operand of each MFMA is
// built per lane in the BF16 path's column order, so the step layout is shared.
template <int KERN, int DV, int DP>
__device__ __forceinline__ void split_body(const Layout& L, const double* __restrict__ xv,
                                           const uint16_t* __restrict__ dtile, int blk,
                                           float* __restrict__ R, float* __restrict__ rowsq,
                                           float* __restrict__ colsq, bool want_rowsq,
                                           bool want_colsq, int wg, double* sx) {
  const int64_t start = (int64_t)blk * L.b;
  const int len = (int)std::min<int64_t>(L.b, L.n - start);
  const int nch = (len + kChunk - 1) / kChunk;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int nl = lane % 32, g = lane / 32;
  const int64_t row0 = (int64_t)wg * kRowsWG + wave * 64;
  const size_t term = (size_t)L.b_pad * kMaxL;

  double xr[2][DV];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int k = 0; k < DV; ++k) xr[t][k] = xv[(row0 + 32 * t + nl) * DP + k];

  f64x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.0;

  for (int ch = 0; ch < nch; ++ch) {
    const int64_t cb = start + (int64_t)ch * kChunk;
    __syncthreads();
    for (int e = threadIdx.x; e < kChunk * DP; e += 256) sx[e] = xv[cb * DP + e];
    __syncthreads();
    f32x16 part[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) part[t][v] = 0.f;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const size_t at = (((size_t)ch * 2 + st) * 64 + lane) * 8;
      const bf16x8 dh = load_bf16x8(dtile + at);
      const bf16x8 dm = load_bf16x8(dtile + term + at);
      const bf16x8 dl = load_bf16x8(dtile + 2 * term + at);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        f32x16 kv;  // only elements 0..7 used: this k-step's eight columns
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int cc = 16 * st + 4 * g + (e % 4) + 8 * (e / 4);
          kv[e] = kmap_acc<KERN>(dist2<DV>(xr[t], sx + cc * DP));
        }
        const bf16x8 kh = pack8(kv, 0);
#pragma unroll
        for (int e = 0; e < 8; ++e) kv[e] -= (float)kh[e];
        const bf16x8 km = pack8(kv, 0);
#pragma unroll
        for (int e = 0; e < 8; ++e) kv[e] -= (float)km[e];
        const bf16x8 kl = pack8(kv, 0);
        part[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(dl, kh, part[t], 0, 0, 0);
        part[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(dh, kl, part[t], 0, 0, 0);
        part[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(dm, km, part[t], 0, 0, 0);
        part[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(dm, kh, part[t], 0, 0, 0);
        part[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(dh, km, part[t], 0, 0, 0);
        part[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(dh, kh, part[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[t][v] += (double)part[t][v];
  }
  epilogue<2, 4>(L, row0, start, len, acc, R, rowsq, colsq, want_rowsq, want_colsq, wg);
}

template <int KERN, int DV, int DP>
__global__ __launch_bounds__(256) void k_fused_split(Layout L, const double* __restrict__ xv,
                                                     const uint16_t* __restrict__ dtile,
                                                     const Ctl* __restrict__ ctl, int block,
                                                     float* __restrict__ R,
                                                     float* __restrict__ rowsq,
                                                     float* __restrict__ colsq, int want_rowsq,
                                                     int want_colsq) {
  __shared__ double sx[kChunk * DP];
  const int blk = resolve_block(block, ctl, L.m);
  if (blk < 0) return;
  split_body<KERN, DV, DP>(L, xv, dtile, blk, R, rowsq, colsq, want_rowsq, want_colsq,
                           (int)blockIdx.x, sx);
}

// Grouped split update of a batch step: each workgroup runs the body for its
// problem's block, with the feature loop over the padded stride (the padded
// features are zero, so r^2 is the same). Every update writes the column
// partials; the batch's epoch-end check reads those of the epoch's last one.
template <int KERN, int WIDE>
__device__ __forceinline__ void split_dispatch(const Layout& L, const Desc* ds, int blk, float* R,
                                               int wg, double* sx) {
  const double* xs = ds->D.xv;
  const uint16_t* dt = (const uint16_t*)ds->D.dtile;
  const bool wr = L.order == 1;
  if constexpr (WIDE == 0) {
    if (L.dp == 4)
      split_body<KERN, 4, 4>(L, xs, dt, blk, R, ds->D.rowsq, ds->D.colsq, wr, true, wg, sx);
    else
      split_body<KERN, 8, 8>(L, xs, dt, blk, R, ds->D.rowsq, ds->D.colsq, wr, true, wg, sx);
  } else {
    if (L.dp == 12)
      split_body<KERN, 12, 12>(L, xs, dt, blk, R, ds->D.rowsq, ds->D.colsq, wr, true, wg, sx);
    else if (L.dp == 16)
      split_body<KERN, 16, 16>(L, xs, dt, blk, R, ds->D.rowsq, ds->D.colsq, wr, true, wg, sx);
    else
      split_body<KERN, 20, 20>(L, xs, dt, blk, R, ds->D.rowsq, ds->D.colsq, wr, true, wg, sx);
  }
}

// WIDE = 0 serves feature strides 4 and 8, WIDE = 1 strides 12 to 20: the
// narrow kernel keeps two waves per SIMD, which the wide variants' registers
// would not allow.
template <int WIDE>
__global__ __launch_bounds__(256) void g_fused_split(Group g) {
  __shared__ double sx[kChunk * (WIDE ? kMaxD : 8)];
  int wg;
  const int p = group_job(g, &wg);
  const Desc* ds = g.desc[p];
  const Layout L = ds->L;
  const int blk =
      resolve_block(L.order != 0 ? kBlockBatchSel : kBlockBatchCyclic, ds->D.ctl, L.m);
  if (blk < 0) return;
  if (L.kernel == 0)
    split_dispatch<0, WIDE>(L, ds, blk, g.R[p], wg, sx);
  else if (L.kernel == 1)
    split_dispatch<1, WIDE>(L, ds, blk, g.R[p], wg, sx);
  else
    split_dispatch<2, WIDE>(L, ds, blk, g.R[p], wg, sx);
}

template <int KERN>
hipError_t launch_bf16(const Layout& L, const Dev& D, int32_t block, float* R, bool wr, bool wc,
                       hipStream_t st) {
  const dim3 g(L.nwg), t(256);
  const uint16_t* dt = (const uint16_t*)D.dtile;
  switch (L.ks) {
    case 1: hipLaunchKernelGGL((k_fused_bf16<KERN, 1>), g, t, 0, st, L, D.xrow, D.xcol, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 2: hipLaunchKernelGGL((k_fused_bf16<KERN, 2>), g, t, 0, st, L, D.xrow, D.xcol, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 3: hipLaunchKernelGGL((k_fused_bf16<KERN, 3>), g, t, 0, st, L, D.xrow, D.xcol, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 4: hipLaunchKernelGGL((k_fused_bf16<KERN, 4>), g, t, 0, st, L, D.xrow, D.xcol, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KERN, int NV>
hipError_t launch_fp32v(const Layout& L, const Dev& D, int32_t block, float* R, bool wr, bool wc,
                        hipStream_t st) {
  const dim3 g(L.nwg), t(256);
  const float* dt = (const float*)D.dtile;
#define AP_FP32V(DV, DP)                                                                  \
  hipLaunchKernelGGL((k_fused_fp32v<KERN, DV, DP, NV>), g, t, 0, st, L, D.xv, D.xn, dt, \
                     D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc)
  if (L.d == 3) {
    AP_FP32V(3, 4);
  } else {
    switch (L.dp) {
      case 4: AP_FP32V(4, 4); break;
      case 8: AP_FP32V(8, 8); break;
      case 12: AP_FP32V(12, 12); break;
      case 16: AP_FP32V(16, 16); break;
      case 20: AP_FP32V(20, 20); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef AP_FP32V
  return hipGetLastError();
}

// Row tiles per wave of the 16-row kernel: the workgroup's 256 rows go to
// 256 / (16 kTilesH) waves. Two tiles (eight waves) keep the row features of a
// lane within the register budget of four waves per SIMD; four tiles held two.
constexpr int kTilesH = 2;
constexpr int kThreadsH = kRowsWG / (16 * kTilesH) * 64;
// Row tiles per wave of the 32-row kernel. One tile (eight waves) raises the
// occupancy but doubles the LDS reads per kernel value, and is slower.
constexpr int kTiles32 = 2;
constexpr int kThreads32 = kRowsWG / (32 * kTiles32) * 64;

template <int KERN>
hipError_t launch_fp32(const Layout& L, const Dev& D, int32_t block, float* R, bool wr, bool wc,
                       hipStream_t st) {
  if (L.l <= 1) return launch_fp32v<KERN, 1>(L, D, block, R, wr, wc, st);
  if (L.l <= 2) return launch_fp32v<KERN, 2>(L, D, block, R, wr, wc, st);
  if (L.l <= 4) return launch_fp32v<KERN, 4>(L, D, block, R, wr, wc, st);
  if (L.l <= 8) return launch_fp32v<KERN, 8>(L, D, block, R, wr, wc, st);
  const dim3 g(L.nwg);
  const float* dt = (const float*)D.dtile;
  const bool half = L.l <= 16;
#define AP_FP32(DV, DP)                                                                          \
  if (half)                                                                                      \
    hipLaunchKernelGGL((k_fused_fp32h<KERN, DV, DP, kTilesH>), g, dim3(kThreadsH), 0, st, L,     \
                       D.xv, D.xn, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc);     \
  else                                                                                           \
    hipLaunchKernelGGL((k_fused_fp32<KERN, DV, DP, kTiles32>), g, dim3(kThreads32), 0, st, L,    \
                       D.xv, D.xn, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc)
  if (L.d == 3) {
    AP_FP32(3, 4);
  } else {
    switch (L.dp) {
      case 4: AP_FP32(4, 4); break;
      case 8: AP_FP32(8, 8); break;
      case 12: AP_FP32(12, 12); break;
      case 16: AP_FP32(16, 16); break;
      case 20: AP_FP32(20, 20); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef AP_FP32
  return hipGetLastError();
}

template <int KERN>
hipError_t launch_split(const Layout& L, const Dev& D, int32_t block, float* R, bool wr,
                        bool wc, hipStream_t st) {
  const dim3 g(L.nwg), t(256);
  const uint16_t* dt = (const uint16_t*)D.dtile;
  if (L.d == 3) {
    hipLaunchKernelGGL((k_fused_split<KERN, 3, 4>), g, t, 0, st, L, D.xv, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc);
    return hipGetLastError();
  }
  switch (L.dp) {
    case 4: hipLaunchKernelGGL((k_fused_split<KERN, 4, 4>), g, t, 0, st, L, D.xv, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 8: hipLaunchKernelGGL((k_fused_split<KERN, 8, 8>), g, t, 0, st, L, D.xv, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 12: hipLaunchKernelGGL((k_fused_split<KERN, 12, 12>), g, t, 0, st, L, D.xv, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 16: hipLaunchKernelGGL((k_fused_split<KERN, 16, 16>), g, t, 0, st, L, D.xv, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    case 20: hipLaunchKernelGGL((k_fused_split<KERN, 20, 20>), g, t, 0, st, L, D.xv, dt, D.ctl, block, R, D.rowsq, D.colsq, (int)wr, (int)wc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_group_split(const Group& g, bool wide, hipStream_t st) {
  if (wide)
    hipLaunchKernelGGL(g_fused_split<1>, dim3(g.wg0[g.count]), dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL(g_fused_split<0>, dim3(g.wg0[g.count]), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_fused_update(const Layout& L, const Dev& D, int32_t block, float* R,
                               bool want_rowsq, bool want_colsq, hipStream_t st) {
  if (L.tile == 1) {
    switch (L.kernel) {
      case 0: return launch_bf16<0>(L, D, block, R, want_rowsq, want_colsq, st);
      case 1: return launch_bf16<1>(L, D, block, R, want_rowsq, want_colsq, st);
      default: return launch_bf16<2>(L, D, block, R, want_rowsq, want_colsq, st);
    }
  }
  if (L.tile == 2) {
    switch (L.kernel) {
      case 0: return launch_split<0>(L, D, block, R, want_rowsq, want_colsq, st);
      case 1: return launch_split<1>(L, D, block, R, want_rowsq, want_colsq, st);
      default: return launch_split<2>(L, D, block, R, want_rowsq, want_colsq, st);
    }
  }
  switch (L.kernel) {
    case 0: return launch_fp32<0>(L, D, block, R, want_rowsq, want_colsq, st);
    case 1: return launch_fp32<1>(L, D, block, R, want_rowsq, want_colsq, st);
    default: return launch_fp32<2>(L, D, block, R, want_rowsq, want_colsq, st);
  }
}

}  // namespace ap
