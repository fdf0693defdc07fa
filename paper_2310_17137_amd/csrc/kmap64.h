// FP64 kernel map shared by the FP64-tile update and the FP64 true residual:
// k = s * map(r^2) with r^2 the ARD squared distance (exact differencing).
//
// The exponential is table driven (P. T. P. Tang, "Table-driven implementation
// of the exponential function in IEEE floating-point arithmetic", ACM TOMS
// 15(2), 1989): for y <= 0, with kk = round(y * 64 / ln 2),
//   y = kk ln2/64 + r,  |r| <= ln2/128,
//   exp(y) = 2^(kk div 64) * 2^((kk mod 64)/64) * (1 + r q(r)),
// where 1 + r q(r) is the degree-5 Taylor polynomial of exp(r) (truncation
// below 2^-54 relative on that range). ln2/64 is split into a head with 21
// trailing zero bits, so kk times the head is exact, and a tail; kk is read
// from the low word of y * 64/ln2 + 1.5 * 2^52. The 64 values s * 2^(j/64)
// (outputscale folded in) sit in LDS, staged once per workgroup. The result
// is within a few units in the last place of s exp(y); gen_exp_table.py prints
// the constants.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ap {

// 2^(j/64), j = 0..63, correctly rounded
constexpr double kExp2Tab[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};
constexpr double kLn2By64Hi = 0x1.62e42fee00000p-7;
constexpr double kLn2By64Lo = 0x1.a39ef35793c76p-39;
constexpr double k64ByLn2 = 0x1.71547652b82fep+6;
constexpr double kRoundMagic = 0x1.8p52;

// tab[j] = s * 2^(j/64); every thread of the workgroup calls it, and a
// barrier must follow before the first lookup.
__device__ inline void scaled_exp_table(double* tab, double s) {
  for (int j = threadIdx.x; j < 64; j += blockDim.x) tab[j] = s * kExp2Tab[j];
}

// s * exp(y) for y <= 0 (tab from scaled_exp_table); 0 below the FP64 range.
__host__ __device__ inline double scaled_exp(double y, const double* tab) {
  y = fmax(y, -746.0);
  const double t = fma(y, k64ByLn2, kRoundMagic);
  const double kd = t - kRoundMagic;
  const int32_t kk = (int32_t)(uint32_t)__builtin_bit_cast(uint64_t, t);
  double r = fma(kd, -kLn2By64Hi, y);
  r = fma(kd, -kLn2By64Lo, r);
  double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  const double T = tab[kk & 63];
  return ldexp(fma(T * r, q, T), kk >> 6);
}

template <int KERN>
__host__ __device__ inline double kernel_fp64(double r2, const double* tab) {
  if constexpr (KERN == 0) {
    return scaled_exp(-0.5 * r2, tab);
  } else if constexpr (KERN == 1) {
    const double t = 1.7320508075688772 * sqrt(r2);
    return (1.0 + t) * scaled_exp(-t, tab);
  } else {
    const double r = sqrt(r2), t = 2.23606797749979 * r;
    return (1.0 + t + (5.0 / 3.0) * r2) * scaled_exp(-t, tab);
  }
}

}  // namespace ap
