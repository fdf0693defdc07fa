/* Test helper: a block's products sum_q K[i][q] d[q][c] formed the way the
 * fused update's matrix cores form them, for the rounding floor of the
 * reduced-precision tiles. Each run of `span` columns (32, or 64 where the
 * kernel sums a pair of chunks in FP32) starts from an FP32 zero and takes
 * `group` products per step; the step's sum (exact in FP64 for these
 * operands' widths) is added to the FP32 accumulator with one rounding. The
 * run sums are added up in FP64. K is n x len (row-major), d is len x l,
 * out is n x l. Built by tests/helpers.py; not part of the solver. */
#include <stdint.h>

void chunk_products(const float* K, const float* d, int64_t n, int len, int l, int group,
                    int span, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const float* Ki = K + i * (int64_t)len;
    for (int c = 0; c < l; ++c) {
      double tot = 0.0;
      for (int c0 = 0; c0 < len; c0 += span) {
        float acc = 0.0f;
        const int c1 = c0 + span < len ? c0 + span : len;
        for (int g0 = c0; g0 < c1; g0 += group) {
          double t = 0.0;
          const int g1 = g0 + group < c1 ? g0 + group : c1;
          for (int q = g0; q < g1; ++q) t += (double)Ki[q] * (double)d[(int64_t)q * l + c];
          acc = (float)((double)acc + t);
        }
        tot += (double)acc;
      }
      out[i * l + c] = tot;
    }
  }
}
