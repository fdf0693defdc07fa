// Host check of the table-driven FP64 exponential and kernel map of the FP64
// tiles against long-double references: prints the largest error in units in
// the last place of the FP64 result over a dense sweep of arguments.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "../paper_2310_17137_amd/csrc/kmap64.h"

static double ulps(double got, long double ref) {
  if (ref == 0.0L) return got == 0.0 ? 0.0 : 1e300;
  const double r = (double)ref;
  const double ulp = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
  return (double)(std::fabs((long double)got - ref) / ulp);
}

int main() {
  const double scales[3] = {1.0, 1.7, 0.3};
  double worst_exp = 0.0, worst_map[3] = {0.0, 0.0, 0.0};
  double worst_y = 0.0;
  std::mt19937_64 rng(7);
  for (double s : scales) {
    double tab[ap::kExpTab];
    for (int j = 0; j < ap::kExpTab; ++j) tab[j] = s * ap::kExp2Tab[j];
    // the exponential: y in [-700, 0] (normal results), uniform and dense near 0
    std::uniform_real_distribution<double> wide(-700.0, 0.0), near(-1.0, 0.0);
    for (int i = 0; i < 400000; ++i) {
      const double y = (i % 2) ? wide(rng) : near(rng);
      const double e = ulps(ap::scaled_exp(y, tab), (long double)s * expl((long double)y));
      if (e > worst_exp) { worst_exp = e; worst_y = y; }
    }
    for (double y : {0.0, -1e-300, -1e-17, -0x1p-60, -0.00135, -0.0027, -0.0054, -0.5, -1.0,
                     -10.0}) {
      const double e = ulps(ap::scaled_exp(y, tab), (long double)s * expl((long double)y));
      if (e > worst_exp) { worst_exp = e; worst_y = y; }
    }
    // the kernel maps on r^2 in [0, 1200]
    std::uniform_real_distribution<double> r2d(0.0, 1200.0), r2n(0.0, 4.0);
    for (int i = 0; i < 200000; ++i) {
      const double r2 = (i % 2) ? r2d(rng) : r2n(rng);
      const long double R2 = r2, R = sqrtl(R2);
      const long double k0 = s * expl(-0.5L * R2);
      const long double t3 = sqrtl(3.0L) * R, k1 = s * (1.0L + t3) * expl(-t3);
      const long double t5 = sqrtl(5.0L) * R, k2 = s * (1.0L + t5 + 5.0L / 3.0L * R2) * expl(-t5);
      const double e0 = ulps(ap::kernel_fp64<0>(r2, tab), k0);
      const double e1 = ulps(ap::kernel_fp64<1>(r2, tab), k1);
      const double e2 = ulps(ap::kernel_fp64<2>(r2, tab), k2);
      // the Matern maps take exp of t = c sqrt(r2): the rounded constant, the
      // square root and the product leave t with a relative error up to
      // 1.5 * 2^-52, which exp turns into t times as much (up to 3 t ulps of
      // the result); with the polynomial factor and exp itself the bound is
      // 4 + 3 t ulps
      const double n1 = e1 / (4.0 + 3.0 * (double)t3), n2 = e2 / (4.0 + 3.0 * (double)t5);
      if (k0 > 1e-300L && e0 > worst_map[0]) worst_map[0] = e0;
      if (k1 > 1e-300L && n1 > worst_map[1]) worst_map[1] = n1;
      if (k2 > 1e-300L && n2 > worst_map[2]) worst_map[2] = n2;
    }
    // the RBF form with the halving folded into the constants is bitwise the
    // general one at -r2 / 2, above the FP64 range's end and beyond
    for (int i = 0; i < 400000; ++i) {
      const double r2 = (i % 4 == 0) ? r2d(rng) : (i % 4 == 1) ? r2n(rng)
                        : (i % 4 == 2) ? std::ldexp(r2n(rng), -(i % 1000)) : 1400.0 + r2n(rng) * 30.0;
      const double a = ap::scaled_exp_nhalf(r2, tab), b = ap::scaled_exp(-0.5 * r2, tab);
      if (std::memcmp(&a, &b, sizeof a) != 0) {
        std::printf("nhalf mismatch at r2 %.17g: %.17g vs %.17g\n", r2, a, b);
        return 1;
      }
    }
    for (double r2 : {0.0, 1e-300, 1492.0, 1493.0, 3000.0, 1e300, (double)INFINITY}) {
      const double a = ap::scaled_exp_nhalf(r2, tab), b = ap::scaled_exp(-0.5 * r2, tab);
      if (std::memcmp(&a, &b, sizeof a) != 0) {
        std::printf("nhalf mismatch at r2 %.17g: %.17g vs %.17g\n", r2, a, b);
        return 1;
      }
    }
    double tab1[ap::kExpTab];
    for (int j = 0; j < ap::kExpTab; ++j) tab1[j] = ap::kExp2Tab[j];
    // below the FP64 range the result is 0 or subnormal, never garbage
    for (double y : {-745.0, -745.2, -746.0, -800.0, -1e6, -1e300}) {
      const double v = ap::scaled_exp(y, tab1);
      if (!(v >= 0.0 && v < 1e-320)) { std::printf("underflow %g -> %g\n", y, v); return 1; }
    }
  }
  std::printf("exp_ulps %.3f at %.17g\nrbf_ulps %.3f\nm32_per_bound %.3f\nm52_per_bound %.3f\n", worst_exp,
              worst_y, worst_map[0], worst_map[1], worst_map[2]);
  return 0;
}
