// Driver for the sanitizer build of the library's float64 host code
// (csrc/host_tables.cpp): SH basis rows, regularised fits (singular ones
// included), shell grouping, cyclic-kernel points and bfloat16 rounding, on
// ordinary and edge inputs.  Built with -fsanitize=address,undefined by
// tests/test_host_sanitizers.py, which also checks the printed values.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "../../paper_1808_01517_amd/csrc/internal.h"

using namespace dlm;

int main() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  // directions: random ones, both poles, the equator, and an unnormalised one
  std::vector<double> dirs;
  for (int i = 0; i < 61; ++i)
    for (int c = 0; c < 3; ++c) dirs.push_back(u(rng));
  const double extra[] = {0, 0, 1, 0, 0, -1, 1, 0, 0, 0, 3, 4};
  dirs.insert(dirs.end(), extra, extra + 12);
  const int n = int(dirs.size() / 3);
  std::vector<double> unit(dirs.size());
  for (int i = 0; i < n; ++i)
    if (!unit_dir(dirs.data() + 3 * i, unit.data() + 3 * i)) return 2;
  double zero[3] = {0, 0, 0}, nan3[3] = {std::nan(""), 0, 1}, out[3];
  if (unit_dir(zero, out) || unit_dir(nan3, out)) return 3;

  // basis at every supported order: print the sum over directions of the
  // squared row norms (the addition theorem makes each row's squared norm
  // sum_l (2l+1)/(4 pi) over even l)
  for (int L = 0; L <= kMaxShOrder; L += 2) {
    const int K = sh_num_coeffs(L);
    std::vector<double> B(size_t(n) * K);
    sh_basis_unit(L, unit.data(), n, B.data());
    double s = 0;
    for (double v : B) s += v * v;
    std::printf("basis %d %.12f\n", L, s / n);
  }
  if (sh_order_ok(3) || sh_order_ok(-2) || sh_order_ok(kMaxShOrder + 2)) return 4;

  // fits: full rank, lambda > 0 with too few directions, singular at lambda 0
  for (int L : {2, 4, 8}) {
    const int K = sh_num_coeffs(L);
    for (int m : {K - 1, K, 2 * K}) {
      if (m > n) continue;
      std::vector<double> B(size_t(m) * K), P(size_t(m) * K);
      sh_basis_unit(L, unit.data(), m, B.data());
      for (double lam : {0.0, 0.006}) {
        const bool ok = fit_from_basis(L, B.data(), m, lam, P.data());
        // P B = I at lambda = 0 and full rank: print the largest deviation
        double dev = -1;
        if (ok && lam == 0.0) {
          dev = 0;
          for (int a = 0; a < K; ++a)
            for (int b = 0; b < K; ++b) {
              double s = 0;
              for (int i = 0; i < m; ++i) s += P[size_t(a) * m + i] * B[size_t(i) * K + b];
              dev = std::fmax(dev, std::fabs(s - (a == b ? 1.0 : 0.0)));
            }
        }
        std::printf("fit %d %d %g %d %.3e\n", L, m, lam, int(ok), dev);
      }
    }
  }

  // shells: b0 volumes, three shells in mixed order, all-b0
  const double bvals[] = {0, 5, 1000, 2990, 1010, 2000, 0, 3000, 1990, 30};
  std::vector<std::vector<int64_t>> members;
  std::vector<double> centres;
  group_shells(bvals, 10, 50.0, 0.05, members, centres);
  std::printf("shells %zu", members.size());
  for (size_t s = 0; s < members.size(); ++s) std::printf(" %zu@%.1f", members[s].size(), centres[s]);
  std::printf("\n");
  const double b0s[] = {0, 1, 2};
  group_shells(b0s, 3, 50.0, 0.05, members, centres);
  std::printf("shells_b0 %zu\n", members.size());

  // kernel points: one and two rings, and the largest kernel
  for (int R : {1, 2}) {
    const int ks[] = {8, 8};
    const int T = 1 + 8 * R;
    std::vector<double> pts(size_t(n) * T * 3);
    kernel_points_unit(unit.data(), n, ks, R, 0.5235987755982988, pts.data());
    double worst = 0;
    for (size_t i = 0; i < pts.size() / 3; ++i)
      worst = std::fmax(worst, std::fabs(std::sqrt(pts[3 * i] * pts[3 * i] + pts[3 * i + 1] * pts[3 * i + 1] +
                                                   pts[3 * i + 2] * pts[3 * i + 2]) -
                                         1.0));
    std::printf("points %d %.3e\n", R, worst);
  }
  {
    std::vector<int> ks(1, kMaxTaps - 1);
    std::vector<double> pts(size_t(2) * kMaxTaps * 3);
    kernel_points_unit(unit.data(), 2, ks.data(), 1, 1.0, pts.data());
  }

  // bfloat16 rounding: ties to even, overflow to infinity, NaN stays NaN
  const float fs[] = {1.0f, 1.00390625f, 1.01171875f, -2.5f, 3.0e38f, 1e-40f, 0.0f, -0.0f,
                      std::numeric_limits<float>::infinity(), std::numeric_limits<float>::quiet_NaN()};
  std::printf("bf16");
  for (float f : fs) std::printf(" %04x", unsigned(f32_to_bf16_rne(f)));
  std::printf("\nbf16d %04x %04x\n", unsigned(f64_to_bf16_rne(1.00390625)), unsigned(f64_to_bf16_rne(-1e300)));
  return 0;
}
