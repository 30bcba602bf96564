// Float64 host-side geometry and tables for the DELIMIT layers.
//
// Everything here runs once per gradient table (or once per batch when the
// directions are re-distorted), never per voxel:
//   * real even-order SH basis via the fully normalised associated-Legendre
//     recurrence (the basis the SH layers of Sec. 2.2 work in);
//   * the Laplace-Beltrami regularised fit (B^T B + lambda L)^{-1} B^T by a
//     Cholesky factorisation (Signal2SH, Sec. 2.2, and the LSC refit);
//   * shell grouping of a multi-shell table;
//   * cyclic-kernel point geometry around each direction (Sec. 2.3, Fig. 3).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace dlm {

static const double kPi = 3.14159265358979323846;

int sh_num_coeffs(int L) { return (L + 1) * (L + 2) / 2; }

bool sh_order_ok(int L) { return L >= 0 && L <= kMaxShOrder && (L % 2) == 0; }

bool unit_dir(const double *in, double *out) {
  const double x = in[0], y = in[1], z = in[2];
  if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return false;
  const double n = std::sqrt(x * x + y * y + z * z);
  if (!(n > 1e-12)) return false;
  out[0] = x / n;
  out[1] = y / n;
  out[2] = z / n;
  return true;
}

// One row of the basis at a unit direction u (length K).
// Normalised Legendre \bar P_l^m = N_l^m P_l^m (Condon-Shortley phase):
//   \bar P_0^0 = 1/sqrt(4 pi)
//   \bar P_m^m = -sqrt((2m+1)/(2m)) sin(t) \bar P_{m-1}^{m-1}
//   \bar P_{m+1}^m = sqrt(2m+3) cos(t) \bar P_m^m
//   \bar P_l^m = a_lm (cos(t) \bar P_{l-1}^m - b_lm \bar P_{l-2}^m),
//     a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
void sh_row(int L, const double *u, double *row) {
  const double ct = std::max(-1.0, std::min(1.0, u[2]));
  const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  const double phi = std::atan2(u[1], u[0]);
  // plm[l*(L+1)+m]
  double plm[(kMaxShOrder + 1) * (kMaxShOrder + 1)];
  const int W = L + 1;
  double pmm = 1.0 / std::sqrt(4.0 * kPi);
  for (int m = 0; m <= L; ++m) {
    if (m > 0) pmm = -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * pmm;
    plm[m * W + m] = pmm;
    if (m + 1 <= L) plm[(m + 1) * W + m] = std::sqrt(2.0 * m + 3.0) * ct * pmm;
    for (int l = m + 2; l <= L; ++l) {
      const double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
      const double b = std::sqrt((double(l - 1) * (l - 1) - double(m) * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
      plm[l * W + m] = a * (ct * plm[(l - 1) * W + m] - b * plm[(l - 2) * W + m]);
    }
  }
  const double r2 = std::sqrt(2.0);
  for (int l = 0; l <= L; l += 2) {
    const int base = l * (l + 1) / 2;
    row[base] = plm[l * W + 0];
    for (int m = 1; m <= l; ++m) {
      const double p = plm[l * W + m];
      row[base - m] = r2 * p * std::cos(m * phi);
      row[base + m] = r2 * p * std::sin(m * phi);
    }
  }
}

void sh_basis_unit(int L, const double *u, int64_t n, double *B) {
  const int K = sh_num_coeffs(L);
  for (int64_t i = 0; i < n; ++i) sh_row(L, u + 3 * i, B + i * K);
}

// P (K x n) = (B^T B + lambda diag(l^2(l+1)^2))^{-1} B^T, B is n x K.
bool fit_from_basis(int L, const double *B, int64_t n, double lambda, double *P) {
  const int K = sh_num_coeffs(L);
  std::vector<double> A(size_t(K) * K, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const double *r = B + i * K;
    for (int a = 0; a < K; ++a)
      for (int b = 0; b <= a; ++b) A[size_t(a) * K + b] += r[a] * r[b];
  }
  for (int l = 0; l <= L; l += 2) {
    const double pen = double(l) * l * (l + 1.0) * (l + 1.0);
    for (int m = -l; m <= l; ++m) {
      const int j = l * (l + 1) / 2 + m;
      A[size_t(j) * K + j] += lambda * pen;
    }
  }
  // Cholesky A = G G^T (lower triangle, in place).
  for (int j = 0; j < K; ++j) {
    double d = A[size_t(j) * K + j];
    for (int k = 0; k < j; ++k) d -= A[size_t(j) * K + k] * A[size_t(j) * K + k];
    if (!(d > 1e-13 * (1.0 + std::fabs(A[size_t(j) * K + j])))) return false;
    const double gjj = std::sqrt(d);
    A[size_t(j) * K + j] = gjj;
    for (int i = j + 1; i < K; ++i) {
      double s = A[size_t(i) * K + j];
      for (int k = 0; k < j; ++k) s -= A[size_t(i) * K + k] * A[size_t(j) * K + k];
      A[size_t(i) * K + j] = s / gjj;
    }
  }
  // Solve for every column i of B^T: G z = b, G^T p = z.
  std::vector<double> z(K);
  for (int64_t i = 0; i < n; ++i) {
    const double *b = B + i * K;
    for (int r = 0; r < K; ++r) {
      double s = b[r];
      for (int k = 0; k < r; ++k) s -= A[size_t(r) * K + k] * z[k];
      z[r] = s / A[size_t(r) * K + r];
    }
    for (int r = K - 1; r >= 0; --r) {
      double s = z[r];
      for (int k = r + 1; k < K; ++k) s -= A[size_t(k) * K + r] * P[size_t(k) * n + i];
      P[size_t(r) * n + i] = s / A[size_t(r) * K + r];
    }
  }
  return true;
}

void group_shells(const double *bvals, int64_t n, double b0_max, double rel_tol,
                  std::vector<std::vector<int64_t>> &members, std::vector<double> &centres) {
  std::vector<std::vector<int64_t>> mem;
  std::vector<double> cen, sum;
  for (int64_t i = 0; i < n; ++i) {
    const double b = bvals[i];
    if (b < b0_max) continue;
    bool placed = false;
    for (size_t k = 0; k < cen.size(); ++k) {
      if (std::fabs(b - cen[k]) <= rel_tol * cen[k]) {
        mem[k].push_back(i);
        sum[k] += b;
        cen[k] = sum[k] / double(mem[k].size());
        placed = true;
        break;
      }
    }
    if (!placed) {
      mem.push_back({i});
      cen.push_back(b);
      sum.push_back(b);
    }
  }
  std::vector<size_t> order(cen.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cen[a] < cen[b]; });
  members.clear();
  centres.clear();
  for (size_t k : order) {
    members.push_back(mem[k]);
    centres.push_back(cen[k]);
  }
}

void kernel_points_unit(const double *g, int64_t m, const int *ks, int R, double alpha, double *pts) {
  int T = 1;
  for (int r = 0; r < R; ++r) T += ks[r];
  for (int64_t i = 0; i < m; ++i) {
    const double *u = g + 3 * i;
    const double ct = std::max(-1.0, std::min(1.0, u[2]));
    const double th = std::acos(ct);
    const double ph = std::atan2(u[1], u[0]);
    const double et[3] = {std::cos(th) * std::cos(ph), std::cos(th) * std::sin(ph), -std::sin(th)};
    const double ep[3] = {-std::sin(ph), std::cos(ph), 0.0};
    double *o = pts + size_t(i) * T * 3;
    o[0] = u[0];
    o[1] = u[1];
    o[2] = u[2];
    int t = 1;
    for (int r = 0; r < R; ++r) {
      const double rho = (r + 1) * alpha / R;
      const double cr = std::cos(rho), sr = std::sin(rho);
      for (int b = 0; b < ks[r]; ++b, ++t) {
        const double psi = 2.0 * kPi * b / ks[r];
        const double cp = std::cos(psi), sp = std::sin(psi);
        for (int d = 0; d < 3; ++d) o[3 * t + d] = cr * u[d] + sr * (cp * et[d] + sp * ep[d]);
      }
    }
  }
}

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return uint16_t((u >> 16) | 0x40);  // quiet NaN
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return uint16_t(u >> 16);
}

uint16_t f64_to_bf16_rne(double d) {
  // Round the float64 value to the nearest bfloat16 directly (one rounding),
  // by rounding to float with round-to-odd first, which is exact for the
  // subsequent 16-bit rounding.
  float f = float(d);
  if (double(f) != d && std::isfinite(d)) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    // make the float the truncation toward zero, then set the sticky bit
    if (std::fabs(double(f)) > std::fabs(d)) u -= 1;
    u |= 1u;
    std::memcpy(&f, &u, 4);
  }
  return f32_to_bf16_rne(f);
}

}  // namespace dlm
