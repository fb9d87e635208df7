// Host-side FP64 plan construction for the Kronecker-product solver.
//
// Sec. II.A of arXiv 2501.16572: the discrete Laplacian of a uniform 3D grid is
// the Kronecker sum of three 1D second-derivative operators, so
// L = (V1 (x) V2 (x) V3) Lambda (V1 (x) V2 (x) V3)^H with V_d the eigenvectors of
// the 1D operators (Eq. (FinalRepfL)), and f(L) = (...) f(Lambda) (...)^H with
// f from Eq. (fL).  This file computes, in FP64 on the host:
//   * the central 2p-th order second-derivative weights (closed form);
//   * the 1D eigenpairs per boundary condition: closed forms for periodic
//     (real cosine/sine basis at Gamma) and Bloch-periodic (complex plane
//     waves) axes, a cyclic Jacobi eigensolver for Dirichlet axes;
//   * the table f(lambda1[a] + lambda2[b] + lambda3[c]) over the grid.
#include "plan_host.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace kx {

std::vector<double> fd_weights(int order) {
  // c_s = 2 (-1)^(s+1) (p!)^2 / (s^2 (p-s)! (p+s)!),  c_0 = -2 sum 1/s^2
  // (Fornberg's closed form for the central second derivative).
  const int p = order / 2;
  std::vector<double> c(p + 1, 0.0);
  auto fact = [](int k) {
    long double r = 1;
    for (int i = 2; i <= k; ++i) r *= i;
    return r;
  };
  long double c0 = 0;
  for (int s = 1; s <= p; ++s) {
    long double v = 2.0L * fact(p) * fact(p) / ((long double)s * s * fact(p - s) * fact(p + s));
    c[s] = (double)((s % 2 == 1) ? v : -v);
    c0 -= 2.0L / ((long double)s * s);
  }
  c[0] = (double)c0;
  return c;
}

// FD symbol of the stencil at phase theta*h = t:
//   (c0 + 2 sum_s c_s cos(s t)) / h^2 = -(4/h^2) sum_s c_s sin^2(s t / 2),
// the second form is exact at t = 0 and free of cancellation near it.
static double fd_symbol(const std::vector<double>& c, double t, double h) {
  long double acc = 0;
  for (size_t s = 1; s < c.size(); ++s) {
    long double sn = std::sin(0.5L * (long double)s * t);
    acc += (long double)c[s] * sn * sn;
  }
  return (double)(-4.0L * acc / ((long double)h * h));
}

// Cyclic Jacobi eigensolver for a real symmetric n x n matrix (row-major).
// On return A's diagonal holds the eigenvalues and V[k*n + a] the k-th
// component of eigenvector a.
static void jacobi_eig(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  double fro = 0;
  for (double x : A) fro += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    if (off <= 1e-32 * fro) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = cs * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = cs * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
    }
  }
}

void eig1d(int n, double h, int bc, int order, double kappa, std::vector<double>& lam,
           std::vector<double>& Vre, std::vector<double>& Vim) {
  const std::vector<double> c = fd_weights(order);
  const int p = order / 2;
  lam.assign(n, 0.0);
  Vre.assign((size_t)n * n, 0.0);
  Vim.assign((size_t)n * n, 0.0);
  const double two_pi = 2.0 * M_PI;
  if (bc == 0 && kappa == 0.0) {
    // Real symmetric circulant: eigenvalue symbol(2 pi q / n) for frequency q,
    // shared by q and n - q; orthonormal real basis 1/sqrt(n), sqrt(2/n) cos,
    // sqrt(2/n) sin, and (-1)^j / sqrt(n) for even n.
    struct Col { double l; int kind; int q; };  // kind 0 const, 1 cos, 2 sin, 3 alt
    std::vector<Col> cols;
    cols.push_back({fd_symbol(c, 0.0, h), 0, 0});
    for (int q = 1; 2 * q < n; ++q) {
      double l = fd_symbol(c, two_pi * q / n, h);
      cols.push_back({l, 1, q});
      cols.push_back({l, 2, q});
    }
    if (n % 2 == 0) cols.push_back({fd_symbol(c, M_PI, h), 3, n / 2});
    std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) { return a.l < b.l; });
    const double s0 = 1.0 / std::sqrt((double)n), s1 = std::sqrt(2.0 / n);
    for (int a = 0; a < n; ++a) {
      lam[a] = cols[a].l;
      for (int j = 0; j < n; ++j) {
        // exact phase reduction: angle = 2 pi ((q j) mod n) / n
        long long r = ((long long)cols[a].q * j) % n;
        double ang = two_pi * (double)r / n;
        double v;
        switch (cols[a].kind) {
          case 0: v = s0; break;
          case 1: v = s1 * std::cos(ang); break;
          case 2: v = s1 * std::sin(ang); break;
          default: v = (j % 2 == 0) ? s0 : -s0; break;
        }
        Vre[(size_t)j * n + a] = v;
      }
    }
    return;
  }
  if (bc == 0) {
    // Bloch-periodic: u_q(j) = exp(i (2 pi q / n + kappa h) j) / sqrt(n) with
    // eigenvalue symbol(2 pi q / n + kappa h).
    struct Col { double l; int q; };
    std::vector<Col> cols(n);
    const double kh = kappa * h;
    for (int q = 0; q < n; ++q) cols[q] = {fd_symbol(c, two_pi * q / n + kh, h), q};
    std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) { return a.l < b.l; });
    const double s0 = 1.0 / std::sqrt((double)n);
    for (int a = 0; a < n; ++a) {
      lam[a] = cols[a].l;
      for (int j = 0; j < n; ++j) {
        long long r = ((long long)cols[a].q * j) % n;
        double ang = two_pi * (double)r / n + kh * j;
        Vre[(size_t)j * n + a] = s0 * std::cos(ang);
        Vim[(size_t)j * n + a] = s0 * std::sin(ang);
      }
    }
    return;
  }
  // Dirichlet: truncated symmetric Toeplitz stencil on n interior nodes.
  std::vector<double> A((size_t)n * n, 0.0);
  const double ih2 = 1.0 / (h * h);
  for (int j = 0; j < n; ++j)
    for (int s = -p; s <= p; ++s) {
      int t = j + s;
      if (t >= 0 && t < n) A[(size_t)j * n + t] += c[std::abs(s)] * ih2;
    }
  std::vector<double> V;
  jacobi_eig(n, A, V);
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    return A[(size_t)a * n + a] < A[(size_t)b * n + b];
  });
  for (int a = 0; a < n; ++a) {
    lam[a] = A[(size_t)idx[a] * n + idx[a]];
    for (int j = 0; j < n; ++j) Vre[(size_t)j * n + a] = V[(size_t)j * n + idx[a]];
  }
}

double kernel_f(double lambda, double omega, bool zero_mode) {
  if (zero_mode) return omega > 0 ? M_PI / (omega * omega) : 0.0;
  if (omega > 0) return 4.0 * M_PI * std::expm1(lambda / (4.0 * omega * omega)) / lambda;
  return -4.0 * M_PI / lambda;
}

void f_table(const std::vector<double> lam[3], double omega, std::vector<double>& f) {
  const size_t n1 = lam[0].size(), n2 = lam[1].size(), n3 = lam[2].size();
  double scale = 0;
  for (int d = 0; d < 3; ++d)
    for (double l : lam[d]) scale = std::max(scale, std::fabs(l));
  scale *= 3.0;
  const double zero_tol = 1e-10 * scale;
  f.resize(n1 * n2 * n3);
  for (size_t c3 = 0; c3 < n3; ++c3)
    for (size_t b = 0; b < n2; ++b)
      for (size_t a = 0; a < n1; ++a) {
        double l = lam[0][a] + lam[1][b] + lam[2][c3];
        f[a + n1 * (b + n2 * c3)] = kernel_f(l, omega, std::fabs(l) <= zero_tol);
      }
}

}  // namespace kx
