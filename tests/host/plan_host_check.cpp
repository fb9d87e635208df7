// Host driver for the sanitizer build of the plan's FP64 tables (CPU test).
// Runs fd_weights, eig1d and f_table over the boundary conditions, Bloch
// vectors, axis lengths (1 up to the 160-point limit) and FD orders the
// library accepts, and checks the results it can check without a reference:
// V unitary, D V = V diag(lam) for the operator rebuilt from the weights,
// ascending eigenvalues, finite f.  Exit status 0 when every check passes.
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "plan_host.h"

using cd = std::complex<double>;

// (D v)(j) for the 1D operator: periodic wrap with Bloch phase e^{i kappa n h}
// per wrap, or zero ghosts (Dirichlet).
static cd apply_d(const std::vector<double>& c, int n, double h, int bc, double kappa,
                  const std::vector<cd>& v, int j) {
  const int p = (int)c.size() - 1;
  cd acc = 0;
  for (int s = -p; s <= p; ++s) {
    int k = j + s;
    cd ph = 1;
    if (bc == 1) {
      if (k < 0 || k >= n) continue;
    } else {
      int wraps = (int)std::floor((double)k / n);
      k -= wraps * n;
      ph = std::exp(cd(0, kappa * n * h * wraps));
    }
    acc += c[std::abs(s)] * ph * v[k];
  }
  return acc / (h * h);
}

int main() {
  int bad = 0;
  const int ns[] = {1, 2, 3, 5, 12, 13, 25, 72, 160};
  const int orders[] = {2, 12, 16};
  for (int order : orders)
    for (int n : ns)
      for (int bc = 0; bc < 2; ++bc)
        for (double kappa : {0.0, 0.37, -1.2}) {
          if (bc == 1 && kappa != 0.0) continue;
          const double h = 0.3;
          std::vector<double> lam, vr, vi;
          kx::eig1d(n, h, bc, order, kappa, lam, vr, vi);
          if ((int)lam.size() != n || vr.size() != (size_t)n * n || vi.size() != (size_t)n * n) {
            std::printf("size n=%d bc=%d\n", n, bc);
            ++bad;
            continue;
          }
          const std::vector<double> c = kx::fd_weights(order);
          // the operator's norm is at most 4 sum|c_s| / h^2 (n = 1: the only
          // eigenvalue is the rounding of the zero stencil sum)
          double scale = 0, res = 0, orth = 0;
          for (size_t s = 0; s < c.size(); ++s) scale += 2 * std::fabs(c[s]) / (h * h);
          for (double l : lam) scale = std::fmax(scale, std::fabs(l));
          for (int a = 0; a < n; ++a) {
            std::vector<cd> v(n);
            for (int k = 0; k < n; ++k) v[k] = cd(vr[(size_t)k * n + a], vi[(size_t)k * n + a]);
            for (int j = 0; j < n; ++j) res = std::fmax(res, std::abs(apply_d(c, n, h, bc, kappa, v, j) - lam[a] * v[j]));
            for (int b = 0; b < n; ++b) {
              cd dot = 0;
              for (int k = 0; k < n; ++k) dot += std::conj(v[k]) * cd(vr[(size_t)k * n + b], vi[(size_t)k * n + b]);
              orth = std::fmax(orth, std::abs(dot - (a == b ? 1.0 : 0.0)));
            }
            if (a > 0 && lam[a] < lam[a - 1] - 1e-12 * scale) ++bad;
          }
          if (res > 1e-10 * scale || orth > 1e-12) {
            std::printf("n=%d bc=%d kappa=%g order=%d: residual %.3e (scale %.3e), orthogonality %.3e\n", n, bc,
                        kappa, order, res, scale, orth);
            ++bad;
          }
        }
  // f over small 3D grids, both kernels, periodic (zero mode) and Dirichlet
  for (double omega : {0.0, 0.106, 0.5})
    for (int bc = 0; bc < 2; ++bc) {
      std::vector<double> lam[3], vr, vi;
      const int n3[3] = {1, 4, 7};
      for (int d = 0; d < 3; ++d) kx::eig1d(n3[d], 0.25, bc, 12, 0.0, lam[d], vr, vi);
      std::vector<double> f;
      kx::f_table(lam, omega, f);
      if (f.size() != 28) ++bad;
      for (double x : f)
        if (!std::isfinite(x) || x < 0) ++bad;
    }
  std::printf("%s\n", bad ? "FAILED" : "OK");
  return bad ? 1 : 0;
}
