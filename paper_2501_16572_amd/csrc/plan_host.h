// Host-side FP64 tables of the Kronecker-product plan (no device code).
#pragma once
#include <vector>

namespace kx {

// Weights c_0..c_p of the central 2p-th order second derivative.
std::vector<double> fd_weights(int order);

// Eigenpairs of the 1D second-derivative operator, ascending eigenvalues;
// V[k*n + a] is component k of eigenvector a.  bc: 0 periodic, 1 Dirichlet.
// kappa: Bloch wavevector (periodic only); Vim is all zero when the basis is
// real (periodic at kappa = 0, Dirichlet).
void eig1d(int n, double h, int bc, int order, double kappa, std::vector<double>& lam,
           std::vector<double>& Vre, std::vector<double>& Vim);

// The scalar kernel of Eq. (fL) (screened reading: erfc(omega r)/r).
double kernel_f(double lambda, double omega, bool zero_mode);

// f(lam1[a] + lam2[b] + lam3[c]) at flat index a + n1 (b + n2 c); sums whose
// magnitude is below 1e-10 of the largest possible are the zero mode.
void f_table(const std::vector<double> lam[3], double omega, std::vector<double>& f);

}  // namespace kx
