// Small dense host linear algebra used by the solvers.
#pragma once
#include <complex>
#include <vector>

namespace fno {
// Symmetric eigenproblem of the n x n row-major matrix a: ascending w, columns of v.
void sym_eig(int n, std::vector<double> a, std::vector<double>& w, std::vector<double>& v);
// Solve a x = b in place (b <- x); false when singular.
bool solve(int n, std::vector<double> a, std::vector<double>& b);
// Eigenvalues (real, imaginary parts) of a real nonsymmetric matrix.
bool nonsym_eigvals(int n, std::vector<double> a, std::vector<double>& wr, std::vector<double>& wi);
// Right eigenvector of a for the (real) eigenvalue lambda, unit 2-norm.
void inverse_iteration(int n, const std::vector<double>& a, double lambda, std::vector<double>& x);
// Complex versions: solve in place, and the right eigenvector of a real matrix
// for a complex eigenvalue (unit 2-norm).
bool solve_c(int n, std::vector<std::complex<double>> a, std::vector<std::complex<double>>& b);
void inverse_iteration_c(int n, const std::vector<double>& a, std::complex<double> lambda,
                         std::vector<std::complex<double>>& x);
}  // namespace fno
