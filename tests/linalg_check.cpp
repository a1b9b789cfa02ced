// Host driver for the small dense solvers of the library (csrc/linalg.cpp),
// built with g++ and the address / undefined-behaviour sanitizers by
// tests/test_linalg_host.py.  Reads one problem per line from stdin and writes
// the results on stdout, one line per problem:
//   eig  n a00 a01 ...      -> n pairs "wr wi" (nonsym_eigvals), or "fail"
//   sym  n a00 a01 ...      -> n eigenvalues, then the n x n eigenvector matrix (row-major)
//   solve n a00 ... b0 ...  -> x, or "singular"
//   inv  n lambda a00 ...   -> unit right eigenvector for the real eigenvalue lambda
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../paper_2509_14157_amd/csrc/linalg.hpp"

int main() {
  std::string line;
  std::cout.precision(17);
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string op;
    int n = 0;
    if (!(in >> op >> n) || n < 0) continue;
    double lambda = 0;
    if (op == "inv") in >> lambda;
    std::vector<double> a((size_t)n * n);
    for (auto& x : a) in >> x;
    if (op == "eig") {
      std::vector<double> wr, wi;
      if (!fno::nonsym_eigvals(n, a, wr, wi)) {
        std::cout << "fail\n";
        continue;
      }
      for (int i = 0; i < n; ++i) std::cout << wr[i] << ' ' << wi[i] << ' ';
      std::cout << '\n';
    } else if (op == "sym") {
      std::vector<double> w, v;
      fno::sym_eig(n, a, w, v);
      for (double x : w) std::cout << x << ' ';
      for (double x : v) std::cout << x << ' ';
      std::cout << '\n';
    } else if (op == "solve") {
      std::vector<double> b(n);
      for (auto& x : b) in >> x;
      if (!fno::solve(n, a, b)) {
        std::cout << "singular\n";
        continue;
      }
      for (double x : b) std::cout << x << ' ';
      std::cout << '\n';
    } else if (op == "inv") {
      std::vector<double> x;
      fno::inverse_iteration(n, a, lambda, x);
      for (double y : x) std::cout << y << ' ';
      std::cout << '\n';
    }
  }
  return 0;
}
