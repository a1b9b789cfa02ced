// Small dense FP64 linear algebra on the host (sizes <= a few hundred).
//
// * symmetric eigenproblem: cyclic Jacobi rotations (Golub & Van Loan, 8.5)
// * nonsymmetric eigenvalues: Householder reduction to upper Hessenberg form
//   (GVL Algorithm 7.4.2) followed by the Francis implicit double-shift QR
//   iteration (GVL Algorithms 7.5.1 and 7.5.2)
// * eigenvectors of selected eigenvalues: inverse iteration (real or complex shift)
// * linear systems: Gaussian elimination with partial pivoting
#include "linalg.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>

namespace fno {

void sym_eig(int n, std::vector<double> a, std::vector<double>& w, std::vector<double>& v) {
  // a: n x n row-major symmetric; on return w ascending, v columns = eigenvectors
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  auto V = [&](int i, int j) -> double& { return v[(size_t)i * n + j]; };
  double scale = 0;
  for (double x : a) scale = std::max(scale, std::fabs(x));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A(p, q) * A(p, q);
    if (off <= 1e-32 * std::max(scale * scale, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A(q, q) - A(p, p)) / (2 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * vkq;
          V(k, q) = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  w.resize(n);
  std::vector<double> v2((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    w[j] = A(idx[j], idx[j]);
    for (int i = 0; i < n; ++i) v2[(size_t)i * n + j] = V(i, idx[j]);
  }
  v = v2;
}

bool solve(int n, std::vector<double> a, std::vector<double>& b) {
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A(r, c)) > std::fabs(A(p, c))) p = r;
    if (std::fabs(A(p, c)) < 1e-300) return false;
    if (p != c) {
      for (int k = 0; k < n; ++k) std::swap(A(p, k), A(c, k));
      std::swap(b[p], b[c]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A(r, c) / A(c, c);
      if (f == 0) continue;
      for (int k = c; k < n; ++k) A(r, k) -= f * A(c, k);
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A(r, k) * b[k];
    b[r] = s / A(r, r);
  }
  return true;
}

// ---- nonsymmetric eigenvalues
static void hessenberg(int n, std::vector<double>& a) {
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  for (int k = 0; k < n - 2; ++k) {
    double alpha = 0;
    for (int i = k + 1; i < n; ++i) alpha += A(i, k) * A(i, k);
    alpha = std::sqrt(alpha);
    if (alpha < 1e-300) continue;
    if (A(k + 1, k) > 0) alpha = -alpha;
    std::vector<double> u(n, 0.0);
    u[k + 1] = A(k + 1, k) - alpha;
    for (int i = k + 2; i < n; ++i) u[i] = A(i, k);
    double un = 0;
    for (int i = k + 1; i < n; ++i) un += u[i] * u[i];
    if (un < 1e-300) continue;
    // A = (I - 2uu'/u'u) A (I - 2uu'/u'u)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int i = k + 1; i < n; ++i) s += u[i] * A(i, j);
      s = 2 * s / un;
      for (int i = k + 1; i < n; ++i) A(i, j) -= s * u[i];
    }
    for (int i = 0; i < n; ++i) {
      double s = 0;
      for (int j = k + 1; j < n; ++j) s += A(i, j) * u[j];
      s = 2 * s / un;
      for (int j = k + 1; j < n; ++j) A(i, j) -= s * u[j];
    }
    for (int i = k + 2; i < n; ++i) A(i, k) = 0.0;
  }
}

// Eigenvalues of the 2 x 2 block [[a, b], [c, d]].
static void eig2x2(double a, double b, double c, double d, double& r1, double& i1, double& r2, double& i2) {
  const double mean = 0.5 * (a + d), half = 0.5 * (a - d);
  const double disc = half * half + b * c;
  if (disc >= 0) {
    // the root of larger magnitude first, the other from the determinant
    // (no cancellation between mean and the square root)
    const double root = std::sqrt(disc);
    const double big = mean + (mean >= 0 ? root : -root);
    const double det = a * d - b * c;
    r1 = big;
    r2 = big != 0 ? det / big : mean - root;
    i1 = i2 = 0;
  } else {
    r1 = r2 = mean;
    i1 = std::sqrt(-disc);
    i2 = -i1;
  }
}

// Householder reflector P = I - beta v v^T with v[0] = 1 that maps x (length
// 2 or 3) onto a multiple of e1; returns beta (0 when x is already e1-aligned).
static double house(int len, const double* xin, double* v) {
  // P does not depend on the scale of x: work with x / max|x_i|
  double amax = 0, x[3];
  for (int i = 0; i < len; ++i) amax = std::max(amax, std::fabs(xin[i]));
  v[0] = 1;
  for (int i = 1; i < len; ++i) v[i] = 0;
  if (amax == 0) return 0;
  for (int i = 0; i < len; ++i) x[i] = xin[i] / amax;
  double sigma = 0;
  for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
  for (int i = 1; i < len; ++i) v[i] = x[i];
  if (sigma == 0) return 0;
  const double mu = std::sqrt(x[0] * x[0] + sigma);
  // v0 = x0 - mu, written without cancellation for x0 > 0
  const double v0 = x[0] <= 0 ? x[0] - mu : -sigma / (x[0] + mu);
  const double beta = 2 * v0 * v0 / (sigma + v0 * v0);
  for (int i = 1; i < len; ++i) v[i] /= v0;
  return beta;
}

// One Francis double-shift QR step (GVL Algorithm 7.5.1) on the unreduced
// Hessenberg window lo..hi, with the shifts given by their sum s and product t.
// Only the window is updated: eigenvalues need nothing outside it.
static void francis_step(int n, std::vector<double>& a, int lo, int hi, double s, double t) {
  auto H = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  // first column of (H - s1 I)(H - s2 I) = H^2 - s H + t I, three entries
  double x[3] = {H(lo, lo) * H(lo, lo) + H(lo, lo + 1) * H(lo + 1, lo) - s * H(lo, lo) + t,
                 H(lo + 1, lo) * (H(lo, lo) + H(lo + 1, lo + 1) - s), H(lo + 1, lo) * H(lo + 2, lo + 1)};
  double v[3];
  for (int k = lo; k <= hi - 2; ++k) {
    // chase the bulge: reflect rows/columns k..k+2
    const double beta = house(3, x, v);
    if (beta != 0) {
      const int c0 = std::max(lo, k - 1);
      for (int j = c0; j <= hi; ++j) {
        const double w = beta * (H(k, j) + v[1] * H(k + 1, j) + v[2] * H(k + 2, j));
        H(k, j) -= w;
        H(k + 1, j) -= w * v[1];
        H(k + 2, j) -= w * v[2];
      }
      const int r1 = std::min(k + 3, hi);
      for (int i = lo; i <= r1; ++i) {
        const double w = beta * (H(i, k) + v[1] * H(i, k + 1) + v[2] * H(i, k + 2));
        H(i, k) -= w;
        H(i, k + 1) -= w * v[1];
        H(i, k + 2) -= w * v[2];
      }
    }
    x[0] = H(k + 1, k);
    x[1] = H(k + 2, k);
    x[2] = k + 3 <= hi ? H(k + 3, k) : 0.0;
  }
  // the last reflector acts on two rows/columns
  const double beta = house(2, x, v);
  if (beta != 0) {
    for (int j = hi - 2; j <= hi; ++j) {
      if (j < lo) continue;
      const double w = beta * (H(hi - 1, j) + v[1] * H(hi, j));
      H(hi - 1, j) -= w;
      H(hi, j) -= w * v[1];
    }
    for (int i = lo; i <= hi; ++i) {
      const double w = beta * (H(i, hi - 1) + v[1] * H(i, hi));
      H(i, hi - 1) -= w;
      H(i, hi) -= w * v[1];
    }
  }
  // the bulge chase leaves round-off below the subdiagonal: clear it
  for (int i = lo + 2; i <= hi; ++i)
    for (int j = lo; j < i - 1; ++j) H(i, j) = 0;
}

// Practical QR (GVL Algorithm 7.5.2): deflate at negligible subdiagonal
// entries, read eigenvalues off 1 x 1 and 2 x 2 diagonal blocks, and apply
// Francis steps to the trailing unreduced window.  Shifts are the eigenvalues
// of the window's trailing 2 x 2 block; every tenth step without a split uses
// a complex pair of modulus |h_nn| + |h_(n,n-1)| instead (a different angle
// each time), which breaks the cycles the standard shifts can fall into
// (e.g. on cyclic permutation matrices, where they are exactly zero).
static bool nonsym_eigvals_unit(int n, std::vector<double>& a, std::vector<double>& wr, std::vector<double>& wi) {
  hessenberg(n, a);
  auto H = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  wr.assign(n, 0.0);
  wi.assign(n, 0.0);
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0;
  for (double x : a) anorm = std::max(anorm, std::fabs(x));
  int hi = n - 1, stuck = 0, steps = 0;
  while (hi >= 0) {
    // lo: start of the unreduced window that ends at hi
    int lo = hi;
    while (lo > 0) {
      double scale = std::fabs(H(lo - 1, lo - 1)) + std::fabs(H(lo, lo));
      if (scale == 0) scale = anorm;
      if (std::fabs(H(lo, lo - 1)) <= eps * scale) {
        H(lo, lo - 1) = 0;
        break;
      }
      --lo;
    }
    if (lo == hi) {  // a 1 x 1 block
      wr[hi] = H(hi, hi);
      wi[hi] = 0;
      hi -= 1;
      stuck = 0;
      continue;
    }
    if (lo == hi - 1) {  // a 2 x 2 block
      eig2x2(H(hi - 1, hi - 1), H(hi - 1, hi), H(hi, hi - 1), H(hi, hi), wr[hi - 1], wi[hi - 1], wr[hi], wi[hi]);
      hi -= 2;
      stuck = 0;
      continue;
    }
    if (++steps > 100 * n + 1000) return false;
    ++stuck;
    double s, t;
    if (stuck % 10 == 0) {
      // a complex pair of modulus |h_nn| + |h_(n,n-1)| at an angle that
      // changes with every exceptional step
      const double rho = std::fabs(H(hi, hi)) + std::fabs(H(hi, hi - 1));
      const double angle = 1.1 + 0.37 * (stuck / 10);
      s = 2 * rho * std::cos(angle);
      t = rho * rho;
    } else {
      const double p = H(hi - 1, hi - 1), q = H(hi - 1, hi), r = H(hi, hi - 1), u = H(hi, hi);
      s = p + u;
      t = p * u - q * r;
    }
    francis_step(n, a, lo, hi, s, t);
  }
  return true;
}

bool nonsym_eigvals(int n, std::vector<double> a, std::vector<double>& wr, std::vector<double>& wi) {
  // eigenvalues scale with the matrix: work at unit scale (no under- or
  // overflow in the squares of the shift polynomial) and scale back
  double amax = 0;
  for (double x : a) amax = std::max(amax, std::fabs(x));
  if (!std::isfinite(amax)) return false;
  const double unit = amax > 0 ? amax : 1.0;
  for (double& x : a) x /= unit;
  const bool ok = nonsym_eigvals_unit(n, a, wr, wi);
  for (int i = 0; i < (int)wr.size(); ++i) {
    wr[i] *= unit;
    wi[i] *= unit;
  }
  return ok;
}

void inverse_iteration(int n, const std::vector<double>& a, double lambda, std::vector<double>& x) {
  // (A - (lambda + eps) I) x_new = x_old, a few steps from a fixed start vector
  double scale = 0;
  for (double v : a) scale = std::max(scale, std::fabs(v));
  double shift = lambda + 1e-10 * std::max(scale, 1.0);
  std::vector<double> m(a);
  for (int i = 0; i < n; ++i) m[(size_t)i * n + i] -= shift;
  x.assign(n, 0.0);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.01 * i;
  for (int it = 0; it < 4; ++it) {
    std::vector<double> b = x;
    if (!solve(n, m, b)) {
      // exactly singular: perturb the shift
      for (int i = 0; i < n; ++i) m[(size_t)i * n + i] -= 1e-12 * std::max(scale, 1.0);
      continue;
    }
    double nrm = 0;
    for (double v : b) nrm += v * v;
    nrm = std::sqrt(nrm);
    if (nrm == 0) break;
    for (int i = 0; i < n; ++i) x[i] = b[i] / nrm;
  }
}

bool solve_c(int n, std::vector<std::complex<double>> a, std::vector<std::complex<double>>& b) {
  auto A = [&](int i, int j) -> std::complex<double>& { return a[(size_t)i * n + j]; };
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A(r, c)) > std::abs(A(p, c))) p = r;
    if (std::abs(A(p, c)) < 1e-300) return false;
    if (p != c) {
      for (int k = 0; k < n; ++k) std::swap(A(p, k), A(c, k));
      std::swap(b[p], b[c]);
    }
    for (int r = c + 1; r < n; ++r) {
      const std::complex<double> f = A(r, c) / A(c, c);
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A(r, k) -= f * A(c, k);
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    std::complex<double> s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A(r, k) * b[k];
    b[r] = s / A(r, r);
  }
  return true;
}

void inverse_iteration_c(int n, const std::vector<double>& a, std::complex<double> lambda,
                         std::vector<std::complex<double>>& x) {
  double scale = 0;
  for (double v : a) scale = std::max(scale, std::fabs(v));
  const std::complex<double> shift = lambda + 1e-10 * std::max(scale, 1.0);
  std::vector<std::complex<double>> m(a.begin(), a.end());
  for (int i = 0; i < n; ++i) m[(size_t)i * n + i] -= shift;
  x.assign(n, 0.0);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.01 * i;
  for (int it = 0; it < 4; ++it) {
    std::vector<std::complex<double>> b = x;
    if (!solve_c(n, m, b)) {
      for (int i = 0; i < n; ++i) m[(size_t)i * n + i] -= 1e-12 * std::max(scale, 1.0);
      continue;
    }
    double nrm = 0;
    for (auto v : b) nrm += std::norm(v);
    nrm = std::sqrt(nrm);
    if (nrm == 0) break;
    for (int i = 0; i < n; ++i) x[i] = b[i] / nrm;
  }
}

}  // namespace fno
