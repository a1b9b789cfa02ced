// Small dense FP64 linear algebra on the host (sizes <= a few hundred).
//
// * symmetric eigenproblem: cyclic Jacobi rotations (Golub & Van Loan, 8.5)
// * nonsymmetric eigenvalues: Householder reduction to upper Hessenberg form
//   followed by the Francis implicit double-shift QR iteration (GVL 7.5)
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

bool nonsym_eigvals(int n, std::vector<double> a, std::vector<double>& wr, std::vector<double>& wi) {
  hessenberg(n, a);
  auto H = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  wr.assign(n, 0.0);
  wi.assign(n, 0.0);
  double norm = 0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(i - 1, 0); j < n; ++j) norm += std::fabs(H(i, j));
  int nn = n - 1;
  double t = 0;
  int total_its = 0;
  while (nn >= 0) {
    int its = 0, l;
    do {
      // look for a small subdiagonal element
      for (l = nn; l >= 1; --l) {
        double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
        if (s == 0) s = norm;
        if (std::fabs(H(l, l - 1)) <= std::numeric_limits<double>::epsilon() * s) {
          H(l, l - 1) = 0;
          break;
        }
      }
      double x = H(nn, nn);
      if (l == nn) {  // one root
        wr[nn] = x + t;
        wi[nn] = 0;
        --nn;
      } else {
        double y = H(nn - 1, nn - 1);
        double w = H(nn, nn - 1) * H(nn - 1, nn);
        if (l == nn - 1) {  // two roots
          double p = 0.5 * (y - x);
          double q = p * p + w;
          double z = std::sqrt(std::fabs(q));
          x += t;
          if (q >= 0) {
            z = p + (p >= 0 ? std::fabs(z) : -std::fabs(z));
            wr[nn - 1] = wr[nn] = x + z;
            if (z != 0) wr[nn] = x - w / z;
            wi[nn - 1] = wi[nn] = 0;
          } else {
            wr[nn - 1] = wr[nn] = x + p;
            wi[nn - 1] = -(wi[nn] = z);
          }
          nn -= 2;
        } else {  // double-shift QR step on the active block l..nn
          if (its == 60 || ++total_its > 100000) return false;
          if (its == 10 || its == 20) {  // exceptional shift
            t += x;
            for (int i = 0; i <= nn; ++i) H(i, i) -= x;
            double s = std::fabs(H(nn, nn - 1)) + std::fabs(H(nn - 1, nn - 2));
            y = x = 0.75 * s;
            w = -0.4375 * s * s;
          }
          ++its;
          int m;
          double p = 0, q = 0, r = 0, z;
          for (m = nn - 2; m >= l; --m) {
            z = H(m, m);
            r = x - z;
            double s = y - z;
            p = (r * s - w) / H(m + 1, m) + H(m, m + 1);
            q = H(m + 1, m + 1) - z - r - s;
            r = H(m + 2, m + 1);
            s = std::fabs(p) + std::fabs(q) + std::fabs(r);
            p /= s;
            q /= s;
            r /= s;
            if (m == l) break;
            double u = std::fabs(H(m, m - 1)) * (std::fabs(q) + std::fabs(r));
            double v = std::fabs(p) * (std::fabs(H(m - 1, m - 1)) + std::fabs(z) + std::fabs(H(m + 1, m + 1)));
            if (u <= std::numeric_limits<double>::epsilon() * v) break;
          }
          for (int i = m; i < nn - 1; ++i) {
            H(i + 2, i) = 0;
            if (i != m) H(i + 2, i - 1) = 0;
          }
          for (int k = m; k < nn; ++k) {
            if (k != m) {
              p = H(k, k - 1);
              q = H(k + 1, k - 1);
              r = 0;
              if (k != nn - 1) r = H(k + 2, k - 1);
              if ((x = std::fabs(p) + std::fabs(q) + std::fabs(r)) != 0) {
                p /= x;
                q /= x;
                r /= x;
              }
            }
            double s = std::sqrt(p * p + q * q + r * r);
            if (p < 0) s = -s;
            if (s != 0) {
              if (k == m) {
                if (l != m) H(k, k - 1) = -H(k, k - 1);
              } else {
                H(k, k - 1) = -s * x;
              }
              p += s;
              x = p / s;
              y = q / s;
              z = r / s;
              q /= p;
              r /= p;
              for (int j = k; j <= nn; ++j) {
                p = H(k, j) + q * H(k + 1, j);
                if (k != nn - 1) {
                  p += r * H(k + 2, j);
                  H(k + 2, j) -= p * z;
                }
                H(k + 1, j) -= p * y;
                H(k, j) -= p * x;
              }
              int mmin = nn < k + 3 ? nn : k + 3;
              for (int i = l; i <= mmin; ++i) {
                p = x * H(i, k) + y * H(i, k + 1);
                if (k != nn - 1) {
                  p += z * H(i, k + 2);
                  H(i, k + 2) -= p * r;
                }
                H(i, k + 1) -= p * q;
                H(i, k) -= p;
              }
            }
          }
        }
      }
    } while (l < nn - 1);
  }
  return true;
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
