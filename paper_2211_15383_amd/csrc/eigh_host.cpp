// Small dense Hermitian eigensolver and Cholesky for the Rayleigh-Ritz steps of the
// coarsest-level eigensolver (matrices of order <= a few hundred, host, FP64).
// Cyclic complex Jacobi: each off-diagonal entry h = |h| e^{i phi} is first made real by
// the diagonal unitary diag(1, e^{-i phi}) on (p, q), then annihilated by the classical
// real Jacobi rotation (tan 2 theta = 2 |h| / (a_qq - a_pp)).
#include "eigh_host.h"

#include <algorithm>
#include <cmath>

namespace {
inline std::complex<double>& at(std::vector<std::complex<double>>& A, int n, int i, int j) { return A[(size_t)i * n + j]; }
}  // namespace

// A: n x n Hermitian, row-major; on return w holds eigenvalues (ascending) and Z the
// eigenvectors as columns (row-major n x n).  Returns the number of sweeps used.
int eigh_jacobi(int n, std::vector<std::complex<double>> A, std::vector<double>& w,
                std::vector<std::complex<double>>& Z) {
  using cd = std::complex<double>;
  Z.assign((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) at(Z, n, i, i) = 1.0;
  // symmetrise (use the upper triangle as the definition)
  for (int i = 0; i < n; ++i) {
    at(A, n, i, i) = cd(at(A, n, i, i).real(), 0.0);
    for (int j = i + 1; j < n; ++j) at(A, n, j, i) = std::conj(at(A, n, i, j));
  }
  double fro = 0.0;
  for (auto& v : A) fro += std::norm(v);
  fro = std::sqrt(fro);
  int sweep = 0;
  for (; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += std::norm(at(A, n, i, j));
    if (std::sqrt(2.0 * off) <= 1e-15 * fro || fro == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const cd h = at(A, n, p, q);
        const double g = std::abs(h);
        if (g <= 1e-300) continue;
        const cd e = h / g;  // e^{i phi}
        // A <- E^H A E with E = diag(1, conj(e)) on q: column q *= conj(e), row q *= e
        for (int k = 0; k < n; ++k) {
          at(A, n, k, q) *= std::conj(e);
          at(A, n, q, k) *= e;
        }
        for (int k = 0; k < n; ++k) at(Z, n, k, q) *= std::conj(e);
        const double a = at(A, n, p, p).real(), b = at(A, n, q, q).real();
        const double theta = (b - a) / (2.0 * g);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // rotation on columns p, q: [p', q'] = [p, q] [[c, s], [-s, c]]
        for (int k = 0; k < n; ++k) {
          const cd akp = at(A, n, k, p), akq = at(A, n, k, q);
          at(A, n, k, p) = c * akp - s * akq;
          at(A, n, k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const cd apk = at(A, n, p, k), aqk = at(A, n, q, k);
          at(A, n, p, k) = c * apk - s * aqk;
          at(A, n, q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const cd zkp = at(Z, n, k, p), zkq = at(Z, n, k, q);
          at(Z, n, k, p) = c * zkp - s * zkq;
          at(Z, n, k, q) = s * zkp + c * zkq;
        }
        at(A, n, p, q) = at(A, n, q, p) = cd(0.0, 0.0);
      }
    }
  }
  // sort ascending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int i, int j) { return at(A, n, i, i).real() < at(A, n, j, j).real(); });
  w.resize(n);
  std::vector<cd> Zs((size_t)n * n);
  for (int jj = 0; jj < n; ++jj) {
    w[jj] = at(A, n, idx[jj], idx[jj]).real();
    for (int k = 0; k < n; ++k) Zs[(size_t)k * n + jj] = at(Z, n, k, idx[jj]);
  }
  Z.swap(Zs);
  return sweep;
}

// Lower Cholesky factor of a Hermitian positive definite matrix (row-major, in place);
// returns false when a pivot is not positive.
bool cholesky_lower(int n, std::vector<std::complex<double>>& A) {
  using cd = std::complex<double>;
  for (int j = 0; j < n; ++j) {
    double d = at(A, n, j, j).real();
    for (int k = 0; k < j; ++k) d -= std::norm(at(A, n, j, k));
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    at(A, n, j, j) = ljj;
    for (int i = j + 1; i < n; ++i) {
      cd s = at(A, n, i, j);
      for (int k = 0; k < j; ++k) s -= at(A, n, i, k) * std::conj(at(A, n, j, k));
      at(A, n, i, j) = s / ljj;
    }
    for (int k = j + 1; k < n; ++k) at(A, n, j, k) = 0.0;
  }
  return true;
}

// Inverse of a lower-triangular matrix (row-major, in place).
void lower_inverse(int n, std::vector<std::complex<double>>& Lm) {
  using cd = std::complex<double>;
  std::vector<cd> I((size_t)n * n, cd(0.0, 0.0));
  for (int j = 0; j < n; ++j) {
    I[(size_t)j * n + j] = 1.0 / Lm[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      cd s = 0.0;
      for (int k = j; k < i; ++k) s += Lm[(size_t)i * n + k] * I[(size_t)k * n + j];
      I[(size_t)i * n + j] = -s / Lm[(size_t)i * n + i];
    }
  }
  Lm.swap(I);
}
