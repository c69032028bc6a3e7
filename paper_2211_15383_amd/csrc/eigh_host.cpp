// Dense Hermitian eigensolvers and Cholesky for the Rayleigh-Ritz steps of the
// eigensolvers (host, FP64).
// eigh_jacobi: cyclic complex Jacobi: each off-diagonal entry h = |h| e^{i phi} is first
// made real by the diagonal unitary diag(1, e^{-i phi}) on (p, q), then annihilated by
// the classical real Jacobi rotation (tan 2 theta = 2 |h| / (a_qq - a_pp)); O(n^3) per
// sweep with strided column updates, for small orders.
// eigh_tridiag: Householder reduction to a Hermitian tridiagonal matrix, a diagonal
// unitary that makes its off-diagonal real and non-negative, the implicit QL iteration
// with Wilkinson shifts on the real tridiagonal (Givens rotations accumulated into the
// eigenvectors), and the back-transformation; about 20 n^3 real flops in all, with
// contiguous inner loops, for the Rayleigh-Ritz matrices of order up to a few thousand.
#include "eigh_host.h"

#include <algorithm>
#include <cmath>
#include <thread>

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

// ---------------------------------------------------------------- Householder + QL
namespace {

// f(begin, end) over [0, n) split into contiguous chunks on up to 16 threads (each index
// is handled by exactly one thread in a fixed order, so results do not depend on the
// thread count)
template <class F>
void par_for(int n, int min_chunk, F f) {
  int T = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
  T = std::min(T, std::max(1, n / std::max(1, min_chunk)));
  if (T <= 1) {
    f(0, n);
    return;
  }
  const int chunk = (n + T - 1) / T;
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) {
    const int b = t * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back(f, b, e);
  }
  f(0, std::min(n, chunk));
  for (auto& x : th) x.join();
}

}  // namespace

int eigh_tridiag(int n, std::vector<std::complex<double>> A, std::vector<double>& w,
                 std::vector<std::complex<double>>& Z) {
  using cd = std::complex<double>;
  w.assign(n, 0.0);
  Z.assign((size_t)n * n, cd(0.0, 0.0));
  if (n == 0) return 0;
  // Hermitian from the upper triangle
  for (int i = 0; i < n; ++i) {
    at(A, n, i, i) = cd(at(A, n, i, i).real(), 0.0);
    for (int j = i + 1; j < n; ++j) at(A, n, j, i) = std::conj(at(A, n, i, j));
  }
  // complex entries as (re, im) double pairs in the inner loops
  double* a = reinterpret_cast<double*>(A.data());
  // 1. reduction: step k maps column k below the diagonal, x = A[k+1.., k], to alpha e_1
  //    with the reflector H_k = I - 2 v v^H (|v| = 1) acting on indices k+1..n-1
  std::vector<cd> hv((size_t)n * n, cd(0.0, 0.0));  // row k: v of step k at k+1..n-1
  std::vector<cd> sub(n, cd(0.0, 0.0));              // sub[i] = T[i+1][i]
  std::vector<cd> p(n), wv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    cd* v = &hv[(size_t)k * n + k + 1];
    double xn = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = std::conj(at(A, n, k, k + 1 + i));  // A[k+1+i][k] (Hermitian)
      xn += std::norm(v[i]);
    }
    xn = std::sqrt(xn);
    if (xn == 0.0) {
      for (int i = 0; i < m; ++i) v[i] = 0.0;
      sub[k] = 0.0;
      continue;
    }
    const double a0 = std::abs(v[0]);
    const cd ph = a0 > 0.0 ? v[0] / a0 : cd(1.0, 0.0);
    const cd alpha = -ph * xn;
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < m; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    for (int i = 0; i < m; ++i) v[i] /= vn;
    const double* vd = reinterpret_cast<const double*>(v);
    // p = A_sub v
    par_for(m, 64, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        const double* row = a + 2 * ((size_t)(k + 1 + i) * n + k + 1);
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < m; ++j) {
          sr += row[2 * j] * vd[2 * j] - row[2 * j + 1] * vd[2 * j + 1];
          si += row[2 * j] * vd[2 * j + 1] + row[2 * j + 1] * vd[2 * j];
        }
        p[i] = cd(sr, si);
      }
    });
    // beta = v^H p (real), w = 2 p - 2 beta v
    double beta = 0.0;
    for (int i = 0; i < m; ++i) beta += (std::conj(v[i]) * p[i]).real();
    for (int i = 0; i < m; ++i) wv[i] = 2.0 * p[i] - 2.0 * beta * v[i];
    const double* wd = reinterpret_cast<const double*>(wv.data());
    // A_sub -= v w^H + w v^H
    par_for(m, 64, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        double* row = a + 2 * ((size_t)(k + 1 + i) * n + k + 1);
        const double vr = vd[2 * i], vi = vd[2 * i + 1], wr = wd[2 * i], wi = wd[2 * i + 1];
        for (int j = 0; j < m; ++j) {
          // v_i conj(w_j) + w_i conj(v_j)
          const double xr = wd[2 * j], xi = wd[2 * j + 1], yr = vd[2 * j], yi = vd[2 * j + 1];
          row[2 * j] -= vr * xr + vi * xi + wr * yr + wi * yi;
          row[2 * j + 1] -= vi * xr - vr * xi + wi * yr - wr * yi;
        }
      }
    });
    sub[k] = alpha;
  }
  if (n >= 2) sub[n - 2] = std::conj(at(A, n, n - 2, n - 1));
  // 2. real tridiagonal: T = D T' D^H with D = diag(delta), delta_0 = 1,
  //    delta_{i+1} = delta_i sub_i / |sub_i|, so that T'[i+1][i] = |sub_i|
  std::vector<double> d(n), e(n, 0.0);
  std::vector<cd> delta(n, cd(1.0, 0.0));
  for (int i = 0; i < n; ++i) d[i] = at(A, n, i, i).real();
  for (int i = 0; i + 1 < n; ++i) {
    const double aa = std::abs(sub[i]);
    e[i] = aa;
    delta[i + 1] = aa > 0.0 ? delta[i] * (sub[i] / aa) : delta[i];
  }
  // 3. implicit QL with Wilkinson shifts; Vt row i is the eigenvector of T' that ends in d[i]
  std::vector<double> Vt((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Vt[(size_t)i * n + i] = 1.0;
  const double tiny = 2.220446049250313e-16;
  int total = 0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= tiny * dd) break;
      }
      if (m == l) break;
      if (iter >= 200) return -1;  // no convergence (does not happen for finite input)
      ++total;
      // shift from the leading 2 x 2 block at l: the eigenvalue of it closer to d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, shift_acc = 0.0;
      bool deflated = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // an exactly zero rotation splits the matrix here
          d[i + 1] -= shift_acc;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - shift_acc;
        r = (d[i] - g) * s + 2.0 * c * b;
        shift_acc = s * r;
        d[i + 1] = g + shift_acc;
        g = c * r - b;
        double* vi = &Vt[(size_t)i * n];
        double* vj = &Vt[(size_t)(i + 1) * n];
        for (int q = 0; q < n; ++q) {
          const double t = vj[q];
          vj[q] = s * vi[q] + c * t;
          vi[q] = c * vi[q] - s * t;
        }
      }
      if (deflated) continue;
      d[l] -= shift_acc;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // 4. ascending order; eigenvector j of A = H_0 ... H_{n-3} D (row of Vt), blocks of
  //    eigenvectors run through all reflectors while they stay in cache
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int jj = 0; jj < n; ++jj) w[jj] = d[idx[jj]];
  std::vector<cd> Y((size_t)n * n);  // row jj: eigenvector jj
  constexpr int EB = 32;
  const int nblk = (n + EB - 1) / EB;
  par_for(nblk, 1, [&](int b0, int b1) {
    for (int blk = b0; blk < b1; ++blk) {
      const int j0 = blk * EB, j1 = std::min(n, j0 + EB);
      for (int jj = j0; jj < j1; ++jj) {
        const double* vr = &Vt[(size_t)idx[jj] * n];
        cd* y = &Y[(size_t)jj * n];
        for (int i = 0; i < n; ++i) y[i] = delta[i] * vr[i];
      }
      for (int k = n - 3; k >= 0; --k) {
        const double* v = reinterpret_cast<const double*>(&hv[(size_t)k * n + k + 1]);
        const int m = n - k - 1;
        for (int jj = j0; jj < j1; ++jj) {
          double* y = reinterpret_cast<double*>(&Y[(size_t)jj * n + k + 1]);
          double dr = 0.0, di = 0.0;  // v^H y
          for (int i = 0; i < m; ++i) {
            dr += v[2 * i] * y[2 * i] + v[2 * i + 1] * y[2 * i + 1];
            di += v[2 * i] * y[2 * i + 1] - v[2 * i + 1] * y[2 * i];
          }
          if (dr == 0.0 && di == 0.0) continue;
          dr *= 2.0;
          di *= 2.0;
          for (int i = 0; i < m; ++i) {  // y -= 2 (v^H y) v
            y[2 * i] -= dr * v[2 * i] - di * v[2 * i + 1];
            y[2 * i + 1] -= dr * v[2 * i + 1] + di * v[2 * i];
          }
        }
      }
    }
  });
  for (int jj = 0; jj < n; ++jj)
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + jj] = Y[(size_t)jj * n + i];
  return total;
}
