// Fast diagonalisation of a 1D CFE axis (host, FP64, once per axis shape).
//
// Every directional system of the scheme is (alpha M + beta K) x = b with the
// axis' fixed mass and stiffness matrices and scalars alpha, beta that change
// every sweep.  With the generalised eigenvectors V of (K, M),
//   V^T M V = I,  V^T K V = diag(mu),
// the solve is x = V diag(1 / (alpha + beta mu)) V^T b: two dense products
// that spread over the whole GPU instead of a sequential banded recurrence.
//
// V is formed as L^-T Q from the banded Cholesky factor M = L L^T and the
// eigenvectors Q of C = L^-1 K L^-T, C = Q diag(mu) Q^T.  C is reduced to
// tridiagonal form by Householder reflections (accumulated into Q) and the
// tridiagonal problem is solved by the implicit QL iteration with shifts
// from the leading 2 x 2 block, its plane rotations applied to Q.  Both steps
// are the published methods (Householder reduction of a symmetric matrix to
// tridiagonal form; the QL algorithm with implicit shifts of Bowdler,
// Martin, Reinsch and Wilkinson, Numer. Math. 11 (1968), the procedure
// EISPACK distributes as tql2), written here for this use.
#include "ctd_internal.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace ctd {

namespace {

// Banded Cholesky of the lower band (B+1) x n (row t: A[j+t, j] at t*n + j):
// returns L in the same layout.
bool band_cholesky(int n, int B, const std::vector<double>& A, std::vector<double>& L) {
  L.assign((size_t)(B + 1) * n, 0.0);
  auto at = [&](std::vector<double>& X, int i, int j) -> double& { return X[(size_t)(i - j) * n + j]; };
  for (int j = 0; j < n; ++j) {
    double s = A[j];
    for (int k = std::max(0, j - B); k < j; ++k) s -= at(L, j, k) * at(L, j, k);
    if (!(s > 0.0)) return false;
    const double g = std::sqrt(s);
    at(L, j, j) = g;
    for (int i = j + 1; i <= std::min(n - 1, j + B); ++i) {
      double t = A[(size_t)(i - j) * n + j];
      for (int k = std::max(0, i - B); k < j; ++k) t -= at(L, i, k) * at(L, j, k);
      at(L, i, j) = t / g;
    }
  }
  return true;
}

// Householder reduction of the symmetric n x n matrix C (row-major, both
// triangles) to tridiagonal (d, e: e[i] couples i and i+1); Qt receives the
// transpose of the accumulated orthogonal factor (row k = column k of Q).
void tridiagonalize(int n, std::vector<double>& C, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& Qt) {
  std::vector<std::vector<double>> vs(n > 2 ? n - 2 : 0);
  std::vector<double> p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;            // size of the trailing block
    double* col = &q[0];
    for (int i = 0; i < m; ++i) col[i] = C[(size_t)(k + 1 + i) * n + k];
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += col[i] * col[i];
    nrm = std::sqrt(nrm);
    std::vector<double>& v = vs[k];
    if (nrm == 0.0) continue;
    const double alpha = col[0] > 0 ? -nrm : nrm;
    v.assign(col, col + m);
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < m; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0.0) { v.clear(); continue; }
    for (int i = 0; i < m; ++i) v[i] /= vn;
    // p = A22 v, K = v.p, q = p - K v; A22 -= 2 v q^T + 2 q v^T
    for (int i = 0; i < m; ++i) {
      const double* row = &C[(size_t)(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
    }
    double K = 0.0;
    for (int i = 0; i < m; ++i) K += v[i] * p[i];
    for (int i = 0; i < m; ++i) q[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = &C[(size_t)(k + 1 + i) * n + k + 1];
      const double vi = 2.0 * v[i], qi = 2.0 * q[i];
      for (int j = 0; j < m; ++j) row[j] -= vi * q[j] + qi * v[j];
    }
    C[(size_t)(k + 1) * n + k] = alpha;
    C[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) {
      C[(size_t)(k + 1 + i) * n + k] = 0.0;
      C[(size_t)k * n + k + 1 + i] = 0.0;
    }
  }
  d.assign(n, 0.0);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = C[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = C[(size_t)(i + 1) * n + i];
  // Q = H_0 H_1 ... H_{n-3}, accumulated from the right; Qt = Q^T so that
  // each reflection updates whole rows: Q^T <- Q^T H_k on columns k+1..
  Qt.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Qt[(size_t)i * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    const std::vector<double>& v = vs[k];
    if (v.empty()) continue;
    const int m = n - k - 1;
    // rows r of Q^T with nonzeros in columns k+1.. are r >= k+1
    for (int r = k + 1; r < n; ++r) {
      double* row = &Qt[(size_t)r * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      s *= 2.0;
      for (int j = 0; j < m; ++j) row[j] -= s * v[j];
    }
  }
}

// Implicit QL on the tridiagonal (d, e) (Bowdler, Martin, Reinsch and
// Wilkinson 1968; EISPACK tql2): deflate at the first negligible
// off-diagonal, shift by the eigenvalue of the leading 2 x 2 block nearer its
// corner, chase the bulge with plane rotations; the rotations update the rows
// of Qt (columns of Q).  On return d holds the eigenvalues.
bool tridiag_ql(int n, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Qt) {
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (iter > 80) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double* qa = &Qt[(size_t)i * n];
        double* qb = &Qt[(size_t)(i + 1) * n];
        for (int k = 0; k < n; ++k) {
          const double fa = qa[k], fb = qb[k];
          qb[k] = s * fa + c * fb;
          qa[k] = c * fa - s * fb;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

}  // namespace

bool fast_diag(const AxisTables& T, std::vector<double>& V, std::vector<double>& mu, std::string& err) {
  const int n = T.n, B = T.B;
  std::vector<double> L;
  if (!band_cholesky(n, B, T.Mb, L)) { err = "mass matrix not positive definite"; return false; }
  auto Lat = [&](int i, int j) { return L[(size_t)(i - j) * n + j]; };
  // dense K, then Y = L^-1 K (forward substitution on rows of K^T = K)
  std::vector<double> C((size_t)n * n, 0.0);
  for (int t = 0; t <= B; ++t)
    for (int j = 0; j + t < n; ++j) {
      const double v = T.Kb[(size_t)t * n + j];
      C[(size_t)(j + t) * n + j] = v;
      C[(size_t)j * n + j + t] = v;
    }
  // rows of C: row i of Y = (row i of K - sum_k L[i,k] row k of Y) / L[i,i]
  for (int i = 0; i < n; ++i) {
    double* yi = &C[(size_t)i * n];
    for (int k = std::max(0, i - B); k < i; ++k) {
      const double lik = Lat(i, k);
      const double* yk = &C[(size_t)k * n];
      for (int j = 0; j < n; ++j) yi[j] -= lik * yk[j];
    }
    const double inv = 1.0 / Lat(i, i);
    for (int j = 0; j < n; ++j) yi[j] *= inv;
  }
  // C = Y L^-T: transpose, the same forward substitution, transpose back
  std::vector<double> Yt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Yt[(size_t)j * n + i] = C[(size_t)i * n + j];
  for (int i = 0; i < n; ++i) {
    double* yi = &Yt[(size_t)i * n];
    for (int k = std::max(0, i - B); k < i; ++k) {
      const double lik = Lat(i, k);
      const double* yk = &Yt[(size_t)k * n];
      for (int j = 0; j < n; ++j) yi[j] -= lik * yk[j];
    }
    const double inv = 1.0 / Lat(i, i);
    for (int j = 0; j < n; ++j) yi[j] *= inv;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[(size_t)i * n + j] = 0.5 * (Yt[(size_t)j * n + i] + Yt[(size_t)i * n + j]);
  std::vector<double> d, e, Qt;
  tridiagonalize(n, C, d, e, Qt);
  if (!tridiag_ql(n, d, e, Qt)) { err = "tridiagonal QL did not converge"; return false; }
  // V = L^-T Q: back substitution on rows (row i of V over all eigenvectors)
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) V[(size_t)i * n + k] = Qt[(size_t)k * n + i];
  for (int i = n - 1; i >= 0; --i) {
    double* vi = &V[(size_t)i * n];
    for (int j = i + 1; j <= std::min(n - 1, i + B); ++j) {
      const double lji = Lat(j, i);
      const double* vj = &V[(size_t)j * n];
      for (int k = 0; k < n; ++k) vi[k] -= lji * vj[k];
    }
    const double inv = 1.0 / Lat(i, i);
    for (int k = 0; k < n; ++k) vi[k] *= inv;
  }
  mu = d;
  return true;
}

// Process-wide cache: every axis of the same shape shares one factorisation.
std::shared_ptr<const FastDiag> fast_diag_cached(const AxisTables& T, std::string& err) {
  static std::mutex mu_lock;
  static std::map<std::tuple<int, double, double, int, int, double, int>,
                  std::shared_ptr<const FastDiag>> cache;
  const auto key = std::make_tuple(T.n, T.lo, T.hi, T.s, T.p, T.a, T.ng);
  {
    std::lock_guard<std::mutex> g(mu_lock);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto fd = std::make_shared<FastDiag>();
  if (!fast_diag(T, fd->V, fd->mu, err)) return nullptr;
  std::lock_guard<std::mutex> g(mu_lock);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  cache[key] = fd;
  return fd;
}

}  // namespace ctd

extern "C" int ctd_axis_fast_diag(int64_t n, double lo, double hi, int32_t s, int32_t p, double a,
                                  int32_t ng, double* V, double* mu) {
  if (!V || !mu) return CTD_EINVAL;
  ctd::AxisTables T;
  std::string err;
  int rc = ctd::build_axis(n, lo, hi, s, p, a == 0.0 ? 12.0 : a, ng == 0 ? 5 : ng, T, err);
  if (rc) return rc;
  std::vector<double> Vv, m;
  if (!ctd::fast_diag(T, Vv, m, err)) return CTD_EUNSUPPORTED;
  std::copy(Vv.begin(), Vv.end(), V);
  std::copy(m.begin(), m.end(), mu);
  return CTD_OK;
}
