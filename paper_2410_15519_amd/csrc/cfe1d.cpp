// 1D convolution-FE tables, built once per axis on the host in FP64.
//
// Patch functions follow App. B: on the nodal patch of node i the
// interpolant u^i(xi) = Psi_a(xi) k + p(xi) l satisfies the interpolation
// and moment conditions (eq. reproducecondition).  Instead of forming R0^-1
// as printed, the (np + p + 1) saddle-point system
//     [ R0   P ] [k]   [u]
//     [ P^T  0 ] [l] = [0]
// is solved by LU with partial pivoting for every unit u, which yields the
// same K and L.  Shape functions follow App. C (FE-weighted sum of the two
// nodal patch functions of an element); matrices follow eq. (KxxMxx) with
// Gauss-Legendre quadrature.
//
// Storage: element e owns the SW = 2s+2 consecutive columns starting at
// st(e) = clamp(e - s, 0, n - SW); near the boundary the truncated patches
// leave zeros in part of that window.
#include "ctd_internal.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace ctd {

static double kernel_psi(double z) {
  z = std::fabs(z);
  if (z <= 0.5) return 2.0 / 3.0 - 4.0 * z * z + 4.0 * z * z * z;
  if (z <= 1.0) return 4.0 / 3.0 - 4.0 * z + 4.0 * z * z - (4.0 / 3.0) * z * z * z;
  return 0.0;
}

static double kernel_dpsi(double z) {  // d Psi / dz, z >= 0
  if (z <= 0.5) return -8.0 * z + 12.0 * z * z;
  if (z <= 1.0) return -4.0 + 8.0 * z - 4.0 * z * z;
  return 0.0;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n with
// the three-term recurrence.
void gauss_legendre(int ng, std::vector<double>& x, std::vector<double>& w) {
  x.assign(ng, 0.0);
  w.assign(ng, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < ng; ++i) {
    double t = std::cos(pi * (i + 0.75) / (ng + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= ng; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (ng == 1) { p1 = t; p0 = 1.0; }
      dp = ng * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= ng; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (ng == 1) { p1 = t; p0 = 1.0; }
      dp = ng * (t * p1 - p0) / (t * t - 1.0);
    }
    x[ng - 1 - i] = t;
    w[ng - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Dense LU with partial pivoting; solves A X = B in place (A: m x m
// row-major, B: m x r row-major).  Returns false if singular.
static bool lu_solve(int m, std::vector<double> A, std::vector<double>& B, int r) {
  std::vector<int> piv(m);
  for (int k = 0; k < m; ++k) {
    int pk = k;
    double best = std::fabs(A[k * m + k]);
    for (int i = k + 1; i < m; ++i)
      if (std::fabs(A[i * m + k]) > best) { best = std::fabs(A[i * m + k]); pk = i; }
    if (best == 0.0) return false;
    if (pk != k) {
      for (int j = 0; j < m; ++j) std::swap(A[k * m + j], A[pk * m + j]);
      for (int j = 0; j < r; ++j) std::swap(B[k * r + j], B[pk * r + j]);
    }
    for (int i = k + 1; i < m; ++i) {
      double f = A[i * m + k] / A[k * m + k];
      if (f == 0.0) continue;
      for (int j = k; j < m; ++j) A[i * m + j] -= f * A[k * m + j];
      for (int j = 0; j < r; ++j) B[i * r + j] -= f * B[k * r + j];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    for (int j = 0; j < r; ++j) {
      double s = B[k * r + j];
      for (int c = k + 1; c < m; ++c) s -= A[k * m + c] * B[c * r + j];
      B[k * r + j] = s / A[k * m + k];
    }
  }
  return true;
}

// Coefficients of the patch interpolant for patch nodes xn (natural
// coordinates): W(xi) = Psi(xi) Kc + p(xi) Lc, Kc: np x np, Lc: (p+1) x np,
// both row-major.
static bool patch_coeffs(const std::vector<double>& xn, double a, int p,
                         std::vector<double>& Kc, std::vector<double>& Lc) {
  const int np = (int)xn.size();
  const int m = np + p + 1;
  std::vector<double> A(m * m, 0.0), B(m * np, 0.0);
  for (int j = 0; j < np; ++j) {
    for (int l = 0; l < np; ++l) A[j * m + l] = kernel_psi(std::fabs(xn[j] - xn[l]) / a);
    double pw = 1.0;
    for (int t = 0; t <= p; ++t) {
      A[j * m + np + t] = pw;
      A[(np + t) * m + j] = pw;
      pw *= xn[j];
    }
    B[j * np + j] = 1.0;
  }
  if (!lu_solve(m, A, B, np)) return false;
  Kc.assign(B.begin(), B.begin() + np * np);
  Lc.assign(B.begin() + np * np, B.end());
  return true;
}

// Patch function values/derivatives at xi for patch nodes xn.
static void patch_eval(double xi, const std::vector<double>& xn, double a, int p,
                       const std::vector<double>& Kc, const std::vector<double>& Lc,
                       double* W, double* dW) {
  const int np = (int)xn.size();
  for (int j = 0; j < np; ++j) { W[j] = 0.0; dW[j] = 0.0; }
  for (int l = 0; l < np; ++l) {
    double t = xi - xn[l];
    double z = std::fabs(t) / a;
    double ps = kernel_psi(z);
    double dps = kernel_dpsi(z) * (t > 0 ? 1.0 : (t < 0 ? -1.0 : 0.0)) / a;
    for (int j = 0; j < np; ++j) {
      W[j] += ps * Kc[l * np + j];
      dW[j] += dps * Kc[l * np + j];
    }
  }
  double pw = 1.0, dpw = 0.0;
  for (int t = 0; t <= p; ++t) {
    for (int j = 0; j < np; ++j) {
      W[j] += pw * Lc[t * np + j];
      dW[j] += dpw * Lc[t * np + j];
    }
    dpw = (t + 1) * pw;  // derivative of xi^(t+1)
    pw *= xi;
  }
}

int build_axis(int64_t n64, double lo, double hi, int s, int p, double a, int ng,
               AxisTables& ax, std::string& err) {
  if (s < 1 || p < 0 || p > s) { err = "need patch_s >= 1 and 0 <= poly_p <= patch_s"; return CTD_EINVAL; }
  if (ng < 1 || ng > 16) { err = "gauss_points must be in [1, 16]"; return CTD_EINVAL; }
  if (!(a > 0.0) || !std::isfinite(a)) { err = "dilation_a must be positive"; return CTD_EINVAL; }
  if (!(hi > lo)) { err = "need hi > lo on every axis"; return CTD_EINVAL; }
  const int SW = 2 * s + 2;
  if (n64 < SW) { err = "need at least 2*patch_s+2 nodes per axis"; return CTD_EINVAL; }
  if (n64 > (1 << 20)) { err = "too many nodes per axis"; return CTD_EUNSUPPORTED; }
  const int n = (int)n64;
  ax.n = n; ax.s = s; ax.p = p; ax.a = a; ax.ng = ng;
  ax.SW = SW; ax.B = 2 * s + 1;
  ax.lo = lo; ax.hi = hi; ax.h = (hi - lo) / (n - 1);
  ax.ne = n - 1;
  ax.nq = ax.ne * ng;
  std::vector<double> xg, wg;
  gauss_legendre(ng, xg, wg);
  ax.phi.assign((size_t)ax.nq * SW, 0.0);
  ax.dphi.assign((size_t)ax.nq * SW, 0.0);
  ax.w.assign(ax.nq, 0.0);
  // Patch coefficient cache: on a uniform mesh the patch of node i depends
  // only on how it is truncated, and relative natural coordinates make the
  // coefficients translation invariant; cache by (left extent, right extent)
  // in coordinates relative to node i.
  struct Entry { int left, right; std::vector<double> Kc, Lc; };
  std::vector<Entry> cache;
  auto coeffs_for = [&](int i, const std::vector<double>*& Kc,
                        const std::vector<double>*& Lc) -> bool {
    int left = i - std::max(0, i - s), right = std::min(n - 1, i + s) - i;
    for (auto& e : cache)
      if (e.left == left && e.right == right) { Kc = &e.Kc; Lc = &e.Lc; return true; }
    std::vector<double> xn;
    for (int j = -left; j <= right; ++j) xn.push_back(2.0 * j);
    Entry e;
    e.left = left; e.right = right;
    if (!patch_coeffs(xn, a, p, e.Kc, e.Lc)) return false;
    cache.push_back(std::move(e));
    Kc = &cache.back().Kc; Lc = &cache.back().Lc;
    return true;
  };
  std::vector<double> W(2 * s + 1), dW(2 * s + 1);
  for (int e = 0; e < ax.ne; ++e) {
    int st = e - s;
    if (st < 0) st = 0;
    if (st > n - SW) st = n - SW;
    for (int side = 0; side < 2; ++side) {
      int i = e + side;
      const std::vector<double>* Kc;
      const std::vector<double>* Lc;
      if (!coeffs_for(i, Kc, Lc)) { err = "singular patch system"; return CTD_EINVAL; }
      int j0 = std::max(0, i - s), j1 = std::min(n - 1, i + s);
      std::vector<double> xn;
      // coordinates relative to node i; xi of node i in element e is -1 (left) or +1 (right)
      for (int j = j0; j <= j1; ++j) xn.push_back(2.0 * (j - i));
      double xi_i = side == 0 ? -1.0 : 1.0;
      for (int g = 0; g < ng; ++g) {
        double xi = xg[g];
        patch_eval(xi - xi_i, xn, a, p, *Kc, *Lc, W.data(), dW.data());
        double Ni = side == 0 ? 0.5 * (1.0 - xi) : 0.5 * (1.0 + xi);
        double dNi = side == 0 ? -0.5 : 0.5;
        size_t q = (size_t)e * ng + g;
        for (int j = j0; j <= j1; ++j) {
          int c = j - st;
          double wv = W[j - j0], dwv = dW[j - j0];
          ax.phi[q * SW + c] += Ni * wv;
          ax.dphi[q * SW + c] += (dNi * wv + Ni * dwv) * (2.0 / ax.h);
        }
      }
    }
    for (int g = 0; g < ng; ++g) ax.w[(size_t)e * ng + g] = wg[g] * ax.h * 0.5;
  }
  // banded mass and stiffness: lower band [t * n + i] = A[i + t][i]
  const int B = ax.B;
  ax.Mb.assign((size_t)(B + 1) * n, 0.0);
  ax.Kb.assign((size_t)(B + 1) * n, 0.0);
  for (int e = 0; e < ax.ne; ++e) {
    int st = std::min(std::max(e - s, 0), n - SW);
    for (int g = 0; g < ng; ++g) {
      size_t q = (size_t)e * ng + g;
      double wq = ax.w[q];
      for (int r = 0; r < SW; ++r)
        for (int c = 0; c <= r; ++c) {
          int i = st + r, j = st + c;  // i >= j
          int t = i - j;
          if (t > B) continue;
          ax.Mb[(size_t)t * n + j] += wq * ax.phi[q * SW + r] * ax.phi[q * SW + c];
          ax.Kb[(size_t)t * n + j] += wq * ax.dphi[q * SW + r] * ax.dphi[q * SW + c];
        }
    }
  }
  return CTD_OK;
}

}  // namespace ctd
