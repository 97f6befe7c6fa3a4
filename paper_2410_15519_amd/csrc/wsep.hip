// Separated integration of the 2D M_xy (Sec. 3.3, eq. MxySep).
//
// The Gauss-grid values of L w(u^k) = omega (u^3 - u), U = Xh_0 Xh_1^T, are
// replaced by a sum of Q rank-one terms a_q b_q^T found by the progressive
// (greedy rank-one) decomposition: terms are added one at a time, each from
// a fixed count of alternating updates, each update the least-squares factor
// against the residual R = W - sum_{p<q} a_p b_p^T with the other fixed,
//   a <- R b / (b.b),   b <- R^T a / (a.a)      (a zero denominator: 0),
// b starting from the counter-based vector keyed (seed, 0, q, 7).  Then
//   M_xy = sum_q (Phi_0^T W_0 a_q)(Phi_1^T W_1 b_q)^T,
// a product of 1D integrals per term.  W and W^T are held in full (both
// formed by the FP64 MFMA product with the cubic epilogue and unit weights;
// rows and the terms' columns at even strides, so that they are read as
// 16-byte pairs), so both updates are row-by-row products read once,
// coalesced.
#include "ctd_internal.h"

namespace ctd {

namespace {

__device__ __forceinline__ double ws_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int ws_elem_start(int e, int s, int n, int SW) {
  int st = e - s;
  st = st < 0 ? 0 : st;
  return st > n - SW ? n - SW : st;
}

// splitmix64 (Steele, Lea, Flood 2014): the counter-based start vector
__device__ __forceinline__ uint64_t ws_splitmix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// b[i] = 2 U53(splitmix64(key + i)) - 1, key = (((seed 1000003 + 0) 1000003
// + q) 8 + 7) << 32: the initial-guess key with step 0 and direction slot 7
__global__ void k_ws_start(double* b, int n, uint64_t seed, int q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = seed * 1000003ull;
  k = k * 1000003ull + (uint64_t)q;
  k = (k * 8ull + 7ull) << 32;
  const uint64_t z = ws_splitmix(k + (uint64_t)i);
  b[i] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// out[p] = V[:, p] . x for p < q, out[q] = x . x; one workgroup per product
// (grid q + 1), four 256-wide segments in flight per pass, sums added in
// fixed order (segments, lanes, waves).  V: n x Q, column stride ldv.
__global__ __launch_bounds__(256) void k_ws_dots(const double* V, int ldv, const double* x, int n, int q,
                                                 double* out) {
  __shared__ double red[4];
  const int p = blockIdx.x, t = threadIdx.x;
  const double* col = p < q ? V + (size_t)p * ldv : x;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  int i = t;
  for (; i + 3 * 256 < n; i += 4 * 256) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = col[i + 256 * u];
      b[u] = x[i + 256 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) part[u] += a[u] * b[u];
  }
  for (int u = 0; i < n; i += 256, ++u) part[u] += col[i] * x[i];
  double s = ws_wave_sum((part[0] + part[1]) + (part[2] + part[3]));
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) out[p] = (red[0] + red[1]) + (red[2] + red[3]);
}

// y[i] = (M[i, :] . x - sum_{p<q} U[i, p] dots[p]) / dots[q] (0 when
// dots[q] = 0); M: r x c rows of even stride ldm, x 16-byte aligned, U: r x
// Q, column stride ldu.  One wave per row, read as 16-byte pairs, eight
// 64-pair segments in flight per pass (eight partial sums, added in fixed
// order), the odd last column by lane 0.
__global__ __launch_bounds__(256) void k_ws_update(const double* M, int r, int c, int ldm, const double* x,
                                                   const double* U, int ldu, const double* dots, int q,
                                                   double* y) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (i >= r) return;
  const double* row = M + (size_t)i * ldm;
  const double2* row2 = (const double2*)row;
  const double2* x2 = (const double2*)x;
  const int c2 = c >> 1;
  double part[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int j = l;
  for (; j + 7 * 64 < c2; j += 8 * 64) {
    double2 m[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m[u] = row2[j + 64 * u];
      v[u] = x2[j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) part[u] += m[u].x * v[u].x + m[u].y * v[u].y;
  }
  for (int u = 0; j < c2; j += 64, ++u) part[u] += row2[j].x * x2[j].x + row2[j].y * x2[j].y;
  if ((c & 1) && l == 0) part[7] += row[c - 1] * x[c - 1];
  double s = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
  s = ws_wave_sum(s);
  if (l != 0) return;
  double corr = 0.0;
  for (int p = 0; p < q; ++p) corr += U[(size_t)p * ldu + i] * dots[p];
  const double den = dots[q];
  y[i] = den != 0.0 ? (s - corr) / den : 0.0;
}

// P[i, q] = sum over the Gauss points g of the elements around node i of
// Phi[g, i] W[g] F[g, q] (elements in increasing order): the 1D integrals
// int N~_i w^(q) of every term.  F: nq x Q (column stride ldf), P: n x Q.
__global__ void k_ws_project(DevAxis A, const double* F, int ldf, int Q, double* P) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)A.n * Q) return;
  const int q = (int)(idx / A.n), i = (int)(idx % A.n);
  const int ne = A.n - 1;
  const int e0 = i - A.SW < 0 ? 0 : i - A.SW;
  const int e1 = i + A.SW > ne - 1 ? ne - 1 : i + A.SW;
  const double* f = F + (size_t)q * ldf;
  double acc = 0.0;
  for (int e = e0; e <= e1; ++e) {
    const int jj = i - ws_elem_start(e, A.s, A.n, A.SW);
    if (jj < 0 || jj >= A.SW) continue;
    for (int g = 0; g < A.ng; ++g) {
      const int qx = e * A.ng + g;
      acc += A.phi[(size_t)qx * A.SW + jj] * A.w[qx] * f[qx];
    }
  }
  P[idx] = acc;
}

// M_xy[i, j] = sum_q Pa[i, q] Pb[j, q], stored with its transpose.
template <class T>
__global__ void k_ws_mxy(const double* Pa, const double* Pb, int nx, int ny, int Q, T* Mxy, T* MxyT) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nx * ny) return;
  const int i = (int)(idx / ny), j = (int)(idx % ny);
  double acc = 0.0;
  for (int q = 0; q < Q; ++q) acc += Pa[(size_t)q * nx + i] * Pb[(size_t)q * ny + j];
  Mxy[(size_t)i * ny + j] = (T)acc;
  MxyT[(size_t)j * nx + i] = (T)acc;
}

}  // namespace

hipError_t launch_mxy_separated(const DevInst& I, const WsepBufs& B, hipStream_t st) {
  const DevAxis& X = I.ax[0];
  const DevAxis& Y = I.ax[1];
  const int n0 = X.nq, n1 = Y.nq, Q = B.rank;
  const int ld0 = (int)wsep_ld(n1), ld1 = (int)wsep_ld(n0);   // strides of W rows / B columns, W^T rows / A columns
  if (Q < 1 || Q > kWsepMaxRank || B.iters < 1) return hipErrorInvalidValue;
  hipError_t e = launch_fill(B.ones, n0 > n1 ? n0 : n1, 1.0, st);
  if (e != hipSuccess) return e;
  // W = omega (U^3 - U) and its transpose on the full Gauss grid
  for (int t = 0; t < 2; ++t) {
    const DevAxis& R = t == 0 ? X : Y;
    const DevAxis& C = t == 0 ? Y : X;
    GemmArgs g;
    g.m = R.nq; g.n = C.nq; g.K = I.Mk; g.epi = kEpiCubic;
    g.A = R.Xh; g.a_i = I.Mkp; g.a_k = 1;
    g.B = C.Xh; g.b_k = 1; g.b_j = I.Mkp;
    g.C = t == 0 ? B.W : B.Wt; g.c_i = t == 0 ? ld0 : ld1; g.c_j = 1;
    g.alpha = I.omega; g.w0 = B.ones; g.w1 = B.ones;
    if ((e = launch_gemm64(g, st)) != hipSuccess) return e;
  }
  const int rb0 = (n0 + 3) / 4, rb1 = (n1 + 3) / 4;
  for (int q = 0; q < Q; ++q) {
    double* a = B.A + (size_t)q * ld1;
    double* b = B.B + (size_t)q * ld0;
    k_ws_start<<<(n1 + 255) / 256, 256, 0, st>>>(b, n1, I.seed, q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int it = 0; it < B.iters; ++it) {
      // a <- (W b - A (B^T b)) / (b.b)
      k_ws_dots<<<q + 1, 256, 0, st>>>(B.B, ld0, b, n1, q, B.dots);
      k_ws_update<<<rb0, 256, 0, st>>>(B.W, n0, n1, ld0, b, B.A, ld1, B.dots, q, a);
      // b <- (W^T a - B (A^T a)) / (a.a)
      k_ws_dots<<<q + 1, 256, 0, st>>>(B.A, ld1, a, n0, q, B.dots);
      k_ws_update<<<rb1, 256, 0, st>>>(B.Wt, n1, n0, ld1, a, B.B, ld0, B.dots, q, b);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // the 1D integrals of every term, then M_xy
  const size_t p0 = (size_t)X.n * Q, p1 = (size_t)Y.n * Q;
  k_ws_project<<<(int)((p0 + 255) / 256), 256, 0, st>>>(X, B.A, ld1, Q, B.Pa);
  k_ws_project<<<(int)((p1 + 255) / 256), 256, 0, st>>>(Y, B.B, ld0, Q, B.Pb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t t2 = (size_t)X.n * Y.n;
  if (I.mixed)
    k_ws_mxy<float><<<(int)((t2 + 255) / 256), 256, 0, st>>>(B.Pa, B.Pb, X.n, Y.n, Q, (float*)I.Mxy,
                                                              (float*)I.MxyT);
  else
    k_ws_mxy<double><<<(int)((t2 + 255) / 256), 256, 0, st>>>(B.Pa, B.Pb, X.n, Y.n, Q, (double*)I.Mxy,
                                                               (double*)I.MxyT);
  return hipGetLastError();
}

}  // namespace ctd
