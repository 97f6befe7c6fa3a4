// Dense FP64 products of the 2D full CFE step (the adaptive algorithm's
// fallback past the mode cap, Sec. 3.3), of the 2D M_xy integrand and of the
// 2D energy's quartic term.
//
// Full step: the tensor-product CFE system of eq. AC-discrete-semi-stable-K,
//   (c M_0 (x) M_1 + lam (K_0 (x) M_1 + M_0 (x) K_1)) vec U' = vec Q,
//   Q = c M_0 U^k M_1 - F,   F_ij = int N~_i N~_j L w(u^k)  (the M_xy matrix),
// solved exactly in the generalised eigenbases V_d of (K_d, M_d)
// (V^T M V = I, V^T K V = diag mu):
//   U' = V_0 [(V_0^T Q V_1) / (c + lam (mu_0i + mu_1j))] V_1^T.
// Every product is one launch of k_gemm64 (FP64 MFMA 16x16x4, 64x64 tiles
// staged through LDS, operands addressed through strides so that no
// transposed copy is formed).
#include "ctd_internal.h"

namespace ctd {

typedef double g4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 16;
constexpr int kPad = kBM + 1;

__device__ __forceinline__ double lane_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_gemm64(GemmArgs g) {
  __shared__ double As[kBK * kPad];
  __shared__ double Bs[kBK * kPad];
  __shared__ double red[4];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int i0 = blockIdx.y * kBM, j0 = blockIdx.x * kBN;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  g4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = g4{0, 0, 0, 0};
  // load maps: along the contiguous index of each operand
  const bool a_rows = g.a_i == 1;
  const bool b_cols = g.b_j == 1;
  double av[4], bv[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = a_rows ? (t & 63) : (t >> 4) + 16 * u;
      const int k = a_rows ? (t >> 6) + 4 * u : (t & 15);
      const int gi = i0 + r, gk = k0 + k;
      double v = 0.0;
      if (gi < g.m && gk < g.K) {
        v = g.A[(int64_t)gi * g.a_i + (int64_t)gk * g.a_k];
        if (g.ks) v *= g.ks[gk];
      }
      av[u] = v;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = b_cols ? (t & 63) : (t >> 4) + 16 * u;
      const int k = b_cols ? (t >> 6) + 4 * u : (t & 15);
      const int gj = j0 + c, gk = k0 + k;
      bv[u] = (gj < g.n && gk < g.K) ? g.B[(int64_t)gk * g.b_k + (int64_t)gj * g.b_j] : 0.0;
    }
  };
  if (g.K > 0) fetch(0);
  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    __syncthreads();   // the previous chunk's LDS reads are done
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = a_rows ? (t & 63) : (t >> 4) + 16 * u;
      const int k = a_rows ? (t >> 6) + 4 * u : (t & 15);
      As[k * kPad + r] = av[u];
      const int c = b_cols ? (t & 63) : (t >> 4) + 16 * u;
      const int kb = b_cols ? (t >> 6) + 4 * u : (t & 15);
      Bs[kb * kPad + c] = bv[u];
    }
    __syncthreads();
    // the next chunk's global loads are in flight during this chunk's MFMAs
    if (k0 + kBK < g.K) fetch(k0 + kBK);
#pragma unroll
    for (int ks = 0; ks < kBK; ks += 4) {
      const int k = ks + (l >> 4);
      double a0 = As[k * kPad + wr + (l & 15)];
      double a1 = As[k * kPad + wr + 16 + (l & 15)];
      double b0 = Bs[k * kPad + wc + (l & 15)];
      double b1 = Bs[k * kPad + wc + 16 + (l & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  // epilogue; the f64 16x16x4 MFMA holds rows (l >> 4) + 4 e of column l & 15
  double part = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + wr + 16 * a + (l >> 4) + 4 * e;
        const int j = j0 + wc + 16 * b + (l & 15);
        if (i >= g.m || j >= g.n) continue;
        const double v = acc[a][b][e];
        if (g.epi == kEpiU4) {
          const double v2 = v * v;
          part += g.w0[i] * g.w1[j] * (v2 * v2);
          continue;
        }
        double r = v;
        if (g.epi == kEpiAxpby) {
          const int64_t di = (int64_t)i * g.d_i + (int64_t)j * g.d_j;
          const double dv = g.d_f32 ? (double)((const float*)g.D)[di] : ((const double*)g.D)[di];
          r = g.alpha * v - dv;
        } else if (g.epi == kEpiFdDiv) {
          r = v / (g.c + g.lam * (g.mu0[i] + g.mu1[j]));
        } else if (g.epi == kEpiCubic) {
          r = g.alpha * g.w0[i] * g.w1[j] * (v * v * v - v);
        }
        g.C[(int64_t)i * g.c_i + (int64_t)j * g.c_j] = r;
      }
  if (g.epi == kEpiU4) {
    // fixed-order reduction: lanes, then the four waves
    part = lane_sum(part);
    if (l == 0) red[w] = part;
    __syncthreads();
    if (t == 0) g.part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

__global__ void k_unit_columns(double* X, int n, int ncols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * ncols) return;
  const int m = (int)(idx / n), i = (int)(idx % n);
  X[idx] = i == m ? 1.0 : 0.0;
}

__global__ void k_fill(double* x, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ------------------------------------------------------------ 3D field state
// A 3D field state (the field of a full step, Sec. 3.3 adaptive algorithm)
// is the nodal tensor U[i0][i1][i2] (row-major).  The next step's integrals
// of u^k are those of the field: the tensor
//   R = c (M_0 (x) M_1 (x) M_2) U - int N~ (x) N~ (x) N~ omega (u^3 - u)
// (the 3D counterpart of c M_0 U M_1 - M_xy) is formed once per step, and a
// directional right-hand side contracts R with the two other factors.  The
// passes below apply one axis at a time; one thread per output element, sums
// in fixed order.

__device__ __forceinline__ int elem_start3(int e, int s, int n, int SW) {
  int st = e - s;
  st = st < 0 ? 0 : st;
  return st > n - SW ? n - SW : st;
}

// strides of a row-major (d0, d1, d2) tensor along each axis
__device__ __forceinline__ void axis_split(int64_t idx, int o1, int o2, int& c0, int& c1, int& c2) {
  c2 = (int)(idx % o2);
  const int64_t r = idx / o2;
  c1 = (int)(r % o1);
  c0 = (int)(r / o1);
}

// out = Phi along axis a: input dims d[] with d[a] = n nodes, output the
// same with nq Gauss points on axis a.
__global__ void k_field_phi(const double* __restrict__ in, double* __restrict__ out, int d0, int d1,
                            int d2, int a, const double* __restrict__ phi, int n, int nq, int SW,
                            int ng, int s) {
  const int o0 = a == 0 ? nq : d0, o1 = a == 1 ? nq : d1, o2 = a == 2 ? nq : d2;
  const int64_t total = (int64_t)o0 * o1 * o2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int c0, c1, c2;
  axis_split(idx, o1, o2, c0, c1, c2);
  const int q = a == 0 ? c0 : (a == 1 ? c1 : c2);
  const int st = elem_start3(q / ng, s, n, SW);
  const int64_t str = a == 0 ? (int64_t)d1 * d2 : (a == 1 ? d2 : 1);
  const int64_t base = a == 0 ? (int64_t)c1 * d2 + c2
                              : (a == 1 ? (int64_t)c0 * d1 * d2 + c2 : ((int64_t)c0 * d1 + c1) * d2);
  double acc = 0.0;
  for (int jj = 0; jj < SW; ++jj) acc += phi[(int64_t)q * SW + jj] * in[base + (st + jj) * str];
  out[idx] = acc;
}

// out = Phi^T along axis a: input dims d[] with d[a] = nq, output with n
// nodes on axis a (elements, then Gauss points, in increasing order).
__global__ void k_field_phit(const double* __restrict__ in, double* __restrict__ out, int d0, int d1,
                             int d2, int a, const double* __restrict__ phi, int n, int nq, int SW,
                             int ng, int s) {
  const int o0 = a == 0 ? n : d0, o1 = a == 1 ? n : d1, o2 = a == 2 ? n : d2;
  const int64_t total = (int64_t)o0 * o1 * o2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int c0, c1, c2;
  axis_split(idx, o1, o2, c0, c1, c2);
  const int i = a == 0 ? c0 : (a == 1 ? c1 : c2);
  const int64_t str = a == 0 ? (int64_t)d1 * d2 : (a == 1 ? d2 : 1);
  const int64_t base = a == 0 ? (int64_t)c1 * d2 + c2
                              : (a == 1 ? (int64_t)c0 * d1 * d2 + c2 : ((int64_t)c0 * d1 + c1) * d2);
  const int ne = n - 1;
  int e0 = i - SW, e1 = i + SW;
  e0 = e0 < 0 ? 0 : e0;
  e1 = e1 > ne - 1 ? ne - 1 : e1;
  double acc = 0.0;
  for (int e = e0; e <= e1; ++e) {
    const int jj = i - elem_start3(e, s, n, SW);
    if (jj < 0 || jj >= SW) continue;
    for (int g = 0; g < ng; ++g) {
      const int q = e * ng + g;
      acc += phi[(int64_t)q * SW + jj] * in[base + q * str];
    }
  }
  out[idx] = acc;
}

// out = A along axis a for a symmetric band matrix in lower storage
// ((B+1) x n, row t holds A[i+t, i] at [t n + i]); dims d[] with d[a] = n.
__global__ void k_field_band(const double* __restrict__ in, double* __restrict__ out, int d0, int d1,
                             int d2, int a, const double* __restrict__ band, int n, int B) {
  const int64_t total = (int64_t)d0 * d1 * d2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int c0, c1, c2;
  axis_split(idx, d1, d2, c0, c1, c2);
  const int i = a == 0 ? c0 : (a == 1 ? c1 : c2);
  const int64_t str = a == 0 ? (int64_t)d1 * d2 : (a == 1 ? d2 : 1);
  const int64_t base = idx - (int64_t)i * str;
  double acc = band[i] * in[base + (int64_t)i * str];
  for (int t = 1; t <= B; ++t) {
    if (i + t < n) acc += band[(int64_t)t * n + i] * in[base + (int64_t)(i + t) * str];
    if (i - t >= 0) acc += band[(int64_t)t * n + i - t] * in[base + (int64_t)(i - t) * str];
  }
  out[idx] = acc;
}

// Gauss-grid integrand in place: G = omega (u^3 - u) W_0 W_1 W_2; the
// quartic energy partials a0 W (u^2 - 1)^2 of the same points (fixed-order
// block sums) when part != nullptr.
__global__ __launch_bounds__(256) void k_field_integrand(double* __restrict__ G, int q0n, int q1n,
                                                          int q2n, const double* __restrict__ w0,
                                                          const double* __restrict__ w1,
                                                          const double* __restrict__ w2, double omega,
                                                          double a0, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t total = (int64_t)q0n * q1n * q2n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (idx < total) {
    int c0, c1, c2;
    axis_split(idx, q1n, q2n, c0, c1, c2);
    const double u = G[idx];
    const double w = w0[c0] * w1[c1] * w2[c2];
    const double u2 = u * u;
    e = a0 * w * (u2 - 1.0) * (u2 - 1.0);
    G[idx] = omega * (u2 * u - u) * w;
  }
  if (!part) return;
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// R = c MU - T (elementwise)
__global__ void k_field_axpby(double* __restrict__ R, const double* __restrict__ MU,
                              const double* __restrict__ T, double c, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < total) R[idx] = c * MU[idx] - T[idx];
}

// fixed-order block partials of sum_i x_i y_i
__global__ __launch_bounds__(256) void k_field_dot(const double* __restrict__ x, const double* __restrict__ y,
                                                   int64_t total, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  red[threadIdx.x] = idx < total ? x[idx] * y[idx] : 0.0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// T /= c + lam (mu_0[i] + mu_1[j] + mu_2[k])
__global__ void k_field_fd_div(double* __restrict__ T, int n0, int n1, int n2, const double* __restrict__ mu0,
                               const double* __restrict__ mu1, const double* __restrict__ mu2, double c,
                               double lam) {
  const int64_t total = (int64_t)n0 * n1 * n2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int c0, c1, c2;
  axis_split(idx, n1, n2, c0, c1, c2);
  T[idx] = T[idx] / (c + lam * (mu0[c0] + mu1[c1] + mu2[c2]));
}

// Right-hand-side chunks of direction d from R: chunk p of the P chunks
// holds sum over a 1/P share of the first contracted axis; the solve adds
// the chunks in order.  out: P x n_d.
__global__ __launch_bounds__(256) void k_field_contract(const double* __restrict__ R, int n0, int n1, int n2,
                                                        int d, const double* __restrict__ u0,
                                                        const double* __restrict__ u1,
                                                        const double* __restrict__ u2, int P,
                                                        double* __restrict__ out, const int* skip) {
  __shared__ double red[256];
  // a launch of a speculatively enqueued sweep whose mode had ended
  if (skip && *skip) return;
  const int p = blockIdx.y;
  const int tid = threadIdx.x;
  if (d == 2) {
    // out[p][k] = sum_{i in share p} u0[i] sum_j u1[j] R[i][j][k]
    const int k = blockIdx.x * 256 + tid;
    if (k >= n2) return;
    const int per = (n0 + P - 1) / P, ib = p * per, ie = ib + per < n0 ? ib + per : n0;
    double acc = 0.0;
    for (int i = ib; i < ie; ++i) {
      double t = 0.0;
      for (int j = 0; j < n1; ++j) t += u1[j] * R[((int64_t)i * n1 + j) * n2 + k];
      acc += u0[i] * t;
    }
    out[(int64_t)p * n2 + k] = acc;
    return;
  }
  // d = 0: block (i, p), share p of j; d = 1: block (j, p), share p of i;
  // threads over k, then a fixed-order block sum
  const int o = blockIdx.x;
  double acc = 0.0;
  if (d == 0) {
    const int per = (n1 + P - 1) / P, jb = p * per, je = jb + per < n1 ? jb + per : n1;
    for (int j = jb; j < je; ++j) {
      double t = 0.0;
      for (int k = tid; k < n2; k += 256) t += R[((int64_t)o * n1 + j) * n2 + k] * u2[k];
      acc += u1[j] * t;
    }
  } else {
    const int per = (n0 + P - 1) / P, ib = p * per, ie = ib + per < n0 ? ib + per : n0;
    for (int i = ib; i < ie; ++i) {
      double t = 0.0;
      for (int k = tid; k < n2; k += 256) t += R[((int64_t)i * n1 + o) * n2 + k] * u2[k];
      acc += u0[i] * t;
    }
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) out[(int64_t)p * (d == 0 ? n0 : n1) + o] = red[0];
}

__global__ void k_field_to_f32(const double* __restrict__ X, float* __restrict__ Y, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < total) Y[idx] = (float)X[idx];
}

unsigned blocks_of(int64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

hipError_t launch_field_to_f32(const double* X, float* Y, int64_t total, hipStream_t st) {
  if (total == 0) return hipSuccess;
  k_field_to_f32<<<blocks_of(total), 256, 0, st>>>(X, Y, total);
  return hipGetLastError();
}

hipError_t launch_field_phi(const double* in, double* out, const int* dims, int a, const DevAxis& A,
                            hipStream_t st) {
  int64_t total = 1;
  for (int e = 0; e < 3; ++e) total *= e == a ? A.nq : dims[e];
  if (total == 0) return hipSuccess;
  k_field_phi<<<blocks_of(total), 256, 0, st>>>(in, out, dims[0], dims[1], dims[2], a, A.phi, A.n, A.nq,
                                                 A.SW, A.ng, A.s);
  return hipGetLastError();
}

hipError_t launch_field_phit(const double* in, double* out, const int* dims, int a, const DevAxis& A,
                             hipStream_t st) {
  int64_t total = 1;
  for (int e = 0; e < 3; ++e) total *= e == a ? A.n : dims[e];
  if (total == 0) return hipSuccess;
  k_field_phit<<<blocks_of(total), 256, 0, st>>>(in, out, dims[0], dims[1], dims[2], a, A.phi, A.n, A.nq,
                                                  A.SW, A.ng, A.s);
  return hipGetLastError();
}

hipError_t launch_field_band(const double* in, double* out, const int* dims, int a, const double* band,
                             int n, int B, hipStream_t st) {
  const int64_t total = (int64_t)dims[0] * dims[1] * dims[2];
  if (total == 0) return hipSuccess;
  k_field_band<<<blocks_of(total), 256, 0, st>>>(in, out, dims[0], dims[1], dims[2], a, band, n, B);
  return hipGetLastError();
}

hipError_t launch_field_integrand(double* G, const int* qdims, const double* w0, const double* w1,
                                  const double* w2, double omega, double a0, double* part,
                                  hipStream_t st) {
  const int64_t total = (int64_t)qdims[0] * qdims[1] * qdims[2];
  if (total == 0) return hipSuccess;
  k_field_integrand<<<blocks_of(total), 256, 0, st>>>(G, qdims[0], qdims[1], qdims[2], w0, w1, w2, omega,
                                                       a0, part);
  return hipGetLastError();
}

int64_t field_partials(int64_t total) { return (int64_t)blocks_of(total); }

hipError_t launch_field_axpby(double* R, const double* MU, const double* T, double c, int64_t total,
                              hipStream_t st) {
  if (total == 0) return hipSuccess;
  k_field_axpby<<<blocks_of(total), 256, 0, st>>>(R, MU, T, c, total);
  return hipGetLastError();
}

hipError_t launch_field_dot(const double* x, const double* y, int64_t total, double* part, hipStream_t st) {
  if (total == 0) return hipSuccess;
  k_field_dot<<<blocks_of(total), 256, 0, st>>>(x, y, total, part);
  return hipGetLastError();
}

hipError_t launch_field_fd_div(double* T, const int* dims, const double* mu0, const double* mu1,
                               const double* mu2, double c, double lam, hipStream_t st) {
  const int64_t total = (int64_t)dims[0] * dims[1] * dims[2];
  if (total == 0) return hipSuccess;
  k_field_fd_div<<<blocks_of(total), 256, 0, st>>>(T, dims[0], dims[1], dims[2], mu0, mu1, mu2, c, lam);
  return hipGetLastError();
}

hipError_t launch_field_contract(const double* R, const int* dims, int d, const double* u0, const double* u1,
                                 const double* u2, int P, double* out, const int* skip, hipStream_t st) {
  dim3 grid(d == 2 ? (dims[2] + 255) / 256 : dims[d], P);
  k_field_contract<<<grid, 256, 0, st>>>(R, dims[0], dims[1], dims[2], d, u0, u1, u2, P, out, skip);
  return hipGetLastError();
}

// Mode product along axis a of a row-major (n0, n1, n2) tensor with the
// axis' generalised eigenvectors V (row-major n_a x n_a, column m = vector
// m): forward Y = V^T x_a X, backward Y = V x_a X (FP64 MFMA products; axis
// 1 one product per slab of axis 0).
hipError_t launch_field_eig(const double* X, double* Y, const int* dims, int a, const double* V, int forward,
                            hipStream_t st) {
  const int n0 = dims[0], n1 = dims[1], n2 = dims[2];
  const int na = dims[a];
  GemmArgs g;
  g.A = V;
  // forward: A(r, k) = V[k][r] (a_i = 1, a_k = na); backward: A(r, k) = V[r][k]
  if (a == 0) {
    g.m = n0; g.n = n1 * n2; g.K = n0;
    g.a_i = forward ? 1 : na; g.a_k = forward ? na : 1;
    g.B = X; g.b_k = (int64_t)n1 * n2; g.b_j = 1;
    g.C = Y; g.c_i = (int64_t)n1 * n2; g.c_j = 1;
    return launch_gemm64(g, st);
  }
  if (a == 2) {
    // Y[r][c] = sum_k X[r][k] B(k, c): B(k, c) = V[k][c] (forward) or V[c][k]
    GemmArgs h;
    h.m = n0 * n1; h.n = n2; h.K = n2;
    h.A = X; h.a_i = n2; h.a_k = 1;
    h.B = V; h.b_k = forward ? n2 : 1; h.b_j = forward ? 1 : n2;
    h.C = Y; h.c_i = n2; h.c_j = 1;
    return launch_gemm64(h, st);
  }
  g.m = n1; g.n = n2; g.K = n1;
  g.a_i = forward ? 1 : na; g.a_k = forward ? na : 1;
  g.b_k = n2; g.b_j = 1;
  g.c_i = n2; g.c_j = 1;
  for (int i = 0; i < n0; ++i) {
    g.B = X + (int64_t)i * n1 * n2;
    g.C = Y + (int64_t)i * n1 * n2;
    hipError_t e = launch_gemm64(g, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int gemm64_blocks(int m, int n) { return ((m + kBM - 1) / kBM) * ((n + kBN - 1) / kBN); }

hipError_t launch_gemm64(const GemmArgs& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0) return hipSuccess;
  dim3 grid((g.n + kBN - 1) / kBN, (g.m + kBM - 1) / kBM);
  k_gemm64<<<grid, 256, 0, st>>>(g);
  return hipGetLastError();
}

hipError_t launch_unit_columns(double* X, int n, int ncols, hipStream_t st) {
  const int64_t total = (int64_t)n * ncols;
  if (total == 0) return hipSuccess;
  k_unit_columns<<<(int)((total + 255) / 256), 256, 0, st>>>(X, n, ncols);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<(n + 255) / 256, 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}

}  // namespace ctd
