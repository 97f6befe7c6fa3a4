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

}  // namespace

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
