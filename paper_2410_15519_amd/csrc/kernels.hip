// HIP kernels of the CTD step for gfx950.
//
// Notation (Sec. 3.3 / App. D): for the directional solve in direction d the
// other directions' factors u_e are fixed; c = 1/dt + alpha L, lam = L kappa,
// omega = 4 a0 L.  Quadrature tables: Phi_d (nq x n, SW = 2s+2 nonzeros per
// row starting at column st(e)), weights W_d.  u^k = sum_j sk_j prod_d X^k_d[:,j]
// and its Gauss-point tables Xh_d = Phi_d X^k_d diag(sk^(1/D)).
#include "ctd_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace ctd {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <class T> struct Vec4;
template <> struct Vec4<float> { typedef f4 type; };
template <> struct Vec4<double> { typedef d4 type; };

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output row held in accumulator element k by lane l (column = l & 15).
// Measured on gfx950: the f32 16x16x4 MFMA keeps four consecutive rows per
// lane, the f64 one interleaves them with stride 4.
template <class T> __device__ __forceinline__ int mfma_row(int l, int k);
template <> __device__ __forceinline__ int mfma_row<float>(int l, int k) { return (l >> 4) * 4 + k; }
template <> __device__ __forceinline__ int mfma_row<double>(int l, int k) { return (l >> 4) + 4 * k; }

// A speculatively enqueued sweep launch whose mode already ended: return at
// once (the flag was written by an earlier launch on the same stream).
__device__ __forceinline__ bool spec_skip(const DevInst& I) {
  return I.spec_check && I.sc->done;
}

__device__ __forceinline__ int elem_start(int e, int s, int n, int SW) {
  int st = e - s;
  st = st < 0 ? 0 : st;
  return st > n - SW ? n - SW : st;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Fixed-order block reduction (deterministic); red: >= blockDim/64 doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}
__device__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int i = 1; i < nw; ++i) t = fmax(t, red[i]);
  return t;
}

// Symmetric band matrix-vector product at row i (lower band storage).
__device__ __forceinline__ double band_row(const double* band, int n, int B,
                                           const double* x, int i) {
  double y = band[i] * x[i];
  for (int t = 1; t <= B; ++t) {
    if (i + t < n) y += band[(size_t)t * n + i] * x[i + t];
    if (i - t >= 0) y += band[(size_t)t * n + i - t] * x[i - t];
  }
  return y;
}

// ------------------------------------------------------------ quad eval
// Xh[q, a] = sk_a^pw * sum_j Phi[q, j] X^k[st + j, a]; zero for a >= Mk.
__global__ void k_quad_eval(DevAxis A, int Mk, int ldh, const double* sk,
                            double pw, int mixed, int tile_major) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)A.nq * ldh;
  if (idx >= total) return;
  const int q = (int)(idx / ldh), a = (int)(idx % ldh);
  double val = 0.0;
  if (a < Mk) {
    const int e = q / A.ng;
    const int st = elem_start(e, A.s, A.n, A.SW);
    const double* ph = A.phi + (size_t)q * A.SW;
    const double* x = A.Xk + (size_t)a * A.n + st;
    for (int j = 0; j < A.SW; ++j) val += ph[j] * x[j];
    val *= pow(sk[a], pw);
  }
  A.Xh[idx] = val;
  if (mixed) {
    // The FP32 copy of the 3D path is tile-major over the 64-padded point
    // count, [a / 16][q][slot]: a tile's values at consecutive points are
    // contiguous.  Inside a tile, mode i sits in slot 4 (i % 4) + i / 4, so
    // that the 16-byte word g holds modes g, g+4, g+8, g+12.
    size_t dst = idx;
    if (tile_major) {
      const size_t nqp = (size_t)(A.nq + 63) / 64 * 64;
      const int i = a & 15;
      dst = ((size_t)(a >> 4) * nqp + q) * kTile + ((i & 3) << 2) + (i >> 2);
      // the g contraction's copy groups four consecutive points per mode:
      // [a / 16][q / 4][a % 16][q % 4], a 16-byte word holding one mode at
      // four points
      A.Xhg[((size_t)(a >> 4) * (nqp >> 2) + (q >> 2)) * 64 + i * 4 + (q & 3)] = (float)val;
    }
    A.Xhf[dst] = (float)val;
  }
}

hipError_t launch_quad_eval(const DevInst& I, int d, hipStream_t st) {
  const DevAxis& A = I.ax[d];
  size_t total = (size_t)A.nq * I.Mkp;
  int blocks = (int)((total + 255) / 256);
  if (blocks == 0) return hipSuccess;
  k_quad_eval<<<blocks, 256, 0, st>>>(A, I.Mk, I.Mkp, I.sk, 1.0 / I.dim, I.mixed, I.dim == 3);
  return hipGetLastError();
}

// ------------------------------------------------------------ band mv
__global__ void k_band_mv(int n, int B, const double* band, const double* X,
                          double* Y, int ncols) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * ncols) return;
  const int c = (int)(idx / n), i = (int)(idx % n);
  Y[idx] = band_row(band, n, B, X + (size_t)c * n, i);
}

hipError_t launch_band_mv(const DevAxis& A, const double* band, const double* X,
                          double* Y, int ncols, hipStream_t st) {
  size_t total = (size_t)A.n * ncols;
  if (total == 0) return hipSuccess;
  k_band_mv<<<(int)((total + 255) / 256), 256, 0, st>>>(A.n, A.B, band, X, Y, ncols);
  return hipGetLastError();
}

// ------------------------------------------------------------ mode init
// Counter-based initial guess (splitmix64 of Steele, Lea, Flood 2014):
// u_d[i] = 2 * U53(splitmix64(key(seed, step, mode, d) + i)) - 1.
__device__ __forceinline__ uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ void init_mode_body(const DevInst& I, uint64_t step, int mode, int warm,
                                               int bx, int d) {
  const DevAxis& A = I.ax[d];
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double val;
  if (warm && mode < I.Mk) {
    val = A.Xk[(size_t)mode * A.n + i];
  } else {
    uint64_t k = I.seed * 1000003ull + step;
    k = k * 1000003ull + (uint64_t)mode;
    k = k * 8ull + (uint64_t)d;
    k <<= 32;
    uint64_t z = sm64(k + (uint64_t)i);
    val = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
  }
  A.u[i] = val;
}

__global__ void k_init_mode(DevInst I, uint64_t step, int mode, int warm) {
  init_mode_body(I, step, mode, warm, blockIdx.x, blockIdx.y);
}

hipError_t launch_init_mode(const DevInst& I, int64_t step, int mode, int warm,
                            hipStream_t st) {
  int nmax = 0;
  for (int d = 0; d < I.dim; ++d) nmax = I.ax[d].n > nmax ? I.ax[d].n : nmax;
  dim3 grid((nmax + 255) / 256, I.dim);
  k_init_mode<<<grid, 256, 0, st>>>(I, (uint64_t)step, mode, warm);
  return hipGetLastError();
}

// ------------------------------------------------------------ finalize
// Normalise the raw factor in A.u to unit M-norm, cache M u, K u and the dot
// products used by the fixed-point test; at the last direction of a sweep
// evaluate the relative Frobenius change of the rank-one term.
// Fixed-order block reduction of NS sums and one max in one pass (two
// barriers); red: >= 16 (NS + 1) doubles.
template <int NS>
__device__ void block_sums_max(double (&v)[NS], double& mx, double* red) {
#pragma unroll
  for (int j = 0; j < NS; ++j) v[j] = wave_sum(v[j]);
  mx = wave_max(mx);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int j = 0; j < NS; ++j) red[j * 16 + w] = v[j];
    red[NS * 16 + w] = mx;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[j * 16 + i];
    v[j] = t;
  }
  mx = red[NS * 16];
  for (int i = 1; i < nw; ++i) mx = fmax(mx, red[NS * 16 + i]);
}

// Symmetric band row i of (lower band storage) times x, x in LDS; B fixed so
// that the band loads are issued together.
// Branch-free: the band storage holds exact zeros past the last row, and
// the entries before the first row are replaced by zero.
template <int B>
__device__ __forceinline__ double band_row_lds(const double* band, int n, const double* x, int i) {
  double y = band[i] * x[i];
#pragma unroll
  for (int t = 1; t <= B; ++t) {
    const int ip = i + t < n ? i + t : n - 1;
    const int im = i - t >= 0 ? i - t : 0;
    const double up = band[(size_t)t * n + i];
    const double lo = band[(size_t)t * n + im];
    y += up * x[ip];
    y += (i - t >= 0 ? lo : 0.0) * x[im];
  }
  return y;
}

// The same product with the 2B+1 band values of row i loaded ahead (into
// registers, before the vector x is ready); same summation order.
template <int B>
struct BandRow {
  double c0, up[B], lo[B];
};

template <int B>
__device__ __forceinline__ void band_row_load(const double* band, int n, int i, BandRow<B>& r) {
  r.c0 = band[i];
#pragma unroll
  for (int t = 1; t <= B; ++t) {
    const int im = i - t >= 0 ? i - t : 0;
    r.up[t - 1] = band[(size_t)t * n + i];
    r.lo[t - 1] = band[(size_t)t * n + im];
  }
}

template <int B>
__device__ __forceinline__ double band_row_apply(const BandRow<B>& r, int n, const double* x, int i) {
  double y = r.c0 * x[i];
#pragma unroll
  for (int t = 1; t <= B; ++t) {
    const int ip = i + t < n ? i + t : n - 1;
    const int im = i - t >= 0 ? i - t : 0;
    y += r.up[t - 1] * x[ip];
    y += (i - t >= 0 ? r.lo[t - 1] : 0.0) * x[im];
  }
  return y;
}

// Normalise the solved factor u_d to unit M-norm (sigma = its norm), cache
// M u, K u, and the Gram scalars of the fixed-point test.  One fused pass:
// the sums of the unnormalised u are rescaled by 1/sigma afterwards.
// red: >= 96 doubles of LDS; ul: 3n doubles of scratch (LDS) for u, M u, K u.
// writer = false (the fused normalisation + Grams launch): the same sums,
// but no stores to the instance; the normalised factor is left in ul for the
// caller (the previous factor is not read: only the writer needs it).
template <int B>
__device__ __forceinline__ void finalize_body(const DevInst& I, int d, int sweep, int from_init, double* red, double* ul,
                              int nparts = 0, bool writer = true) {
  const DevAxis& A = I.ax[d];
  DevScalars* sc = I.sc;
  const int n = A.n;
  double* ml = ul + n;
  double* kl = ul + 2 * n;
  // the other directions' Gram scalars of the fixed-point test, requested
  // at the start (they were written by earlier launches)
  double puu_o = 1.0, pupup_o = 1.0, puup_o = 1.0, sigma_prev = 0.0;
  if (writer && threadIdx.x == 0 && !from_init && d == I.dim - 1) {
    double a0[kMaxDim], a1[kMaxDim], a2[kMaxDim];
#pragma unroll
    for (int e = 0; e < kMaxDim; ++e) {
      a0[e] = sc->uu[e];
      a1[e] = sc->upup[e];
      a2[e] = sc->uup[e];
    }
    sigma_prev = sc->sigma_prev;
#pragma unroll
    for (int e = 0; e < kMaxDim; ++e) {
      if (e >= I.dim || e == d) continue;
      puu_o *= a0[e];
      pupup_o *= a1[e];
      puup_o *= a2[e];
    }
  }
  // one row per thread: the band rows and the previous factor value are
  // requested before the solved factor is staged (bandwidths up to 5: wider
  // rows would not fit the registers of a 1024-thread workgroup)
  const bool one = B <= 5 && n <= (int)blockDim.x;
  const int i1 = threadIdx.x < n ? threadIdx.x : n - 1;
  BandRow<B> rm, rk;
  double up1 = 0.0;
  if (one) {
    band_row_load<B>(A.Mb, n, i1, rm);
    band_row_load<B>(A.Kb, n, i1, rk);
    up1 = writer ? A.up[i1] : 0.0;
  }
  // the solved factor: u, or the sum of the back-projection partials (fixed order)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    if (nparts == 0) {
      v = A.u[i];
    } else {
      double p[kFdKb];
#pragma unroll
      for (int k = 0; k < kFdKb; ++k) p[k] = A.fdu[(size_t)k * n + i];
#pragma unroll
      for (int k = 0; k < kFdKb; ++k) v += p[k];
    }
    ul[i] = v;
  }
  __syncthreads();
  // u.Mu, u.Ku, u.u, u.up, up.up and max|u|
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double um = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double mu = one ? band_row_apply<B>(rm, n, ul, i) : band_row_lds<B>(A.Mb, n, ul, i);
    const double ku = one ? band_row_apply<B>(rk, n, ul, i) : band_row_lds<B>(A.Kb, n, ul, i);
    ml[i] = mu;
    kl[i] = ku;
    const double u = ul[i], up = one ? up1 : (writer ? A.up[i] : 0.0);
    acc[0] += u * mu;
    acc[1] += u * ku;
    acc[2] += u * u;
    acc[3] += u * up;
    acc[4] += up * up;
    um = fmax(um, fabs(u));
  }
  block_sums_max<5>(acc, um, red);
  const double s2 = acc[0];
  const double sigma = sqrt(s2);
  const bool bad = !(sigma == sigma) || isinf(sigma);
  const bool zero = sigma == 0.0;
  const double inv = (bad || zero) ? 0.0 : 1.0 / sigma;
  const double m = s2 * inv * inv, k = acc[1] * inv * inv, uu = acc[2] * inv * inv;
  const double uup = acc[3] * inv, upup = acc[4];
  um *= inv;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double u = ul[i] * inv;
    if (!writer) {
      ul[i] = u;
      continue;
    }
    A.u[i] = u;
    A.up[i] = u;
    A.Mu[i] = ml[i] * inv;
    A.Ku[i] = kl[i] * inv;
  }
  if (!writer) {
    __syncthreads();
    return;
  }
  if (threadIdx.x == 0) {
    sc->m[d] = m;
    sc->k[d] = k;
    sc->uu[d] = uu;
    sc->uup[d] = uup;
    sc->upup[d] = upup;
    sc->umax[d] = um;
    if (!from_init) {
      sc->sigma[d] = sigma;
      if (bad) sc->nonfinite = 1;
      if (zero) sc->zero = 1;
      if (d == I.dim - 1) {
        int conv = 0;
        if (sweep >= 2) {
          // products over the directions, in direction order (this one last)
          const double puu = puu_o * uu, pupup = pupup_o * upup, puup = puup_o * uup;
          const double nn = sigma * sigma * puu;
          const double oo = sigma_prev * sigma_prev * pupup;
          const double no = sigma * sigma_prev * puup;
          double r2 = nn + oo - 2.0 * no;
          r2 = r2 > 0.0 ? r2 : 0.0;
          double r = nn > 0.0 ? sqrt(r2 / nn) : 0.0;
          sc->change = r;
          conv = r <= I.fp_tol ? 1 : 0;
          sc->converged = conv;
        }
        sc->sigma_prev = sigma;
        // the host's end-of-mode test, for the speculatively enqueued next sweep
        if (I.spec_nsw > 0)
          sc->done = (sc->zero || sc->nonfinite || conv || sweep >= I.spec_nsw) ? 1 : 0;
      }
    }
  }
}

template <int B>
__global__ __launch_bounds__(1024) void k_finalize(DevInst I, int d, int sweep, int from_init, int nparts) {
  if (spec_skip(I)) return;
  __shared__ double red[96];
  extern __shared__ double ul[];
  // d < 0: every direction at once, one workgroup each (the initial guesses)
  finalize_body<B>(I, d < 0 ? (int)blockIdx.x : d, sweep, from_init, red, ul, nparts);
}

hipError_t launch_finalize_init(const DevInst& I, hipStream_t st) {
  int n = 0;
  for (int e = 0; e < I.dim; ++e) {
    if (I.ax[e].B != I.ax[0].B) return hipErrorInvalidValue;
    n = n > I.ax[e].n ? n : I.ax[e].n;
  }
  const size_t shm = sizeof(double) * 3 * (size_t)n;
  const int nt = n >= 1024 ? 1024 : (n + 63) / 64 * 64;
  switch (I.ax[0].B) {
    case 3: k_finalize<3><<<I.dim, nt, shm, st>>>(I, -1, 0, 1, 0); break;
    case 5: k_finalize<5><<<I.dim, nt, shm, st>>>(I, -1, 0, 1, 0); break;
    case 7: k_finalize<7><<<I.dim, nt, shm, st>>>(I, -1, 0, 1, 0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const DevInst& I, int d, int sweep, int from_init,
                           hipStream_t st, int nparts) {
  const int n = I.ax[d].n;
  const size_t shm = sizeof(double) * 3 * (size_t)n;
  const int nt = n >= 1024 ? 1024 : (n + 63) / 64 * 64;
  switch (I.ax[d].B) {
    case 3: k_finalize<3><<<1, nt, shm, st>>>(I, d, sweep, from_init, nparts); break;
    case 5: k_finalize<5><<<1, nt, shm, st>>>(I, d, sweep, from_init, nparts); break;
    case 7: k_finalize<7><<<1, nt, shm, st>>>(I, d, sweep, from_init, nparts); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ signature
// Grams of the freshly solved factor u_d against the stored columns
// (gm = X^T M u, gk = X^T K u over the M modes of u^{k+1}, gmk = X^kT M u)
// and v = W * (Phi u) at the Gauss points (3D cubic route).
__device__ __forceinline__ void signature_body(const DevInst& I, int d, int M, int ndot_blocks, int want_v,
                                               int bx, int by) {
  // d < 0: every direction at once, direction by (the initial guesses)
  const DevAxis& A = I.ax[d < 0 ? by : d];
  const int n = A.n;
  if (bx < ndot_blocks) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int idx = bx * 4 + w;
    const int total = 2 * M + I.Mk;
    if (idx >= total) return;
    const double* col;
    double* out;
    if (idx < M) { col = A.MX + (size_t)idx * n; out = A.gm + idx; }
    else if (idx < 2 * M) { col = A.KX + (size_t)(idx - M) * n; out = A.gk + (idx - M); }
    else { col = A.MXk + (size_t)(idx - 2 * M) * n; out = A.gmk + (idx - 2 * M); }
    double s = 0.0;
#pragma unroll 16
    for (int i = l; i < n; i += 64) s += col[i] * A.u[i];
    s = wave_sum(s);
    if (l == 0) *out = s;
    return;
  }
  if (!want_v) return;
  const int q = (bx - ndot_blocks) * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  const int st = elem_start(q / A.ng, A.s, n, A.SW);
  const double* ph = A.phi + (size_t)q * A.SW;
  double val = 0.0;
  for (int j = 0; j < A.SW; ++j) val += ph[j] * A.u[st + j];
  val *= A.w[q];
  A.v[q] = val;
  if (I.mixed) A.vf[q] = (float)val;
}

__global__ void k_signature(DevInst I, int d, int M, int ndot_blocks, int want_v) {
  if (spec_skip(I)) return;
  signature_body(I, d, M, ndot_blocks, want_v, blockIdx.x, blockIdx.y);
}

hipError_t launch_signature(const DevInst& I, int d, int M, hipStream_t st) {
  const int total = 2 * M + I.Mk;
  const int ndot = (total + 3) / 4;
  const int want_v = I.dim == 3;
  const int nv = want_v ? (I.ax[d].nq + 255) / 256 : 0;
  if (ndot + nv == 0) return hipSuccess;
  k_signature<<<ndot + nv, 256, 0, st>>>(I, d, M, ndot, want_v);
  return hipGetLastError();
}

hipError_t launch_signature_all(const DevInst& I, int M, hipStream_t st) {
  const int total = 2 * M + I.Mk;
  const int ndot = (total + 3) / 4;
  const int want_v = I.dim == 3;
  int nv = 0;
  for (int e = 0; want_v && e < I.dim; ++e) nv = nv > (I.ax[e].nq + 255) / 256 ? nv : (I.ax[e].nq + 255) / 256;
  if (ndot + nv == 0) return hipSuccess;
  k_signature<<<dim3(ndot + nv, I.dim), 256, 0, st>>>(I, -1, M, ndot, want_v);
  return hipGetLastError();
}

// Normalisation and Grams in one launch (fast-diagonalisation solves: the
// raw factor is the sum of the back-projection partials, which nothing in
// the launch writes).  Workgroup 0 is k_finalize's (stores the factor, M u,
// K u, the previous-sweep copy and the scalars); every other workgroup
// forms the same normalised factor in LDS with the same sums in the same
// order (so its values are those workgroup 0 stores) and then does one
// block of k_signature's work: one stored column's Gram per wave, or the
// Gauss-point values of nt points.  Saves a launch and its dependent
// round trip per directional solve; the results equal the two-launch
// sequence bitwise.
template <int B>
__global__ __launch_bounds__(1024) void k_finalize_sig(DevInst I, int d, int sweep, int M, int ndot_blocks,
                                                       int want_v, int nparts) {
  if (spec_skip(I)) return;
  __shared__ double red[96];
  extern __shared__ double ul[];
  const int b = blockIdx.x;
  finalize_body<B>(I, d, sweep, 0, red, ul, nparts, b == 0);
  if (b == 0) return;
  const DevAxis& A = I.ax[d];
  const int n = A.n;
  const int nw = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (b - 1 < ndot_blocks) {
    const int idx = (b - 1) * nw + w;
    const int total = 2 * M + I.Mk;
    if (idx >= total) return;
    const double* col;
    double* out;
    if (idx < M) { col = A.MX + (size_t)idx * n; out = A.gm + idx; }
    else if (idx < 2 * M) { col = A.KX + (size_t)(idx - M) * n; out = A.gk + (idx - M); }
    else { col = A.MXk + (size_t)(idx - 2 * M) * n; out = A.gmk + (idx - 2 * M); }
    double sum = 0.0;
#pragma unroll 16
    for (int i = l; i < n; i += 64) sum += col[i] * ul[i];
    sum = wave_sum(sum);
    if (l == 0) *out = sum;
    return;
  }
  if (!want_v) return;
  const int q = (b - 1 - ndot_blocks) * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  const int st = elem_start(q / A.ng, A.s, n, A.SW);
  const double* ph = A.phi + (size_t)q * A.SW;
  double val = 0.0;
  for (int j = 0; j < A.SW; ++j) val += ph[j] * ul[st + j];
  val *= A.w[q];
  A.v[q] = val;
  if (I.mixed) A.vf[q] = (float)val;
}

hipError_t launch_finalize_sig(const DevInst& I, int d, int sweep, int M, hipStream_t st, int nparts) {
  if (nparts <= 0) return hipErrorInvalidValue;   // the raw factor must not be the one workgroup 0 stores
  const int n = I.ax[d].n;
  const size_t shm = sizeof(double) * 3 * (size_t)n;
  const int nt = n >= 1024 ? 1024 : (n + 63) / 64 * 64;
  const int total = 2 * M + I.Mk;
  const int ndot = (total + nt / 64 - 1) / (nt / 64);
  const int want_v = I.dim == 3;
  const int nv = want_v ? (I.ax[d].nq + nt - 1) / nt : 0;
  const dim3 grid(1 + ndot + nv);
  switch (I.ax[d].B) {
    case 3: k_finalize_sig<3><<<grid, nt, shm, st>>>(I, d, sweep, M, ndot, want_v, nparts); break;
    case 5: k_finalize_sig<5><<<grid, nt, shm, st>>>(I, d, sweep, M, ndot, want_v, nparts); break;
    case 7: k_finalize_sig<7><<<grid, nt, shm, st>>>(I, d, sweep, M, ndot, want_v, nparts); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ rhs
// Right-hand side of the directional system (eq. KxQx and its 3D analogue):
//   Q_d = ck MXk (sk * a^k) - MX (sn (c a + lam b)) - lam KX (sn a) - F_d,
// ck = c with the 2D M_xy load (which contains the full w), ck = c + omega
// with the 3D cubic load F_d = omega Phi^T W h.
// Grid: row blocks of 64 x (column chunks of 64 over [MXk | MX | KX], plus
// the load chunks: 3D four chunks for -F_d (16 rows each); 2D the columns of the M_xy
// product F_d = M_xy u_e (d = 0) or M_xy^T u_e (d = 1), 64 per chunk, each
// column stored contiguously over the rows of d (a row of M_xy^T or M_xy)).
// Each block writes its partial sums to rpart[chunk][row]; the solve kernel
// adds the chunks in fixed order.
__device__ __forceinline__ int rhs_columns(const DevInst& I, int M, int load_only) {
  return load_only ? (I.dim == 3 ? I.Mk : 0) : I.Mk + 2 * M;
}

__device__ __forceinline__ void rhs_body(const DevInst& I, int d, int M, int load_only, int nchunk,
                                         int bx, int y) {
  // nchunk: the linear column chunks; the load chunks follow
  extern __shared__ double hl[];
  __shared__ double coef[64];
  __shared__ double part[256];
  const DevAxis& A = I.ax[d];
  const int n = A.n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r0 = bx * 64, i = r0 + l;
  if (y < nchunk) {
    const int ctot = rhs_columns(I, M, load_only);
    // 16 columns per wave, loaded before the coefficients are ready.  The
    // column bases are read into registers first: choosing between fields
    // of the by-value instance by address would make the compiler copy the
    // whole instance to scratch memory.
    const double* const MXk = A.MXk;
    const double* const MX = A.MX;
    const double* const KX = A.KX;
    double cv[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int c = y * 64 + w * 16 + cc;
      const double* col = c < I.Mk ? MXk + (size_t)c * n
                                   : (c < I.Mk + M ? MX + (size_t)(c - I.Mk) * n
                                                   : KX + (size_t)(c - I.Mk - M) * n);
      cv[cc] = (c < ctot && i < n) ? col[i] : 0.0;
    }
    const double ck = load_only ? -I.omega : (I.dim == 3 ? I.c + I.omega : I.c);
    if (tid < 64) {
      const int c = y * 64 + tid;
      double v = 0.0;
      if (c < I.Mk) {
        v = ck * I.sk[c];
        for (int e = 0; e < I.dim; ++e)
          if (e != d) v *= I.ax[e].gmk[c];
      } else if (c < ctot) {
        const int m = (c - I.Mk) % M;
        double am = 1.0, bm = 0.0;
        for (int e = 0; e < I.dim; ++e) {
          if (e == d) continue;
          am *= I.ax[e].gm[m];
          double t = I.ax[e].gk[m];
          for (int f = 0; f < I.dim; ++f)
            if (f != d && f != e) t *= I.ax[f].gm[m];
          bm += t;
        }
        v = (c - I.Mk < M) ? -I.sn[m] * (I.c * am + I.lam * bm) : -I.lam * I.sn[m] * am;
      }
      coef[tid] = v;
    }
    __syncthreads();
    double acc = 0.0;
    if (i < n) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc += coef[w * 16 + cc] * cv[cc];
    }
    part[tid] = acc;
    __syncthreads();
    if (w == 0 && i < n) A.rpart[(size_t)y * n + i] = part[l] + part[64 + l] + part[128 + l] + part[192 + l];
    return;
  }
  if (I.dim == 2) {
    // load chunk of the 2D M_xy product: 16 columns per wave, loaded before
    // the coefficients -u_e[j] (+u_e[j] for the load alone)
    const int o = 1 - d, nco = I.ax[o].n;
    const int j0 = (y - nchunk) * 64;
    const void* const mxyt = I.MxyT;
    const void* const mxy = I.Mxy;
    const void* base = d == 0 ? mxyt : mxy;
    double cv[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int j = j0 + w * 16 + cc;
      const size_t at = (size_t)j * n + i;
      double v = 0.0;
      if (j < nco && i < n) v = I.mixed ? (double)((const float*)base)[at] : ((const double*)base)[at];
      cv[cc] = v;
    }
    if (tid < 64) {
      const int j = j0 + tid;
      coef[tid] = j < nco ? (load_only ? I.ax[o].u[j] : -I.ax[o].u[j]) : 0.0;
    }
    __syncthreads();
    double acc = 0.0;
    if (i < n) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc += coef[w * 16 + cc] * cv[cc];
    }
    part[tid] = acc;
    __syncthreads();
    if (w == 0 && i < n) A.rpart[(size_t)y * n + i] = part[l] + part[64 + l] + part[128 + l] + part[192 + l];
    return;
  }
  // chunks nchunk + s, s < kLoadSub: the projected nonlinear load
  // F_i = omega sum_q Phi[q, i] W_q h_q of rows r0 + 16 s .. r0 + 16 s + 15
  // (zero in the block's other rows), so that a workgroup sums the h splits
  // of only the Gauss points around 16 rows; h and the Phi rows of those
  // elements are staged in LDS, and the elements of a row are split over the
  // four waves (summed in wave order).  A row's sum is the same whichever
  // sub-chunk computes it, and the solve adds the zeros exactly.
  double F = 0.0;
  {
    const int ne = n - 1;
    const int SW = A.SW;
    const int ra = r0 + 16 * (y - nchunk), rb = ra + 16;
    const int e_lo = ra - SW > 0 ? ra - SW : 0;
    const int e_hi = rb - 1 + SW < ne - 1 ? rb - 1 + SW : ne - 1;
    const int q_lo = e_lo * A.ng, qcount = (e_hi - e_lo + 1) * A.ng;
    double* phl = hl + qcount;    // qcount x SW
    for (int idx = tid; idx < qcount; idx += blockDim.x) {
      const int q = q_lo + idx;
      // the h splits in order, sixteen loads in flight at a time
      const int ns = I.nsplit_h;
      double h = 0.0;
      for (int s0 = 0; s0 < ns; s0 += 16) {
        double hp[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) hp[k] = s0 + k < ns ? I.hpart[(size_t)(s0 + k) * A.nq + q] : 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) h += hp[k];
      }
      hl[idx] = h * A.w[q];
    }
    for (int idx = tid; idx < qcount * SW; idx += blockDim.x)
      phl[idx] = A.phi[(size_t)q_lo * SW + idx];
    __syncthreads();
    double Fw = 0.0;
    if (i < n && i >= ra && i < rb) {
      int e0 = i - SW;
      e0 = e0 < e_lo ? e_lo : e0;
      int e1 = i + SW;
      e1 = e1 > e_hi ? e_hi : e1;
      for (int e = e0 + w; e <= e1; e += 4) {
        const int st = elem_start(e, A.s, n, SW);
        const int jj = i - st;
        if (jj < 0 || jj >= SW) continue;
        for (int g = 0; g < A.ng; ++g) {
          const int qq = e * A.ng + g - q_lo;
          Fw += phl[qq * SW + jj] * hl[qq];
        }
      }
    }
    part[tid] = Fw;
    __syncthreads();
    if (w == 0) F = I.omega * (part[l] + part[64 + l] + part[128 + l] + part[192 + l]);
  }
  if (w == 0 && i < n) A.rpart[(size_t)y * n + i] = load_only ? F : -F;
}

__global__ __launch_bounds__(256) void k_rhs(DevInst I, int d, int M, int load_only, int nchunk) {
  if (spec_skip(I)) return;
  rhs_body(I, d, M, load_only, nchunk, blockIdx.x, blockIdx.y);
}

static int rhs_linear_chunks(const DevInst& I, int M, int load_only) {
  const int ctot = load_only ? (I.dim == 3 ? I.Mk : 0) : I.Mk + 2 * M;
  return (ctot + 63) / 64;
}

int rhs_load_chunks(const DevInst& I, int d) {
  if (I.dim == 2) return (I.ax[1 - d].n + 63) / 64;
  return I.fparts > 0 ? I.fparts : kLoadSub;
}

int rhs_chunks(const DevInst& I, int d, int M, int load_only) {
  return rhs_linear_chunks(I, M, load_only) + rhs_load_chunks(I, d) - 1;
}

hipError_t launch_rhs(const DevInst& I, int d, int M, hipStream_t st, int load_only) {
  const DevAxis& A = I.ax[d];
  const int nchunk = rhs_linear_chunks(I, M, load_only);
  if (I.dim == 3 && I.fparts > 0) {
    // 3D field state: the linear chunks of the new modes, then the load
    // chunks from the contraction of R3 with the other directions' factors
    if (nchunk > 0) {
      dim3 grid((A.n + 63) / 64, nchunk);
      k_rhs<<<grid, 256, 0, st>>>(I, d, M, load_only, nchunk);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    const int dims[3] = {I.ax[0].n, I.ax[1].n, I.ax[2].n};
    return launch_field_contract(I.R3, dims, d, I.ax[0].u, I.ax[1].u, I.ax[2].u, I.fparts,
                                 A.rpart + (size_t)nchunk * A.n, I.spec_check ? &I.sc->done : nullptr, st);
  }
  dim3 grid((A.n + 63) / 64, nchunk + rhs_load_chunks(I, d));
  // h (qcount) and the Phi rows (qcount x SW) of the elements around a row block
  const size_t shm = sizeof(double) * (size_t)(64 + 2 * A.SW + 2) * A.ng * (1 + A.SW);
  k_rhs<<<grid, 256, shm, st>>>(I, d, M, load_only, nchunk);
  return hipGetLastError();
}

// rhs[i] = sum of the chunk partials (fixed order)
__device__ __forceinline__ double rhs_at(const DevAxis& A, int i, int nchunk) {
  double v = 0.0;
  for (int y = 0; y <= nchunk; ++y) v += A.rpart[(size_t)y * A.n + i];
  return v;
}

__global__ void k_rhs_sum(DevInst I, int d, int nchunk) {
  DevAxis& A = I.ax[d];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < A.n) A.rhs[i] = rhs_at(A, i, nchunk);
}

hipError_t launch_rhs_sum(const DevInst& I, int d, int M, int load_only, hipStream_t st) {
  k_rhs_sum<<<(I.ax[d].n + 255) / 256, 256, 0, st>>>(I, d, rhs_chunks(I, d, M, load_only));
  return hipGetLastError();
}

// ------------------------------------------------------------ band solve
// SPD banded systems (alpha M + beta K) x = b, half-bandwidth B.

int max_lds_bytes();

// ---- block cyclic reduction (block data in LDS, or in a global workspace) ----
// The band matrix is block tridiagonal with B x B blocks: D_I (diagonal),
// L_I = A[block I, block I-1] (upper triangular at the start).  At level
// l (stride s = 2^l) the active blocks are I = s-1 + k s; those with even k
// are eliminated, the odd ones receive the Schur complements
//   D_I -= V1^T V1 + V2^T V2,   L_I <- -V1^T W1,   b_I -= V1^T y1 + V2^T y2,
// V1 = G1^-1 L_I^T, W1 = G1^-1 L_J1, y1 = G1^-1 b_J1, V2 = G2^-1 L_J2,
// y2 = G2^-1 b_J2, with G1 G1^T = D_J1, G2 G2^T = D_J2 (J1 = I-s, J2 = I+s).
// The back substitution walks the levels down:
//   x_J = G_J^-T G_J^-1 (b_J - L_J x_{J-s} - L_{J+s}^T x_{J+s}).
// One group of B lanes per kept block, lane c owning column c; both
// neighbour Cholesky factors are formed redundantly in every lane of the
// group, and the columns are exchanged with in-wave shuffles, so a level
// costs one workgroup barrier.  Per block (block-major, odd stride in
// doubles): D (packed, B(B+1)/2), L (B^2), copy of the L_{J+s} the
// back substitution needs (B^2), b/x (B), Cholesky factor G of the block
// when it is eliminated (packed; 1/g on its diagonal).
template <int B>
struct Bcr {
  static constexpr int NP = B * (B + 1) / 2;
  static constexpr int OL = NP, OLN = NP + B * B, OB = NP + 2 * B * B, OG = NP + 2 * B * B + B;
  static constexpr int STRIDE = (2 * NP + 2 * B * B + B) | 1;
  __host__ __device__ static constexpr int pk(int r, int c) { return r * (r + 1) / 2 + c; }   // c <= r
  // Cholesky of a packed SPD block; diagonal stored as 1/g
  __device__ static void chol(double* D) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double s = D[pk(j, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= D[pk(j, k)] * D[pk(j, k)];
      // 1/sqrt(s): hardware estimate refined by two Newton steps
      double rg = __builtin_amdgcn_rsq(s);
      rg = rg * fma(-0.5 * s * rg, rg, 1.5);
      rg = rg * fma(-0.5 * s * rg, rg, 1.5);
      D[pk(j, j)] = rg;
#pragma unroll
      for (int i = j + 1; i < B; ++i) {
        double t = D[pk(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= D[pk(i, k)] * D[pk(j, k)];
        D[pk(i, j)] = t * rg;
      }
    }
  }
  __device__ static void fwd(const double* G, double* v) {   // v <- G^-1 v
#pragma unroll
    for (int i = 0; i < B; ++i) {
      double t = v[i];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= G[pk(i, k)] * v[k];
      v[i] = t * G[pk(i, i)];
    }
  }
  __device__ static void bwd(const double* G, double* v) {   // v <- G^-T v
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
      double t = v[i];
#pragma unroll
      for (int k = i + 1; k < B; ++k) t -= G[pk(k, i)] * v[k];
      v[i] = t * G[pk(i, i)];
    }
  }
};

// Threads of the solve workgroup: one wave per 64/B kept blocks of the first
// level (one round up to n ~ 1.1k at B = 5), 4 waves at least, and at most
// as many as keep the per-lane registers of a level (which grow as B^2) free
// of spills.
__host__ __device__ constexpr int bcr_max_waves(int B) { return B >= 7 ? 8 : 10; }
__host__ __device__ inline int bcr_threads(int n, int B) {
  const int N = (n + B - 1) / B;
  const int gpw = 64 / B, wmax = bcr_max_waves(B);
  int w = ((N / 2) + gpw - 1) / gpw;
  w = w < 4 ? 4 : (w > wmax ? wmax : w);
  return 64 * w;
}

// Block storage of the cyclic reduction.  MODE 0: every block in LDS (sa);
// 1: every block in global memory (sa); 2: odd blocks in LDS (sa), even
// blocks in global memory (sb).  Levels s >= 2 and the back substitution
// above s = 1 touch odd blocks only, so in mode 2 only the first level and
// the last back-substitution level reach global memory.  Each access takes
// the branch of its block's parity, so LDS blocks keep LDS instructions.
template <int B, int MODE>
struct BcrMem {
  static constexpr int S = Bcr<B>::STRIDE;
  double* sa;
  double* sb;
  // P: parity of block I known at the call site (1 odd, 2 even) or 0
  template <int P = 0>
  __device__ __forceinline__ double ld(int e, int I) const {
    if (MODE == 2) {
      if (P == 1 || (P == 0 && (I & 1))) return sa[(size_t)(I >> 1) * S + e];
      return sb[(size_t)(I >> 1) * S + e];
    }
    return sa[(size_t)I * S + e];
  }
  template <int P = 0>
  __device__ __forceinline__ void st(int e, int I, double v) const {
    if (MODE == 2) {
      if (P == 1 || (P == 0 && (I & 1))) sa[(size_t)(I >> 1) * S + e] = v;
      else sb[(size_t)(I >> 1) * S + e] = v;
      return;
    }
    sa[(size_t)I * S + e] = v;
  }
  // odd blocks only in mode 2 (the kept blocks of every level)
  __device__ __forceinline__ double* odd_ptr(int e, int I) const {
    return MODE == 2 ? sa + (size_t)(I >> 1) * S + e : sa + (size_t)I * S + e;
  }
};

template <int B, int MODE>
__device__ __forceinline__ void bcr_solve_par(int n, const double* Mb, const double* Kb, double al, double be,
                              const double* rpart, int nchunk, double* out, BcrMem<B, MODE> mem) {
  typedef Bcr<B> T;
  static_assert(B <= 8, "a group of B lanes per block");
  constexpr int NP = T::NP;
  constexpr int GPW = 64 / B;                  // groups per wave
  const int N = (n + B - 1) / B;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ln = tid & 63, gi = ln / B;
  const bool lane_ok = gi < GPW;
  const int c = lane_ok ? ln - gi * B : 0;     // column owned by this lane
  const int gbase = lane_ok ? gi * B : 0;      // first lane of the group in its wave
  const int grp = (tid >> 6) * GPW + (lane_ok ? gi : 0), ngrp = (nt >> 6) * GPW;
#define BLD(e, I) mem.ld((e), (I))
#define BST(e, I, v) mem.st((e), (I), (v))
  // kept blocks (odd in every level) and their neighbours (even in the
  // first level, odd above it): parity known at compile time per level kind
#define BLDO(e, I) mem.template ld<1>((e), (I))
#define BSTO(e, I, v) mem.template st<1>((e), (I), (v))
#define BLDN(e, I) mem.template ld<NP_>((e), (I))
#define BSTN(e, I, v) mem.template st<NP_>((e), (I), (v))
  // D, L and b of every block: clear D and L (padding rows of the last block
  // get a unit diagonal), scatter the band entries with coalesced loads
  // issued four at a time, and sum the RHS partials
  for (int idx = tid; idx < N * (NP + B * B); idx += nt) {
    const int I = idx / (NP + B * B), e = idx - I * (NP + B * B);
    double v = 0.0;
    if (e < NP) {
      int r = 0;
      while (T::pk(r + 1, 0) <= e) ++r;
      if (I * B + r >= n && e == T::pk(r, r)) v = 1.0;
    }
    BST(e, I, v);
  }
  for (int i = tid; i < N * B; i += nt) {
    const int I = i / B, r = i - I * B;
    double v = 0.0;
    if (i < n)
      for (int y = 0; y <= nchunk; ++y) v += rpart[(size_t)y * n + i];
    BST(T::OB + r, I, v);
  }
  __syncthreads();
  {
    const int total = (B + 1) * n;
    for (int base = tid; base < total; base += 4 * nt) {
      double mv[4], kv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = base + u * nt;
        mv[u] = idx < total ? Mb[idx] : 0.0;
        kv[u] = idx < total ? Kb[idx] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = base + u * nt;
        const int t = idx / n, j = idx - t * n, i = j + t;   // entry A[i, j], i = j + t
        if (idx < total && i < n) {
          const double v = al * mv[u] + be * kv[u];
          const int I = i / B, r = i - I * B, J = j / B, cc = j - J * B;
          if (I == J) BST(T::pk(r, cc), I, v);
          else BST(T::OL + r * B + cc, I, v);
        }
      }
    }
  }
  __syncthreads();
  // one reduction level; FIRST: the first level (s = 1), whose neighbour
  // blocks J1, J2 are even
  auto level = [&](auto first_tag, const int s) {
    constexpr int NP_ = decltype(first_tag)::value ? 2 : 1;
    const int first = s - 1;
    const int count = (N - first + s - 1) / s;
    const int nkept = count / 2;
    for (int g0 = 0; g0 < nkept; g0 += ngrp) {
      const int g = g0 + grp;
      const bool act = lane_ok && g < nkept;
      // inactive lanes work on kept block 0 of the level (loads stay in
      // range; nothing is stored) so that every lane takes part in the shuffles
      const int k = act ? 2 * g + 1 : 1;
      const int I = first + k * s, J1 = I - s;
      const bool has2 = k + 1 < count;
      const int J2 = has2 ? I + s : J1;
      // V1 = G1^-1 L_I^T and V2 = G2^-1 L_J2 are exchanged between the lanes
      // of the group through the idle slots of the kept block I (its L copy
      // and factor slots are first written when I is eliminated); a group
      // lives in one wave, whose LDS accesses complete in order.
      double* vx = mem.odd_ptr(T::OLN, I);        // V1 (B x B, column-major by lane)
      double w1[B], y1[B], v2[B], y2[B];
      double bc = 0.0;
      {
        // side J1: its factor is kept for the back substitution together
        // with the L_I it will need
        double G[NP], v1[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
          v1[q] = BLDO(T::OL + c * B + q, I);      // row c of L_I
          w1[q] = BLDN(T::OL + q * B + c, J1);     // column c of L_J1
          y1[q] = BLDN(T::OB + q, J1);
        }
        if (act)
#pragma unroll
          for (int q = 0; q < B; ++q) BSTN(T::OLN + c * B + q, J1, v1[q]);
#pragma unroll
        for (int e = 0; e < NP; ++e) G[e] = BLDN(e, J1);
        T::chol(G);
        T::fwd(G, v1);
        T::fwd(G, w1);
        T::fwd(G, y1);
        if (act) {
#pragma unroll
          for (int e = 0; e < NP; ++e)
            if (e % B == c) BSTN(T::OG + e, J1, G[e]);
        }
#pragma unroll
        for (int q = 0; q < B; ++q) bc += v1[q] * y1[q];
        __builtin_amdgcn_wave_barrier();
        if (act)
#pragma unroll
          for (int q = 0; q < B; ++q) vx[c * B + q] = v1[q];
      }
      {
        // side J2 (absent: contributes zero); its factor is kept when it is
        // the last active block, which no other kept block has as J1
        double G[NP];
#pragma unroll
        for (int e = 0; e < NP; ++e) G[e] = BLDN(e, J2);
#pragma unroll
        for (int q = 0; q < B; ++q) {
          v2[q] = BLDN(T::OL + q * B + c, J2);     // column c of L_J2
          y2[q] = BLDN(T::OB + q, J2);
        }
        T::chol(G);
        T::fwd(G, v2);
        T::fwd(G, y2);
        if (act && has2 && k + 1 == count - 1) {
#pragma unroll
          for (int e = 0; e < NP; ++e)
            if (e % B == c) BSTN(T::OG + e, J2, G[e]);
        }
        if (!has2) {
#pragma unroll
          for (int q = 0; q < B; ++q) { v2[q] = 0.0; y2[q] = 0.0; }
        }
#pragma unroll
        for (int q = 0; q < B; ++q) bc += v2[q] * y2[q];
      }
      __builtin_amdgcn_wave_barrier();
      if (act) {
        double v1c[B];
#pragma unroll
        for (int q = 0; q < B; ++q) v1c[q] = vx[c * B + q];
#pragma unroll
        for (int r = 0; r < B; ++r) {
          double d = 0.0, lsum = 0.0;
#pragma unroll
          for (int q = 0; q < B; ++q) {
            const double a1 = vx[r * B + q];                    // V1[q][r]
            const double a2 = __shfl(v2[q], gbase + r, 64);     // V2[q][r]
            d += a1 * v1c[q] + a2 * v2[q];
            lsum += a1 * w1[q];
          }
          if (r >= c) BSTO(T::pk(r, c), I, BLDO(T::pk(r, c), I) - d);
          BSTO(T::OL + r * B + c, I, -lsum);
        }
        BSTO(T::OB + c, I, BLDO(T::OB + c, I) - bc);
      } else {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
          for (int q = 0; q < B; ++q) (void)__shfl(v2[q], gbase + r, 64);
      }
    }
    __syncthreads();
  };
  int top = 1;
  for (int s = 1;; s <<= 1) {
    const int first = s - 1;
    const int count = (N - first + s - 1) / s;
    if (count <= 1) { top = s; break; }
    if (MODE == 2 && s == 1) level(std::true_type{}, s);
    else level(std::false_type{}, s);
  }
  // last active block: x = D^-1 b
  if (tid < B) {
    const int J = top - 1;
    double G[NP], v[B];
#pragma unroll
    for (int e = 0; e < NP; ++e) G[e] = BLD(e, J);
#pragma unroll
    for (int q = 0; q < B; ++q) v[q] = BLD(T::OB + q, J);
    T::chol(G);
    T::fwd(G, v);
    T::bwd(G, v);
    if (tid == 0)
#pragma unroll
      for (int q = 0; q < B; ++q) BST(T::OB + q, J, v[q]);
  }
  __syncthreads();
  // back substitution, top level down; in the last level (s = 1) the
  // solved blocks J are even, their neighbours odd
  auto back = [&](auto last_tag, const int s) {
    constexpr int NP_ = decltype(last_tag)::value ? 2 : 1;
    const int first = s - 1;
    const int count = (N - first + s - 1) / s;
    const int nelim = (count + 1) / 2;
    for (int g0 = 0; g0 < nelim; g0 += ngrp) {
      const int g = g0 + grp;
      const bool act = lane_ok && g < nelim;
      const int J = first + 2 * (act ? g : 0) * s;
      const bool lo = J - s >= 0, hi = J + s < N;
      double t = BLDN(T::OB + c, J);
      if (lo) {
#pragma unroll
        for (int q = 0; q < B; ++q) t -= BLDN(T::OL + c * B + q, J) * BLDO(T::OB + q, J - s);
      }
      if (hi) {
#pragma unroll
        for (int q = 0; q < B; ++q) t -= BLDN(T::OLN + q * B + c, J) * BLDO(T::OB + q, J + s);
      }
      double v[B], G[NP];
#pragma unroll
      for (int q = 0; q < B; ++q) v[q] = __shfl(t, gbase + q, 64);
#pragma unroll
      for (int e = 0; e < NP; ++e) G[e] = BLDN(T::OG + e, J);
      T::fwd(G, v);
      T::bwd(G, v);
      double xc = v[0];
#pragma unroll
      for (int q = 1; q < B; ++q) xc = q == c ? v[q] : xc;
      if (act) BSTN(T::OB + c, J, xc);
    }
    __syncthreads();
  };
  for (int s = top >> 1; s >= 1; s >>= 1) {
    if (MODE == 2 && s == 1) back(std::true_type{}, s);
    else back(std::false_type{}, s);
  }
  for (int i = tid; i < n; i += nt) {
    const int I = i / B, r = i - I * B;
    out[i] = BLD(T::OB + r, I);
  }
  __syncthreads();
#undef BLD
#undef BST
#undef BLDO
#undef BSTO
#undef BLDN
#undef BSTN
}

__host__ __device__ size_t bcr_lds_bytes(int n, int B) {
  const int N = (n + B - 1) / B;
  const int stride = (B * (B + 1) + 2 * B * B + B) | 1;   // Bcr<B>::STRIDE
  return sizeof(double) * (size_t)N * stride;
}

bool bcr_fits(int n, int B) { return bcr_lds_bytes(n, B) + 1024 <= (size_t)max_lds_bytes(); }

// LDS of the split storage (odd blocks in LDS; also the 3n-double scratch of
// the normalisation that follows the solve)
size_t bcr_split_lds_bytes(int n, int B) {
  const int N = (n + B - 1) / B;
  const int stride = (B * (B + 1) + 2 * B * B + B) | 1;
  const size_t odd = sizeof(double) * (size_t)(N / 2) * stride;
  const size_t fin = sizeof(double) * 3 * (size_t)n;
  return odd > fin ? odd : fin;
}
bool bcr_split_fits(int n, int B) { return bcr_split_lds_bytes(n, B) + 1024 <= (size_t)max_lds_bytes(); }

// alpha_d, beta_d of K_d = alpha_d M_d + beta_d K_d (eq. KxQx, 3D analogue)
// from the fixed factors' m_e = u_e.M.u_e, k_e = u_e.K.u_e.
__device__ __forceinline__ void directional_coeffs(const DevInst& I, int d, double& al, double& be) {
  double pm = 1.0, grad = 0.0;
  for (int e = 0; e < I.dim; ++e)
    if (e != d) pm *= I.sc->m[e];
  for (int e = 0; e < I.dim; ++e) {
    if (e == d) continue;
    double t = I.sc->k[e];
    for (int f = 0; f < I.dim; ++f)
      if (f != d && f != e) t *= I.sc->m[f];
    grad += t;
  }
  al = I.c * pm + I.lam * grad;
  be = I.lam * pm;
}

// Directional solve by block cyclic reduction: alpha_d, beta_d from the
// fixed factors, solve, then normalisation and the fixed-point test.
// MODE (BcrMem): 0 block data in LDS, 1 in the global workspace, 2 odd
// blocks in LDS and even blocks in the workspace (separate instantiations,
// so that LDS data keep LDS addressing)
template <int B, int MODE>
__global__ __launch_bounds__(64 * bcr_max_waves(B)) void k_solve_bcr(DevInst I, int d, int sweep, int nchunk, double* gws) {
  if (spec_skip(I)) return;
  extern __shared__ double lds[];
  BcrMem<B, MODE> mem{MODE == 1 ? gws : lds, MODE == 2 ? gws : nullptr};
  double* sm = MODE == 1 ? gws : lds;
  __shared__ double red[96];
  __shared__ double ab[2];
  DevAxis& A = I.ax[d];
  if (threadIdx.x == 0) {
    directional_coeffs(I, d, ab[0], ab[1]);
    I.sc->alpha[d] = ab[0];
    I.sc->beta[d] = ab[1];
  }
  __syncthreads();
  bcr_solve_par<B, MODE>(A.n, A.Mb, A.Kb, ab[0], ab[1], A.rpart, nchunk, A.u, mem);
  finalize_body<B>(I, d, sweep, 0, red, sm);
}

hipError_t launch_solve_bcr(const DevInst& I, int d, int sweep, int M, hipStream_t st) {
  const DevAxis& A = I.ax[d];
  const bool fits = bcr_fits(A.n, A.B);
  const bool split = !fits && bcr_split_fits(A.n, A.B);
  if (!fits && !I.bcr_ws) return hipErrorInvalidValue;
  const size_t shm = fits ? bcr_lds_bytes(A.n, A.B) : (split ? bcr_split_lds_bytes(A.n, A.B) : 0);
  double* gws = fits ? nullptr : I.bcr_ws;
  const int nchunk = rhs_chunks(I, d, M, 0);
  const int nt = bcr_threads(A.n, A.B);
#define SOLVE_BCR(BW)                                                                   \
  (fits ? k_solve_bcr<BW, 0><<<1, nt, shm, st>>>(I, d, sweep, nchunk, nullptr)          \
        : split ? k_solve_bcr<BW, 2><<<1, nt, shm, st>>>(I, d, sweep, nchunk, gws)      \
                : k_solve_bcr<BW, 1><<<1, nt, 0, st>>>(I, d, sweep, nchunk, gws))
  switch (A.B) {
    case 3: SOLVE_BCR(3); break;
    case 5: SOLVE_BCR(5); break;
    case 7: SOLVE_BCR(7); break;
    default: return hipErrorInvalidValue;
  }
#undef SOLVE_BCR
  return hipGetLastError();
}

template <int B, int MODE>
__global__ __launch_bounds__(64 * bcr_max_waves(B)) void k_band_solve_bcr(int n, const double* Mb, const double* Kb,
                                                        const double* alpha, const double* beta,
                                                        const double* b, double* x, double* gws) {
  extern __shared__ double lds[];
  const int k = blockIdx.x;
  double* g = MODE == 0 ? nullptr : gws + (size_t)k * (bcr_lds_bytes(n, B) / sizeof(double));
  BcrMem<B, MODE> mem{MODE == 1 ? g : lds, MODE == 2 ? g : nullptr};
  bcr_solve_par<B, MODE>(n, Mb, Kb, alpha[k], beta[k], b + (size_t)k * n, 0, x + (size_t)k * n, mem);
}

size_t band_solve_workspace_bytes(int n, int bw, int count) {
  return bcr_fits(n, bw) ? 0 : bcr_lds_bytes(n, bw) * (size_t)count;
}

hipError_t launch_band_solve_batch_ws(int n, int bw, const double* Mb, const double* Kb,
                                      const double* alpha, const double* beta, const double* b,
                                      double* x, int count, double* gws, hipStream_t st) {
  const bool fits = bcr_fits(n, bw);
  const bool split = !fits && bcr_split_fits(n, bw);
  if (!fits && !gws) return hipErrorInvalidValue;
  const size_t bytes = bcr_lds_bytes(n, bw);
  const size_t shm = fits ? bytes : (split ? bcr_split_lds_bytes(n, bw) : 0);
  const int nt = bcr_threads(n, bw);
#define BAND_BCR(BW)                                                                               \
  (fits ? k_band_solve_bcr<BW, 0><<<count, nt, shm, st>>>(n, Mb, Kb, alpha, beta, b, x, nullptr)    \
        : split ? k_band_solve_bcr<BW, 2><<<count, nt, shm, st>>>(n, Mb, Kb, alpha, beta, b, x, gws) \
                : k_band_solve_bcr<BW, 1><<<count, nt, 0, st>>>(n, Mb, Kb, alpha, beta, b, x, gws))
  switch (bw) {
    case 3: BAND_BCR(3); break;
    case 5: BAND_BCR(5); break;
    case 7: BAND_BCR(7); break;
    default: return hipErrorInvalidValue;
  }
#undef BAND_BCR
  return hipGetLastError();
}

hipError_t launch_band_solve_batch(int n, int bw, const double* Mb,
                                   const double* Kb, const double* alpha,
                                   const double* beta, const double* b,
                                   double* x, int count, hipStream_t st) {
  const size_t ws = band_solve_workspace_bytes(n, bw, count);
  double* gws = nullptr;
  if (ws) {
    hipError_t e = hipMallocAsync((void**)&gws, ws, st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_band_solve_batch_ws(n, bw, Mb, Kb, alpha, beta, b, x, count, gws, st);
  if (gws) {
    hipError_t f = hipFreeAsync(gws, st);
    if (e == hipSuccess) e = f;
  }
  return e;
}

// ---- fast diagonalisation: x = V diag(1 / (alpha + beta mu)) V^T b ----
// Projection: workgroup (64 eigenvector columns, one of kFdSplit row ranges);
// lane = column, waves interleave the rows.  The right-hand side of the
// row range is summed from its partials into LDS first (same order as the
// cyclic reduction takes them); eight rows' loads are in flight per thread.
__global__ __launch_bounds__(256) void k_fd_project(DevInst I, int d, int nchunk) {
  if (spec_skip(I)) return;
  const DevAxis& A = I.ax[d];
  const int n = A.n;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + l;
  const int per = (n + kFdSplit - 1) / kFdSplit;
  const int i0 = blockIdx.y * per;
  const int i1 = i0 + per < n ? i0 + per : n;
  extern __shared__ double bl[];    // per doubles
  __shared__ double part[4][64];
  const int kk = k < n ? k : n - 1;    // past the end: read in range, never stored
  // the first 32 rows of this wave's share of V are requested before the
  // right-hand side is staged (rows r = w + 4 u)
  constexpr int kPre = 32;
  double vp[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int r = w + 4 * u;
    vp[u] = r < i1 - i0 ? A.fdV[(size_t)(i0 + r) * n + kk] : 0.0;
  }
  for (int r = threadIdx.x; r < i1 - i0; r += blockDim.x) {
    double b = 0.0;
    for (int y = 0; y <= nchunk; ++y) b += A.rpart[(size_t)y * n + i0 + r];
    bl[r] = b;
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int r = w + 4 * u;
    if (r < i1 - i0) acc += vp[u] * bl[r];
  }
  for (int r0 = w + 4 * kPre; r0 < i1 - i0; r0 += 32) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = r0 + 4 * u;
      v[u] = r < i1 - i0 ? A.fdV[(size_t)(i0 + r) * n + kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = r0 + 4 * u;
      if (r < i1 - i0) acc += v[u] * bl[r];
    }
  }
  part[w][l] = acc;
  __syncthreads();
  if (w == 0 && k < n)
    A.fdz[(size_t)blockIdx.y * n + k] = part[0][l] + part[1][l] + part[2][l] + part[3][l];
}

// Back-projection, split over the eigenvectors: workgroup (row block of 32,
// eigenvector block kb of ceil(n / kFdKb)) forms its scaled coefficients
// z_k / (alpha + beta mu_k) in LDS (kFdSplit projection partials, fixed
// order) and writes the partial sums over its block of 8 rows per wave (lanes
// along k, all loads of a lane issued together); the finalize pass adds the
// kFdKb partials in fixed order.
__global__ __launch_bounds__(256) void k_fd_apply(DevInst I, int d) {
  if (spec_skip(I)) return;
  DevAxis& A = I.ax[d];
  const int n = A.n;
  const int K = (n + kFdKb - 1) / kFdKb;
  const int k0 = blockIdx.y * K;
  const int kn = k0 + K < n ? K : (n > k0 ? n - k0 : 0);
  extern __shared__ double zs[];    // K doubles
  __shared__ double ab[2];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ib = blockIdx.x * 32 + w * 8;
  // the eigenvector values of the first 128 columns of the block are
  // requested before the coefficients are formed
  double vp[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int j = l + 64 * h;
      const int row = ib + r < n ? ib + r : n - 1;
      vp[h][r] = j < kn ? A.fdV[(size_t)row * n + k0 + j] : 0.0;
    }
  if (threadIdx.x == 0) {
    directional_coeffs(I, d, ab[0], ab[1]);
    if (blockIdx.x == 0 && blockIdx.y == 0) {
      I.sc->alpha[d] = ab[0];
      I.sc->beta[d] = ab[1];
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kn; j += blockDim.x) {
    double z[kFdSplit];
#pragma unroll
    for (int s = 0; s < kFdSplit; ++s) z[s] = A.fdz[(size_t)s * n + k0 + j];
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < kFdSplit; ++s) t += z[s];
    zs[j] = t / (ab[0] + ab[1] * A.fdmu[k0 + j]);
  }
  __syncthreads();
  double acc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) acc[r] = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = l + 64 * h;
    const double z = j < kn ? zs[j] : 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] += vp[h][r] * z;
  }
  for (int j0 = l + 128; j0 < kn; j0 += 128) {
    double v[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int j = j0 + 64 * h;
        const int row = ib + r < n ? ib + r : n - 1;
        v[h][r] = j < kn ? A.fdV[(size_t)row * n + k0 + j] : 0.0;
      }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = j0 + 64 * h;
      const double z = j < kn ? zs[j] : 0.0;
#pragma unroll
      for (int r = 0; r < 8; ++r) acc[r] += v[h][r] * z;
    }
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const double t = wave_sum(acc[r]);
    if (l == 0 && ib + r < n) A.fdu[(size_t)blockIdx.y * n + ib + r] = t;
  }
}

hipError_t launch_solve_fd(const DevInst& I, int d, int M, hipStream_t st) {
  const DevAxis& A = I.ax[d];
  if (!A.fdV || !A.fdmu || !A.fdz) return hipErrorInvalidValue;
  const int n = A.n;
  const size_t per = (size_t)(n + kFdSplit - 1) / kFdSplit;
  k_fd_project<<<dim3((n + 63) / 64, kFdSplit), 256, sizeof(double) * per, st>>>(I, d, rhs_chunks(I, d, M, 0));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t K = (size_t)(n + kFdKb - 1) / kFdKb;
  k_fd_apply<<<dim3((n + 31) / 32, kFdKb), 256, sizeof(double) * K, st>>>(I, d);
  return hipGetLastError();
}

// ------------------------------------------------------------ copy
// Plain 16-byte-per-lane copy: reads and writes exactly `bytes` once (the
// reference transfer against which the HBM traffic counters are scaled).
__global__ __launch_bounds__(256) void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                size_t words) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) dst[i] = src[i];
}

hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 16;
  const size_t want = (words + 255) / 256;
  const int blocks = (int)std::min<size_t>(want, (size_t)num_cus() * 16);
  k_copy16<<<blocks, 256, 0, st>>>((uint4*)dst, (const uint4*)src, words);
  return hipGetLastError();
}

// ------------------------------------------------------------ append
// Append the converged rank-one term as mode M and take the enrichment
// decision: stop when its nodal max sigma * prod max|u_d| <= enrich_tol, or
// at the mode cap.
__device__ __forceinline__ void append_body(const DevInst& I, int M) {
  const double sigma = I.sc->sigma[I.dim - 1];
  for (int d = 0; d < I.dim; ++d) {
    const DevAxis& A = I.ax[d];
    for (int i = threadIdx.x; i < A.n; i += blockDim.x) {
      A.X[(size_t)M * A.n + i] = A.u[i];
      A.MX[(size_t)M * A.n + i] = A.Mu[i];
      A.KX[(size_t)M * A.n + i] = A.Ku[i];
    }
  }
  if (threadIdx.x == 0) {
    double pu = 1.0;
    for (int d = 0; d < I.dim; ++d) pu *= I.sc->umax[d];
    const double t = sigma * pu;
    I.sn[M] = sigma;
    I.sc->term_max = t;
    I.sc->nmodes = M + 1;
    I.sc->stop = (t <= I.enrich_tol) ? 1 : ((M + 1 >= I.max_modes) ? 2 : 0);
  }
}

__global__ void k_append(DevInst I, int M) { append_body(I, M); }

hipError_t launch_append(const DevInst& I, int M, hipStream_t st) {
  k_append<<<1, 256, 0, st>>>(I, M);
  return hipGetLastError();
}

__global__ void k_reset_scalars(DevScalars* sc) {
  if (threadIdx.x == 0) {
    sc->done = 0;
    sc->converged = 0;
    sc->zero = 0;
    sc->nonfinite = 0;
    sc->change = -1.0;
    sc->sigma_prev = 0.0;
  }
}

hipError_t launch_reset_scalars(const DevInst& I, hipStream_t st) {
  k_reset_scalars<<<1, 64, 0, st>>>(I.sc);
  return hipGetLastError();
}

// ------------------------------------------------------------ cubic (3D)
// Exact separated evaluation of int N~_i u_e u_f (u^k)^3 on the tensor Gauss
// grid.  With Y = Xh_e (Gauss-point table of u^k along e, sk^(1/3) folded):
//   g_e[a,b,c] = sum_q v_e[q] Y[q,a] Y[q,b] Y[q,c],  v_e = W_e * (Phi_e u_e),
//   h_d[q]     = sum_{a,b,c} X[q,a] X[q,b] X[q,c] g_e[a,b,c] g_f[a,b,c],
// and F_d = omega Phi_d^T W_d h_d.  Both contractions are symmetric in
// (a,b,c); they run over 16-wide mode tiles A <= B <= C only, the tile
// multiplicity (6, 3 or 1) folded into S = wt * g_e * g_f.  Each tile triple
// is an MFMA product with K = q (g) or K = 256 mode pairs (h).
constexpr int kGChunk = 64;

// LDS address space pointer for the direct global-to-LDS loads
#define CTD_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// g over one tile triple and one Gauss-point range (split-K).  The Y rows of
// the A, B, C tiles and v are staged in 64-point chunks, each chunk loaded
// straight from global memory into LDS (global_load_lds, 16-byte words, the
// 64 lanes of a wave filling 64 consecutive words per instruction) while the
// MFMAs of the previous chunk run.  The two chunk buffers are separate arrays
// and the chunk loop is unrolled by two, so that the compiler can tell the
// reads of one buffer from the loads into the other and does not wait on
// them.  The Gauss-point tables Y and v have their row count padded to a
// multiple of 64 with zero rows, so a chunk never reads past them.  Each
// workgroup writes its split partial.
template <class T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 3) void k_cubic_g(DevInst I, int d) {
  if (spec_skip(I)) return;
  typedef typename Vec4<T>::type V;
  constexpr int TS = kTileSq * kTile;
  constexpr int WPS = (int)sizeof(T);               // 16-byte words per 16-wide row segment
  constexpr int RW = 3 * WPS;                       // words per Gauss point: A, B, C segments
  constexpr int NW = RW * kGChunk / 256;            // words per thread per chunk
  constexpr int EPW = 16 / (int)sizeof(T);          // elements per word
  constexpr int VW = kGChunk * (int)sizeof(T) / 16; // words of v per chunk
  const DevAxis& A = I.ax[d];
  const T* Y = (const T*)(sizeof(T) == 4 ? (const void*)A.Xhf : (const void*)A.Xh);
  const T* vq = (const T*)(sizeof(T) == 4 ? (const void*)A.vf : (const void*)A.v);
  const int ldh = I.Mkp;
  // Workgroups are dealt to the 8 XCDs round-robin by linear id; with the
  // split count a multiple of 8, XCD x takes the splits x, x+8, ... of every
  // triple, so each XCD's L2 holds only its own Gauss-point range of Y.
  int t, split;
  if ((I.nsplit_g & 7) == 0) {
    const int b = blockIdx.x, m = I.nsplit_g >> 3, r = b >> 3;
    split = (b & 7) + 8 * (r % m);
    t = r / m;
  } else {
    t = blockIdx.x % I.ntri;
    split = blockIdx.x / I.ntri;
  }
  const int4 tr = I.tri[t];
  const int col0[3] = {tr.x * kTile, tr.y * kTile, tr.z * kTile};
  const int nq = A.nq;
  const int per = ((nq + I.nsplit_g - 1) / I.nsplit_g + kGChunk - 1) / kGChunk * kGChunk;
  const int qbeg = split * per;
  const int qend = qbeg + per < nq ? qbeg + per : nq;
  const int nchunk = qend > qbeg ? (qend - qbeg + kGChunk - 1) / kGChunk : 0;
  // chunk buffers.  FP32 (tile-major table): segment (A, B, C), then point,
  // then the 16 slots of the tile; FP64 (row-major table): point, then
  // segments of 16 values.
  constexpr bool TM = sizeof(T) == 4;
  __shared__ uint4 ysA[kGChunk * RW], ysB[kGChunk * RW];
  __shared__ uint4 vsA[VW], vsB[VW];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const size_t nqp = (size_t)(nq + 63) / 64 * 64;
  // word f = tid + 256 k of a chunk lands at word f of the buffer.  FP32:
  // segment f / 256 (= k), point (f % 256) / 4, part f % 4, so the 64 lanes
  // of a wave read 1 KB of consecutive memory; FP64: point f / RW, segment
  // (f % RW) / WPS, part f % WPS.
  auto load_chunk = [&](int q0, uint4* ys, uint4* vs) {
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int f = tid + 256 * k;
      const T* src;
      if (TM) {
        const int arr = f >> 8, row = (f & 255) >> 2, part = f & 3;
        src = Y + ((size_t)(col0[arr] >> 4) * nqp + q0 + row) * kTile + part * EPW;
      } else {
        const int row = f / RW, rem = f % RW, arr = rem / WPS, part = rem % WPS;
        src = Y + (size_t)(q0 + row) * ldh + col0[arr] + part * EPW;
      }
      __builtin_amdgcn_global_load_lds((const void*)src, CTD_LDS(ys + 256 * k + 64 * w), 16, 0, 0);
    }
    if (w == 0 && l < VW)
      __builtin_amdgcn_global_load_lds((const void*)((const uint4*)(vq + q0) + l), CTD_LDS(vs), 16, 0, 0);
  };
  V acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = V{0, 0, 0, 0};
  auto compute = [&](const uint4* ysw, const uint4* vsw) {
    const T* ys = (const T*)ysw;
    const T* vs = (const T*)vsw;
    // mode e of segment s at point qq: FP32 slot 4 (e % 4) + e / 4
    constexpr int SS = TM ? kGChunk * kTile : kTile;   // segment stride
    constexpr int PS = TM ? kTile : 3 * kTile;         // point stride
    const int e = l & 15;
    const int es = TM ? ((e & 3) << 2) + (e >> 2) : e;
#pragma unroll
    for (int ks = 0; ks < kGChunk / 4; ++ks) {
      const int qq = ks * 4 + (l >> 4);
      const T* yr = ys + qq * PS;
      const T bval = yr[2 * SS + es];
      const T ybv = yr[SS + es] * vs[qq];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // A-segment mode of chain r: FP32 w + 4 r (slot 4 w + r: the wave's
        // four values are one 16-byte word), FP64 4 w + r
        const T aval = yr[w * 4 + r];
        acc[r] = mfma16(aval * ybv, bval, acc[r]);
      }
    }
  };
  auto step = [&](int ci, const uint4* ys, const uint4* vs, uint4* ysn, uint4* vsn) {
    if (ci + 1 < nchunk) load_chunk(qbeg + (ci + 1) * kGChunk, ysn, vsn);
    // the next chunk's loads are issued before the MFMAs
    __builtin_amdgcn_sched_barrier(0);
    compute(ys, vs);
    // the next chunk has landed (the compiler's wait before the barrier
    // covers the direct loads) and every wave is done with this buffer
    __syncthreads();
  };
  if (nchunk > 0) load_chunk(qbeg, ysA, vsA);
  __syncthreads();
  for (int ci = 0; ci < nchunk; ci += 2) {
    step(ci, ysA, vsA, ysB, vsB);
    if (ci + 1 < nchunk) step(ci + 1, ysB, vsB, ysA, vsA);
  }
  T* out = (T*)I.gpart + ((size_t)split * I.ntri + t) * TS;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int al = sizeof(T) == 4 ? w + 4 * r : w * 4 + r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = mfma_row<T>(l, k), j = l & 15;
      out[(al * kTile + i) * kTile + j] = acc[r][k];
    }
  }
}

// g for the FP32 path, by triple class.  A workgroup takes one triple and
// one range of Gauss points (split-K), staged in 64-point chunks as in
// k_cubic_g (global_load_lds into two buffers, one barrier per chunk), from
// the point-grouped copy of the table (a 16-byte word holds one mode at four
// consecutive points, so one LDS read serves four k-steps).
// Triples of three distinct tiles (A < B < C): each wave runs 4 of the 16
// chains (mode a of A) over every point of a chunk, output blocks (b, c).
// Triples with a repeated tile hold each unordered mode pair of that tile
// once: 136 pairs in 9 blocks of 16 rows, row i of block k the pair
// (i, i + k mod 16) (block 8 holds each of its 8 pairs twice), against the
// 16 modes of the other tile as columns; for A = B <= C the pairs are those
// of A against C, for A < B = C those of B against A.  There each wave runs
// the 9 blocks over 16 of a chunk's 64 points, the A operand of row i the
// product Y_i Y_{i+k} v of the point, and the four waves' sums are added in
// LDS at the end.  9 blocks instead of 16 chains: the repeated-tile
// triples run about 16/9 as many points per split (more points, fewer
// splits), so all workgroups carry about the same work.
__global__ __launch_bounds__(256, 4) void k_cubic_g32(DevInst I, int d) {
  if (spec_skip(I)) return;
  constexpr int TS = kTileSq * kTile;
  constexpr int PS9 = 9 * kTileSq;                  // outputs of a repeated-tile triple
  constexpr int RW = 12;                            // 16-byte words per Gauss point (3 segments)
  constexpr int NW = RW * kGChunk / 256;            // words per thread per chunk
  constexpr int VW = kGChunk * 4 / 16;              // words of v per chunk
  constexpr int SS = kGChunk * kTile;               // segment stride (floats)
  const DevAxis& A = I.ax[d];
  const float* Y = A.Xhg;
  const float* vq = A.vf;
  const int nd = I.ntri_d, np = I.ntri_p;
  const int b = blockIdx.x;
  int rank, split, t;
  bool rep;
  // Workgroups go round-robin over the 8 XCDs (b % 8).  With split counts
  // that are multiples of 8, XCD x takes splits [x n/8, (x+1) n/8) of every
  // triple, so each XCD's L2 holds only its eighth of the Gauss-point tables
  // (every triple of a split reads the same point range).
  auto place = [&](int bb, int ntr, int nsp) {
    if ((nsp & 7) == 0) {
      const int x = b & 7, idx = bb >> 3;
      rank = idx % ntr;
      split = x * (nsp >> 3) + idx / ntr;
    } else {
      rank = bb % ntr;
      split = bb / ntr;
    }
  };
  if (b < nd * I.nsplit_g) {
    place(b, nd, I.nsplit_g);
    rep = false;
    t = I.tlist[rank];
  } else {
    // the XCD of b is that of b2 when the distinct block count is a multiple of 8
    const int b2 = b - nd * I.nsplit_g;
    if (((nd * I.nsplit_g) & 7) == 0) place(b2, np, I.nsplit_p);
    else { rank = b2 % np; split = b2 / np; }
    rep = true;
    t = I.tlist_p[rank];
  }
  const int nsplit = rep ? I.nsplit_p : I.nsplit_g;
  const int4 tr = I.tri[t];
  const int col0[3] = {tr.x * kTile, tr.y * kTile, tr.z * kTile};
  const int nq = A.nq;
  const int per = ((nq + nsplit - 1) / nsplit + kGChunk - 1) / kGChunk * kGChunk;
  const int qbeg = split * per;
  const int qend = qbeg + per < nq ? qbeg + per : nq;
  const int nchunk = qend > qbeg ? (qend - qbeg + kGChunk - 1) / kGChunk : 0;
  __shared__ uint4 ysA[kGChunk * RW], ysB[kGChunk * RW];
  __shared__ uint4 vsA[VW], vsB[VW];
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const size_t nqp = (size_t)(nq + 63) / 64 * 64;
  // word f = tid + 256 k of a chunk: segment f / 256 (= k), point group
  // (f % 256) / 16, mode f % 16 (four consecutive points of one mode per
  // word; a wave reads 1 KB of consecutive memory)
  auto load_chunk = [&](int q0, uint4* ys, uint4* vs) {
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int f = tid + 256 * k;
      const int arr = f >> 8, wi = f & 255;
      const float* src = Y + (((size_t)(col0[arr] >> 4) * (nqp >> 2) + (q0 >> 2)) * 16 + wi) * 4;
      __builtin_amdgcn_global_load_lds((const void*)src, CTD_LDS(ys + 256 * k + 64 * w), 16, 0, 0);
    }
    if (w == 0 && l < VW)
      __builtin_amdgcn_global_load_lds((const void*)((const uint4*)(vq + q0) + l), CTD_LDS(vs), 16, 0, 0);
  };
  const int e = l & 15, kk = l >> 4;   // A row / B column mode e; MFMA k index kk
  auto chunk_loop = [&](auto compute) {
    auto step = [&](int ci, const uint4* ys, const uint4* vs, uint4* ysn, uint4* vsn) {
      if (ci + 1 < nchunk) load_chunk(qbeg + (ci + 1) * kGChunk, ysn, vsn);
      __builtin_amdgcn_sched_barrier(0);
      compute((const float*)ys, (const float*)vs);
      __syncthreads();
    };
    if (nchunk > 0) load_chunk(qbeg, ysA, vsA);
    __syncthreads();
    for (int ci = 0; ci < nchunk; ci += 2) {
      step(ci, ysA, vsA, ysB, vsB);
      if (ci + 1 < nchunk) step(ci + 1, ysB, vsB, ysA, vsA);
    }
  };
  float* gp = (float*)I.gpart;
  if (!rep) {
    f4 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = f4{0, 0, 0, 0};
    // lane group kk takes the chunk's points 16 kk .. 16 kk + 15, four per
    // 16-byte word: per word group the B-row, C-column, v and the wave's
    // four A-mode values are one LDS read each, for four k-steps
    chunk_loop([&](const float* ys, const float* vs) {
      const float4* yw = (const float4*)ys;
      const float4* vw = (const float4*)vs;
#pragma unroll
      for (int G = 0; G < 4; ++G) {
        const int grp = 4 * kk + G;
        const float4 yb = yw[256 + grp * 16 + e];
        const float4 yc = yw[512 + grp * 16 + e];
        const float4 vv = vw[grp];
        float4 ya[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) ya[r] = yw[grp * 16 + w + 4 * r];   // chain r: mode w + 4 r of A
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const float ybv = yb[p] * vv[p];
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] = mfma16(ya[r][p] * ybv, yc[p], acc[r]);
        }
      }
    });
    float* out = gp + ((size_t)rank * I.nsplit_g + split) * TS;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        out[((w + 4 * r) * kTile + mfma_row<float>(l, k)) * kTile + (l & 15)] = acc[r][k];
    return;
  }
  // repeated tile: pair tile and column tile (segments of the chunk)
  const bool p2 = tr.x < tr.y;                        // A < B = C: pairs of B, columns A
  const int pa = p2 ? 1 : 0, pc = p2 ? 0 : 2;
  f4 acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = f4{0, 0, 0, 0};
  // wave w takes the chunk's points 16 w .. 16 w + 15, lane group kk four
  // of them (one word group); the pair tile's modes e .. e + 8 (mod 16),
  // the column mode e and v are one LDS read each for four k-steps
  chunk_loop([&](const float* ys, const float* vs) {
    const float4* yw = (const float4*)ys;
    const float4* vw = (const float4*)vs;
    const int grp = 4 * w + kk;
    float4 yp[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) yp[k] = yw[pa * 256 + grp * 16 + ((e + k) & 15)];
    const float4 yc = yw[pc * 256 + grp * 16 + e];
    const float4 vv = vw[grp];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const float own = yp[0][p] * vv[p];
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[k] = mfma16(own * yp[k][p], yc[p], acc[k]);
    }
  });
  // add the four waves' sums (wave order), three blocks at a time
  float* red = (float*)ysA;                           // 3 waves x 3 blocks x 256 values
  float* out = gp + (size_t)nd * I.nsplit_g * TS + ((size_t)rank * I.nsplit_p + split) * PS9;
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    if (w > 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) red[(((w - 1) * 3 + r) * 4 + k) * 64 + l] = acc[h * 3 + r][k];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int blk = h * 3 + r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float sum = acc[blk][k];
#pragma unroll
          for (int u = 0; u < 3; ++u) sum += red[((u * 3 + r) * 4 + k) * 64 + l];
          out[(blk * kTile + mfma_row<float>(l, k)) * kTile + (l & 15)] = sum;
        }
      }
    }
    __syncthreads();
  }
}

// The 40 k-steps ks = 4 j + u (u >= j / 4) of a repeated-tile triple in
// packed order: blocks J = j / 4 of 4 (4 - J) k-steps, j-major inside.
__host__ __device__ constexpr int packed_ks_base(int J) { return 4 * (4 * J - J * (J - 1) / 2); }
__host__ __device__ constexpr int packed_ks_block(int p) {
  return p < packed_ks_base(1) ? 0 : p < packed_ks_base(2) ? 1 : p < packed_ks_base(3) ? 2 : 3;
}
__host__ __device__ constexpr int packed_ks_j(int p) {
  return 4 * packed_ks_block(p) + (p - packed_ks_base(packed_ks_block(p))) / (4 - packed_ks_block(p));
}
__host__ __device__ constexpr int packed_ks_u(int p) {
  return packed_ks_block(p) + (p - packed_ks_base(packed_ks_block(p))) % (4 - packed_ks_block(p));
}
static_assert(packed_ks_j(39) == 15 && packed_ks_u(39) == 3 && packed_ks_j(16) == 4 &&
                  packed_ks_u(16) == 1 && packed_ks_j(15) == 3 && packed_ks_u(15) == 3,
              "packed k-step order");

// Split-K reduction of the FP32 g by class (fixed split order), and S = w g_d
// g_other in the h kernel's order and layout.  One thread per element of an
// h tile (first mode, second mode, column mode); for a repeated-tile triple
// the element reads its pair's block and row ((f, s) with s - f = k <= 8:
// block k, row f; else block 16 - k, row s), and pairs with f > s are zero.
// g_d is kept in the class layout (only the elements read here are written).
__global__ __launch_bounds__(256) void k_cubic_gred32(DevInst I, int d, int e_other) {
  if (spec_skip(I)) return;
  constexpr int TS = kTileSq * kTile;
  constexpr int PS9 = 9 * kTileSq;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)I.ntri * TS) return;
  const int p = (int)(idx / TS);
  const int eh = (int)(idx - (size_t)p * TS);
  const int f = eh >> 8, sc = (eh >> 4) & 15, col = eh & 15;
  const int t = I.thinv[p];
  const int2 cr = I.trank[t];
  const int nd = I.ntri_d;
  const float* gp = (const float*)I.gpart;
  size_t base, stride, goff;
  int ns, el;
  double pw = 1.0;
  if (cr.x == 0) {
    el = eh;                                           // distinct tiles: (a, b, c) = (f, s, col)
    base = (size_t)cr.y * I.nsplit_g * TS;
    stride = TS;
    ns = I.nsplit_g;
    goff = (size_t)cr.y * TS;
  } else {
    pw = f < sc ? 2.0 : (f == sc ? 1.0 : 0.0);
    const int k = sc - f;
    const int blk = k <= 8 ? k : 16 - k, row = k <= 8 ? f : sc;
    el = (blk * kTile + row) * kTile + col;
    base = (size_t)nd * I.nsplit_g * TS + (size_t)cr.y * I.nsplit_p * PS9;
    stride = PS9;
    ns = I.nsplit_p;
    goff = (size_t)nd * TS + (size_t)cr.y * PS9;
  }
  float* gd = (float*)I.ax[d].g;
  double s = 0.0;
  if (pw != 0.0) {
    int sp = 0;
    for (; sp + 8 <= ns; sp += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = gp[base + (size_t)(sp + u) * stride + el];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; sp < ns; ++sp) s += (double)gp[base + (size_t)sp * stride + el];
    gd[goff + el] = (float)s;
  }
  if (e_other >= 0) {
    const float* go = (const float*)I.ax[e_other].g;
    const float val = pw == 0.0 ? 0.0f : (float)((double)I.tri[t].w * pw * s * (double)go[goff + el]);
    // element eh = 64 ks + l of the tile (k-step ks, lane l) goes where lane
    // l finds k-steps 4j..4j+3 in one 16-byte word: ((j 64 + l) 4 + ks % 4).
    // A repeated-tile triple keeps only the k-steps ks = 4 j + u with
    // u >= j / 4 (the others pair a first mode j above all four second modes
    // 4u..4u+3), packed in (j, u) order: position 4 (4J - J(J-1)/2) +
    // (j % 4)(4 - J) + u - J for J = j / 4.
    const int ks = eh >> 6, l = eh & 63;
    int pk = ks;
    if (cr.x != 0) {
      const int j = ks >> 2, u = ks & 3, J = j >> 2;
      if (u < J) return;
      pk = packed_ks_base(J) + (j & 3) * (4 - J) + (u - J);
    }
    ((float*)I.S)[(size_t)p * TS + ((((pk >> 2) << 6) + l) << 2) + (pk & 3)] = val;
  }
}

// Split-K reduction of g in fixed split order, and S = w g_d g_other.  A
// separate launch: a cross-workgroup reduction inside k_cubic_g needs device-
// scope fences, whose L2 write-back/invalidate on this chip costs more than
// the extra launch.
template <class T>
__global__ __launch_bounds__(256) void k_cubic_gred(DevInst I, int d, int e_other) {
  if (spec_skip(I)) return;
  const size_t per = (size_t)kTileSq * kTile;
  const size_t total = (size_t)I.ntri * per;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const T* gp = (const T*)I.gpart;
  double s = 0.0;
  // fixed split order; eight loads in flight at a time
  int sp = 0;
  for (; sp + 8 <= I.nsplit_g; sp += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = gp[(size_t)(sp + u) * total + idx];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)v[u];
  }
  for (; sp < I.nsplit_g; ++sp) s += (double)gp[(size_t)sp * total + idx];
  ((T*)I.ax[d].g)[idx] = (T)s;
  if (e_other >= 0) {
    const int t = (int)(idx / per);
    const T* go = (const T*)I.ax[e_other].g;
    const int4 tr = I.tri[t];
    const int2 hm = I.trimap[t];
    const int e = (int)(idx - (size_t)t * per);
    // tile element e = (a 16 + b) 16 + c of triple (A, B, C).  h runs the
    // triple at position hm.x of its own order over (first, second) mode
    // pairs against a column tile: (a, b) against c, or for A < B = C
    // (hm.y = 1) the pairs (b, c) against a, so the element goes to
    // e' = (b 16 + c) 16 + a.  Where the two pair tiles coincide only pairs
    // first <= second are taken: weight 2 off the diagonal, 1 on it, 0 below
    // (S is symmetric in the pair there).
    const int a = e >> 8, b = (e >> 4) & 15, c = e & 15;
    const int f = hm.y ? b : a, sec = hm.y ? c : b, col = hm.y ? a : c;
    double wt = (double)tr.w;
    if (hm.y || tr.x == tr.y) wt *= f < sec ? 2.0 : (f == sec ? 1.0 : 0.0);
    const T val = (T)(wt * s * (double)go[idx]);
    const int eh = (f * 16 + sec) * 16 + col;
    size_t dst = (size_t)hm.x * per + eh;
    if (sizeof(T) == 4) {
      // element eh = 64 ks + l of the tile (k-step ks, lane l) goes where lane
      // l finds k-steps 4j..4j+3 in one 16-byte word: ((j 64 + l) 4 + ks % 4)
      const int ks = eh >> 6, l = eh & 63;
      dst = (size_t)hm.x * per + ((((ks >> 2) << 6) + l) << 2) + (ks & 3);
    }
    ((T*)I.S)[dst] = val;
  }
}


// h for the FP32 path.  A workgroup of 8 waves owns 128 Gauss points (16 per
// wave, the MFMA columns) and walks its share of the tile triples; every
// MFMA takes the S tile as its A operand (rows: the 16 column modes c;
// k-steps: mode pairs) and the pair products X_a X_b of the wave's points
// as its B operand, so that the output holds the lane's own point in its
// column and the closing sum over c with X_c is lane-local except for the
// four lane groups' rows.
// Per triple the workgroup stages the S tile and the first tile's factor
// rows at its 128 points in LDS (double-buffered, 24 KB each; S in the
// order k_cubic_gred32 writes it: lane l finds four k-steps in one 16-byte
// word), so the 16 waves of two workgroups share one copy per CU of what
// the MFMAs read most; each lane loads the second tile's four B modes of
// its point (one 16-byte word of the tile-major table) itself, and the
// column tile's values only where a column closes.  The next triple's data
// are fetched while the MFMAs of the current one run and stored to the
// other buffer after them (one barrier per triple).
constexpr int kHWaves = 8;                 // waves per workgroup
constexpr int kHQ = 16 * kHWaves;          // Gauss points per workgroup
constexpr int kHThreads = 64 * kHWaves;
constexpr int kHBufWords = kTileSq * kTile / 4 + kHQ * kTile / 4;   // S tile + first-tile rows

__global__ __launch_bounds__(kHThreads) void k_cubic_h32(DevInst I, int d) {
  if (spec_skip(I)) return;
  extern __shared__ unsigned char smraw[];
  constexpr int TW = kTileSq * kTile / 4;   // 16-byte words per S tile
  static_assert(TW == 2 * kHThreads && kHQ * kTile / 4 == kHThreads, "three staged words per thread");
  const DevAxis& A = I.ax[d];
  const float* X = (const float*)A.Xhf;
  const int nq = A.nq;
  float4* sb = (float4*)smraw;           // 2 x (S tile, first-tile rows)
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int g = l >> 4;                  // lane group: k index of the operands
  const int q0 = blockIdx.x * kHQ;
  const int qw = q0 + w * 16;            // first Gauss point of this wave
  const int split = blockIdx.y;
  int t0, t1;
  if (I.hsb_n == I.nsplit_h) {
    t0 = I.hsb[split];
    t1 = I.hsb[split + 1];
  } else {
    const int per = (I.ntri + I.nsplit_h - 1) / I.nsplit_h;
    t0 = split * per;
    t1 = t0 + per < I.ntri ? t0 + per : I.ntri;
  }
  // Points past the end read the last point (their sums are never stored).
  // The table is tile-major over the 64-padded point count, mode i of a tile
  // in slot 4 (i % 4) + i / 4 (16-byte word i % 4).
  const size_t nqp = (size_t)(nq + 63) / 64 * 64;
  const int qa = qw + (l & 15) < nq ? qw + (l & 15) : nq - 1;        // the lane's point
  const int qs = q0 + (tid >> 2) < nq ? q0 + (tid >> 2) : nq - 1;    // the staging row of this thread
  const int xrow = (w * 16 + (l & 15)) * 4;                          // the lane's row in the staged rows
  // loads use a clamped triple index so they are unconditional (the surplus
  // lands in the idle buffer)
  const int tlast = t1 > t0 ? t1 - 1 : 0;
  auto tcl = [&](int t) { return t < tlast ? t : tlast; };
  const float4* Sp = (const float4*)I.S;
  float4 pre0, pre1, pre2;
  float xb[4], xbn[4], xc[4];
  auto fetch = [&](int tt, int4 tr) __attribute__((always_inline)) {
    const float4* src = Sp + (size_t)tt * TW + tid;
    pre0 = src[0];
    pre1 = src[kHThreads];
    pre2 = *(const float4*)(X + ((size_t)tr.x * nqp + qs) * kTile + 4 * (tid & 3));
    const float4 bq = *(const float4*)(X + ((size_t)tr.y * nqp + qa) * kTile + 4 * g);
    xbn[0] = bq.x; xbn[1] = bq.y; xbn[2] = bq.z; xbn[3] = bq.w;
  };
  auto stage = [&](float4* dst) __attribute__((always_inline)) {
    dst[tid] = pre0;
    dst[kHThreads + tid] = pre1;
    dst[TW + tid] = pre2;
  };
  // the triple table two ahead (scalar loads consumed an iteration later)
  int4 thc = I.trih[tcl(t0)], thn = I.trih[tcl(t0 + 1)];
  fetch(tcl(t0), thc);
  stage(sb);
#pragma unroll
  for (int v = 0; v < 4; ++v) xb[v] = xbn[v];
  __syncthreads();
  double hq = 0.0;
  f4 acc = f4{0, 0, 0, 0};
  int curC = -1;
  // h[q] += sum over the lane's column modes c = 4 g + r of X_c[q] acc[c, q],
  // then over the four lane groups
  auto close_c = [&]() __attribute__((always_inline)) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) v += (double)acc[r] * (double)xc[r];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    hq += v;
    acc = f4{0, 0, 0, 0};
  };
  for (int t = t0; t < t1; ++t) {
    const int4 th = thc;
    // the previous column closes before the prefetch is issued, so that the
    // prefetch's loads stay in flight across the MFMAs
    if (th.z != curC) {
      if (curC >= 0) close_c();
      curC = th.z;
    }
    const int4 thnn = I.trih[tcl(t + 2)];
    fetch(tcl(t + 1), thn);
    if (t + 1 >= t1 || thn.z != th.z) {
      // this triple closes its column: X_c of the lane's modes c = 4 g + r
      // (slot 4 r + g of the point's row)
      const float* xr = X + ((size_t)th.z * nqp + qa) * kTile + g;
#pragma unroll
      for (int r = 0; r < 4; ++r) xc[r] = xr[4 * r];
    }
    const float4* sq = sb + ((t - t0) & 1) * kHBufWords;
    float4 xa4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) xa4[v] = sq[TW + xrow + v];
    // k-step ks = 4 j + u: first mode a = j (word j % 4, slot j / 4 of the
    // point's row), second modes b = 4 u + k over the operands' k index (the
    // lane group).  When the pairs are taken once (first tile = second
    // tile), the k-steps whose four b all lie below a (u < j / 4) meet only
    // zero weights; S holds the other 40 k-steps packed in order, so both
    // forms read whole 16-byte words and branch once per triple.  The
    // schedule is pinned (sched_group_barrier; 0x100 LDS read, 0x002 VALU,
    // 0x008 MFMA): S words read three ahead, each product issued just before
    // its MFMA.
    if (th.w == 0) {
#pragma unroll
      for (int j = 0; j < kTileSq / 16; ++j) {
        const float4 b4 = sq[j * 64 + l];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = mfma16(b4[u], xa4[j & 3][j >> 2] * xb[u], acc);
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
      for (int j = 0; j < kTileSq / 16; ++j) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
        if (j + 3 < kTileSq / 16) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
    } else {
      float4 b4;
#pragma unroll
      for (int p = 0; p < 40; ++p) {
        const int j = packed_ks_j(p), u = packed_ks_u(p);
        if ((p & 3) == 0) b4 = sq[(p >> 2) * 64 + l];
        acc = mfma16(b4[p & 3], xa4[j & 3][j >> 2] * xb[u], acc);
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
      for (int p = 0; p < 40; ++p) {
        __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if ((p & 3) == 3 && (p >> 2) + 3 < 10) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
    }
    stage(sb + ((t + 1 - t0) & 1) * kHBufWords);
#pragma unroll
    for (int v = 0; v < 4; ++v) xb[v] = xbn[v];
    __syncthreads();
    thc = thn;
    thn = thnn;
  }
  if (curC >= 0) close_c();
  if (g == 0 && qw + (l & 15) < nq) I.hpart[(size_t)split * nq + qw + (l & 15)] = hq;
}

// Row stride of the LDS copy of the Gauss-point factor rows in k_cubic_h:
// one 16-byte word of padding makes the stride an odd number of words, so the
// 16 rows that the lane groups of a wave read at once fall in distinct banks.
template <class T>
__host__ __device__ constexpr int h_lds_stride(int ldh) { return ldh + 16 / (int)sizeof(T); }

template <class T>
__global__ __launch_bounds__(256) void k_cubic_h(DevInst I, int d) {
  if (spec_skip(I)) return;
  typedef typename Vec4<T>::type V;
  constexpr int TS = kTileSq * kTile;                 // elements per S tile
  constexpr int NV = TS * (int)sizeof(T) / 16 / 256;  // 16-byte words per thread
  extern __shared__ unsigned char smraw[];
  const DevAxis& A = I.ax[d];
  const T* X = (const T*)(sizeof(T) == 4 ? (const void*)A.Xhf : (const void*)A.Xh);
  const int ldh = I.Mkp;
  const int ldx = h_lds_stride<T>(ldh);    // padded: the 16 rows a lane group reads hit distinct banks
  const int nq = A.nq;
  T* xs = (T*)smraw;                       // 64 x ldx
  T* sb = xs + 64 * ldx;                   // 2 x (256 x 16)
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int q0 = blockIdx.x * 64;
  const int split = blockIdx.y;
  int t0, t1;
  if (I.hsb_n == I.nsplit_h) {
    t0 = I.hsb[split];
    t1 = I.hsb[split + 1];
  } else {
    const int per = (I.ntri + I.nsplit_h - 1) / I.nsplit_h;
    t0 = split * per;
    t1 = t0 + per < I.ntri ? t0 + per : I.ntri;
  }
  for (int idx = tid; idx < 64 * ldh; idx += 256) {
    const int qq = idx / ldh, c = idx % ldh, q = q0 + qq;
    xs[qq * ldx + c] = q < nq ? X[(size_t)q * ldh + c] : (T)0;
  }
  // Prefetch registers; loads are unconditional from a clamped tile index
  // (the surplus store lands in the idle buffer) so they stay in VGPRs.
  const int tlast = t1 > t0 ? t1 - 1 : 0;
  uint4 pre[NV];
  {
    const int tt = t0 < tlast ? t0 : tlast;
    const uint4* src = (const uint4*)((const T*)I.S + (size_t)tt * TS);
#pragma unroll
    for (int v = 0; v < NV; ++v) pre[v] = src[tid * NV + v];
    uint4* dst = (uint4*)sb;
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[tid * NV + v] = pre[v];
  }
  __syncthreads();
  const int rowA = w * 16 + (l & 15);     // A-operand row (q) of this lane
  double hq[4] = {0, 0, 0, 0};
  V acc = V{0, 0, 0, 0};
  int curC = -1;
  for (int t = t0; t < t1; ++t) {
    const int4 tr = I.trih[t];
    {
      const int tn = t + 1 < tlast ? t + 1 : tlast;
      const uint4* src = (const uint4*)((const T*)I.S + (size_t)tn * TS);
#pragma unroll
      for (int v = 0; v < NV; ++v) pre[v] = src[tid * NV + v];
    }
    if (tr.z != curC) {
      if (curC >= 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = w * 16 + mfma_row<T>(l, r);
          double v = (double)acc[r] * (double)xs[row * ldx + curC * kTile + (l & 15)];
          v += __shfl_xor(v, 8, 64);
          v += __shfl_xor(v, 4, 64);
          v += __shfl_xor(v, 2, 64);
          v += __shfl_xor(v, 1, 64);
          hq[r] += v;
        }
      }
      acc = V{0, 0, 0, 0};
      curC = tr.z;
    }
    const T* ss = sb + ((t - t0) & 1) * TS;
    const int A0 = tr.x * kTile, B0 = tr.y * kTile;
    T xa[kTile], xb[4];
#pragma unroll
    for (int a = 0; a < kTile; ++a) xa[a] = xs[rowA * ldx + A0 + a];
#pragma unroll
    for (int m = 0; m < 4; ++m) xb[m] = xs[rowA * ldx + B0 + 4 * m + (l >> 4)];
    // symmetric pair skip when the pair tiles coincide (as in the FP32 kernel)
    const bool full = tr.w == 0;
#pragma unroll
    for (int ks = 0; ks < kTileSq / 4; ++ks) {
      if ((ks & 3) < (ks >> 4) && !full) continue;
      const T aval = xa[ks >> 2] * xb[ks & 3];
      const T bval = ss[(4 * ks + (l >> 4)) * kTile + (l & 15)];
      acc = mfma16(aval, bval, acc);
    }
    {
      uint4* dst = (uint4*)(sb + ((t + 1 - t0) & 1) * TS);
#pragma unroll
      for (int v = 0; v < NV; ++v) dst[tid * NV + v] = pre[v];
    }
    __syncthreads();
  }
  if (curC >= 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + mfma_row<T>(l, r);
      double v = (double)acc[r] * (double)xs[row * ldx + curC * kTile + (l & 15)];
      v += __shfl_xor(v, 8, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 1, 64);
      hq[r] += v;
    }
  }
  if ((l & 15) == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = q0 + w * 16 + mfma_row<T>(l, r);
      if (q < nq) I.hpart[(size_t)split * nq + q] = hq[r];
    }
  }
}

hipError_t launch_cubic_g(const DevInst& I, int d, hipStream_t st) {
  if (I.mixed) {
    const int grid = I.ntri_d * I.nsplit_g + I.ntri_p * I.nsplit_p;
    k_cubic_g32<<<grid, 256, 0, st>>>(I, d);
  } else {
    k_cubic_g<double><<<I.ntri * I.nsplit_g, 256, 0, st>>>(I, d);
  }
  return hipGetLastError();
}

hipError_t launch_cubic_gred(const DevInst& I, int d, int e_other, hipStream_t st) {
  const size_t total = (size_t)I.ntri * kTileSq * kTile;
  const int blocks = (int)((total + 255) / 256);
  if (I.mixed) k_cubic_gred32<<<blocks, 256, 0, st>>>(I, d, e_other);
  else k_cubic_gred<double><<<blocks, 256, 0, st>>>(I, d, e_other);
  return hipGetLastError();
}

size_t cubic_h_lds(const DevInst& I) {
  if (I.mixed) return sizeof(float4) * 2 * kHBufWords;
  return sizeof(double) * (64 * (size_t)h_lds_stride<double>(I.Mkp) + 2 * kTileSq * kTile);
}

int cubic_h_rows(const DevInst& I) { return I.mixed ? kHQ : 64; }

int cubic_h_threads(const DevInst& I) { return I.mixed ? kHThreads : 256; }

size_t cubic_h_lds_total(const DevInst& I) { return cubic_h_lds(I); }

int cubic_h_blocks_per_cu(const DevInst& I) {
  // resident workgroups per CU as the runtime computes them (registers and
  // LDS), cached per LDS size
  static thread_local size_t last_shm[2] = {0, 0};
  static thread_local int last_nb[2] = {0, 0};
  const int k = I.mixed ? 1 : 0;
  const size_t shm = cubic_h_lds(I);
  if (last_nb[k] == 0 || last_shm[k] != shm) {
    int nb = 0;
    const void* f = I.mixed ? (const void*)k_cubic_h32 : (const void*)k_cubic_h<double>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, cubic_h_threads(I), shm) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = std::max(1, (int)((size_t)max_lds_bytes() / shm));
    }
    last_shm[k] = shm;
    last_nb[k] = nb;
  }
  return last_nb[k];
}

hipError_t launch_cubic_h(const DevInst& I, int d, hipStream_t st) {
  const int nq = I.ax[d].nq;
  const int rows = cubic_h_rows(I);
  dim3 grid((nq + rows - 1) / rows, I.nsplit_h);
  if (I.mixed) {
    k_cubic_h32<<<grid, kHThreads, cubic_h_lds(I), st>>>(I, d);
  } else {
    k_cubic_h<double><<<grid, 256, cubic_h_lds(I), st>>>(I, d);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ M_xy (2D)
// Full integration of M_xy = int N~_x^T N~_y L w(u^k) (eq. KxxMxx) on the
// tensor Gauss grid: U = Xh_0 Xh_1^T and G = omega (U^3 - U) W_0 W_1 by the
// FP64 MFMA product (a strip of whole elements of axis 0 at a time, so the
// Gauss-grid buffer stays bounded), T1 = Phi_0^T G accumulated per strip
// (gathered per node, elements in increasing order), M_xy = T1 Phi_1.  With
// rd_tol > 0 each strip first drops the elements outside the reduced domain.
__global__ void k_mxy_t1_strip(DevInst I, int r0, int r1, int i_lo, int i_hi) {
  const DevAxis& X = I.ax[0];
  const int nqy = I.ax[1].nq;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)(i_hi - i_lo) * nqy) return;
  const int i = i_lo + (int)(idx / nqy), qy = (int)(idx % nqy);
  const int n = X.n, ne = n - 1;
  int e0 = i - X.SW;
  e0 = e0 < 0 ? 0 : e0;
  int e1 = i + X.SW;
  e1 = e1 > ne - 1 ? ne - 1 : e1;
  // elements of this strip: rows [r0, r1) are whole elements
  const int ea = r0 / X.ng, eb = r1 / X.ng;
  e0 = e0 < ea ? ea : e0;
  e1 = e1 > eb - 1 ? eb - 1 : e1;
  double acc = 0.0;
  for (int e = e0; e <= e1; ++e) {
    const int st = elem_start(e, X.s, n, X.SW);
    const int jj = i - st;
    if (jj < 0 || jj >= X.SW) continue;
    for (int g = 0; g < X.ng; ++g) {
      const int qx = e * X.ng + g;
      acc += X.phi[(size_t)qx * X.SW + jj] * I.Gq[(size_t)(qx - r0) * nqy + qy];
    }
  }
  I.T1[(size_t)i * nqy + qy] += acc;
}

// Reduced integration domain (Sec. 3.3, eq. MxyRD) on a strip of the Gauss
// grid: an element whose Gauss-point values of w(u^k) = 4 a0 (u^3 - u) all
// satisfy |w| <= rd_tol leaves M_xy.  The strip holds G = omega (u^3 - u)
// W_0 W_1 with omega = 4 a0 L, so the test reads 4 a0 |G| <= rd_tol omega
// W_0 W_1 (no division).  One thread per element; the values of a dropped
// element are zeroed and the dropped elements counted.
__global__ void k_mxy_mask(DevInst I, int r0, int r1) {
  const DevAxis& X = I.ax[0];
  const DevAxis& Y = I.ax[1];
  const int ng0 = X.ng, ng1 = Y.ng, nq1 = Y.nq;
  const int ne1 = nq1 / ng1, nes = (r1 - r0) / ng0;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool drop = false;
  if (idx < (size_t)nes * ne1) {
    const int ex = (int)(idx / ne1), ey = (int)(idx % ne1);
    const double lhs = 4.0 * I.a0, rhs = I.rd_tol * I.omega;
    double* G = I.Gq + (size_t)ex * ng0 * nq1 + (size_t)ey * ng1;
    drop = true;
    for (int gx = 0; gx < ng0 && drop; ++gx) {
      const double wx = rhs * X.w[r0 + ex * ng0 + gx];
      for (int gy = 0; gy < ng1; ++gy)
        if (lhs * fabs(G[(size_t)gx * nq1 + gy]) > wx * Y.w[ey * ng1 + gy]) { drop = false; break; }
    }
    if (drop)
      for (int gx = 0; gx < ng0; ++gx)
        for (int gy = 0; gy < ng1; ++gy) G[(size_t)gx * nq1 + gy] = 0.0;
  }
  const unsigned long long m = __ballot(drop);
  if ((threadIdx.x & 63) == 0 && m != 0) atomicAdd(I.rd_count, (unsigned long long)__popcll(m));
}

__global__ void k_mxy_count_reset(DevInst I) { *I.rd_count = 0; }

template <class T>
__global__ void k_mxy_t2(DevInst I) {
  const DevAxis& X = I.ax[0];
  const DevAxis& Yx = I.ax[1];
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ny = Yx.n, nx = X.n;
  if (idx >= (size_t)nx * ny) return;
  const int i = (int)(idx / ny), j = (int)(idx % ny);
  const int ne = ny - 1;
  int e0 = j - Yx.SW;
  e0 = e0 < 0 ? 0 : e0;
  int e1 = j + Yx.SW;
  e1 = e1 > ne - 1 ? ne - 1 : e1;
  const double* t1 = I.T1 + (size_t)i * Yx.nq;
  double acc = 0.0;
  for (int e = e0; e <= e1; ++e) {
    const int st = elem_start(e, Yx.s, ny, Yx.SW);
    const int jj = j - st;
    if (jj < 0 || jj >= Yx.SW) continue;
    for (int g = 0; g < Yx.ng; ++g) {
      const int qy = e * Yx.ng + g;
      acc += t1[qy] * Yx.phi[(size_t)qy * Yx.SW + jj];
    }
  }
  ((T*)I.Mxy)[(size_t)i * ny + j] = (T)acc;
  ((T*)I.MxyT)[(size_t)j * nx + i] = (T)acc;
}

hipError_t launch_mxy_build(const DevInst& I, hipStream_t st) {
  const DevAxis& X = I.ax[0];
  const int nq0 = X.nq, nq1 = I.ax[1].nq;
  hipError_t e = launch_fill(I.T1, X.n * nq1, 0.0, st);
  if (e != hipSuccess) return e;
  const bool reduced = I.rd_tol > 0.0;
  if (reduced) {
    k_mxy_count_reset<<<1, 1, 0, st>>>(I);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int r0 = 0; r0 < nq0; r0 += I.gq_rows) {
    const int r1 = r0 + I.gq_rows < nq0 ? r0 + I.gq_rows : nq0;
    GemmArgs g;
    g.m = r1 - r0; g.n = nq1; g.K = I.Mk; g.epi = kEpiCubic;
    g.A = X.Xh + (size_t)r0 * I.Mkp; g.a_i = I.Mkp; g.a_k = 1;
    g.B = I.ax[1].Xh; g.b_k = 1; g.b_j = I.Mkp;
    g.C = I.Gq; g.c_i = nq1; g.c_j = 1;
    g.alpha = I.omega; g.w0 = X.w + r0; g.w1 = I.ax[1].w;
    e = launch_gemm64(g, st);
    if (e != hipSuccess) return e;
    if (reduced) {
      const size_t ne = (size_t)((r1 - r0) / X.ng) * (nq1 / I.ax[1].ng);
      k_mxy_mask<<<(int)((ne + 255) / 256), 256, 0, st>>>(I, r0, r1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // nodes whose support meets elements [r0 / ng, r1 / ng)
    int i_lo = r0 / X.ng - X.SW, i_hi = r1 / X.ng + X.SW;
    i_lo = i_lo < 0 ? 0 : i_lo;
    i_hi = i_hi > X.n ? X.n : i_hi;
    const size_t t1 = (size_t)(i_hi - i_lo) * nq1;
    k_mxy_t1_strip<<<(int)((t1 + 255) / 256), 256, 0, st>>>(I, r0, r1, i_lo, i_hi);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t t2 = (size_t)X.n * I.ax[1].n;
  if (I.mixed) k_mxy_t2<float><<<(int)((t2 + 255) / 256), 256, 0, st>>>(I);
  else k_mxy_t2<double><<<(int)((t2 + 255) / 256), 256, 0, st>>>(I);
  return hipGetLastError();
}

// ------------------------------------------------------------ energy
// E = a0 (int u^4 - 2 int u^2 + |Omega|) + kappa/2 int |grad u|^2 on the
// separated tensor Gauss rule (FP64).
// (i) 1D Grams Gm_d = X^T M X, Gk_d = X^T K X give int u^2 and the gradient
//     term;
// (ii) int u^4 = sum over ordered (a,b,c,e) of prod_d G4_d[ab, ce],
//     G4_d = (Xh (.) Xh)^T W (Xh (.) Xh) (Khatri-Rao Gram); evaluated over
//     pair tiles (16 x 16 mode pairs, A <= B) and pair-tile pairs P1 <= P2
//     with multiplicity weights, each 64 x 64 sub-block an FP64 MFMA product.
__global__ void k_energy_grams(DevInst I, int M, double* partial) {
  // block a: sums over b of sigma_a sigma_b [prod_d Gm_d, sum_d Gk_d prod_{e!=d} Gm_e]
  __shared__ double red[16];
  const int a = blockIdx.x;
  double u2 = 0.0, g2 = 0.0;
  for (int b = threadIdx.x; b < M; b += blockDim.x) {
    double gm[kMaxDim], gk[kMaxDim];
    for (int d = 0; d < I.dim; ++d) {
      const DevAxis& A = I.ax[d];
      const double* xa = A.X + (size_t)a * A.n;
      const double* mb = A.MX + (size_t)b * A.n;
      const double* kb = A.KX + (size_t)b * A.n;
      double sm = 0.0, sk = 0.0;
      for (int i = 0; i < A.n; ++i) { sm += xa[i] * mb[i]; sk += xa[i] * kb[i]; }
      gm[d] = sm;
      gk[d] = sk;
    }
    double pm = 1.0;
    for (int d = 0; d < I.dim; ++d) pm *= gm[d];
    const double ss = I.sn[a] * I.sn[b];
    u2 += ss * pm;
    for (int d = 0; d < I.dim; ++d) {
      double t = gk[d];
      for (int e = 0; e < I.dim; ++e)
        if (e != d) t *= gm[e];
      g2 += ss * t;
    }
  }
  u2 = block_sum(u2, red);
  g2 = block_sum(g2, red);
  if (threadIdx.x == 0) { partial[2 * a] = u2; partial[2 * a + 1] = g2; }
}

hipError_t launch_energy_grams(const DevInst& I, int M, double* partial, hipStream_t st) {
  if (M == 0) return hipSuccess;
  k_energy_grams<<<M, 64, 0, st>>>(I, M, partial);
  return hipGetLastError();
}

// Pair tile p (A <= B) of nb tiles: decode to (A, B).
__device__ __forceinline__ void pair_decode(int p, int nb, int& A, int& B) {
  int a = 0, rem = p;
  while (rem >= nb - a) { rem -= nb - a; ++a; }
  A = a;
  B = a + rem;
}

__global__ __launch_bounds__(256) void k_energy_u4(DevInst I, int nb, int npt,
                                                   double* partial) {
  typedef d4 V;
  // block -> (P1 <= P2, sub-block sr, sc)
  const int bid = blockIdx.x;
  const int sub = bid & 15, pp = bid >> 4;
  int P1 = 0, rem = pp;
  while (rem >= npt - P1) { rem -= npt - P1; ++P1; }
  const int P2 = P1 + rem;
  int A1, B1, A2, B2;
  pair_decode(P1, nb, A1, B1);
  pair_decode(P2, nb, A2, B2);
  const int sr = sub >> 2, scb = sub & 3;   // 64-row / 64-col sub-blocks
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  __shared__ double xa[kGChunk][4], xb[kGChunk][kTile], xc[kGChunk][4], xe[kGChunk][kTile];
  __shared__ double wq[kGChunk];
  __shared__ double red[16];
  // wave w: rows 16w..16w+15 of the 64-row sub-block: a_local = sr*4 + w, b = 0..15
  // columns: 4 MFMA tiles (c_local = scb*4 + ct, e = 0..15)
  V prod[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) prod[ct] = V{1, 1, 1, 1};
  const int ldh = I.Mkp;
  for (int d = 0; d < I.dim; ++d) {
    const DevAxis& Ax = I.ax[d];
    const double* Xh = Ax.Xh;
    V acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = V{0, 0, 0, 0};
    for (int q0 = 0; q0 < Ax.nq; q0 += kGChunk) {
      for (int idx = tid; idx < kGChunk * kTile; idx += 256) {
        const int qq = idx / kTile, cc = idx % kTile, q = q0 + qq;
        const bool ok = q < Ax.nq;
        const double* row = Xh + (size_t)(ok ? q : 0) * ldh;
        xb[qq][cc] = ok ? row[B1 * kTile + cc] : 0.0;
        xe[qq][cc] = ok ? row[B2 * kTile + cc] : 0.0;
        if (cc < 4) {
          xa[qq][cc] = ok ? row[A1 * kTile + sr * 4 + cc] : 0.0;
          xc[qq][cc] = ok ? row[A2 * kTile + scb * 4 + cc] : 0.0;
        }
        if (cc == 0) wq[qq] = ok ? Ax.w[q] : 0.0;
      }
      __syncthreads();
      for (int ks = 0; ks < kGChunk / 4; ++ks) {
        const int qq = ks * 4 + (l >> 4);
        const double aval = wq[qq] * xa[qq][w] * xb[qq][l & 15];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const double bval = xc[qq][ct] * xe[qq][l & 15];
          acc[ct] = mfma16(aval, bval, acc[ct]);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int k = 0; k < 4; ++k) prod[ct][k] *= acc[ct][k];
  }
  double s = 0.0;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int k = 0; k < 4; ++k) s += prod[ct][k];
  const double wt = (A1 < B1 ? 2.0 : 1.0) * (A2 < B2 ? 2.0 : 1.0) * (P1 < P2 ? 2.0 : 1.0);
  s = block_sum(s, red) * wt;
  if (tid == 0) partial[bid] = s;
}

hipError_t launch_energy(const DevInst& I, double* partial, int* npartial,
                         hipStream_t st) {
  const int nb = I.nb;
  const int npt = nb * (nb + 1) / 2;
  const int blocks = npt * (npt + 1) / 2 * 16;
  *npartial = blocks;
  if (blocks == 0) return hipSuccess;
  k_energy_u4<<<blocks, 256, 0, st>>>(I, nb, npt, partial);
  return hipGetLastError();
}

// ------------------------------------------------------------ reconstruction
// Dense nodal field u = sum_m sn_m prod_d X_d[:, m] (Kronecker-delta property:
// nodal coefficients are nodal values).
template <class T>
__global__ void k_reconstruct(DevInst I, int M, T* out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t total = 1;
  for (int d = 0; d < I.dim; ++d) total *= (size_t)I.ax[d].n;
  if (idx >= total) return;
  int id[kMaxDim];
  size_t r = idx;
  for (int d = I.dim - 1; d >= 0; --d) {
    id[d] = (int)(r % I.ax[d].n);
    r /= I.ax[d].n;
  }
  double s = 0.0;
  for (int m = 0; m < M; ++m) {
    double p = I.sn[m];
    for (int d = 0; d < I.dim; ++d) p *= I.ax[d].X[(size_t)m * I.ax[d].n + id[d]];
    s += p;
  }
  out[idx] = (T)s;
}

// Tiled reconstruction: a workgroup owns a 64 x 64 tile of the last two
// axes, keeps both factor tiles (M x 64, mode-major) in LDS and walks its
// range of slabs of the first axis (3D; one slab in 2D); per slab each thread
// forms a 4 x 4 block of nodes, sum over modes in FP64, mode order.
template <class T>
__global__ __launch_bounds__(256) void k_reconstruct_tile(DevInst I, int M, T* out) {
  const int D = I.dim;
  const DevAxis& AY = I.ax[D - 2];
  const DevAxis& AZ = I.ax[D - 1];
  const int nj = AY.n, nl = AZ.n;
  const int ni = D == 3 ? I.ax[0].n : 1;
  extern __shared__ double lds[];
  double* ys = lds;            // M x 64
  double* zs = ys + M * 64;    // M x 64
  double* sx = zs + M * 64;    // M
  const int j0 = blockIdx.y * 64, l0 = blockIdx.x * 64;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int idx = tid; idx < M * 64; idx += blockDim.x) {
    const int m = idx >> 6, c = idx & 63;
    ys[idx] = j0 + c < nj ? AY.X[(size_t)m * nj + j0 + c] : 0.0;
    zs[idx] = l0 + c < nl ? AZ.X[(size_t)m * nl + l0 + c] : 0.0;
  }
  const int per = (ni + (int)gridDim.z - 1) / (int)gridDim.z;
  const int i0 = blockIdx.z * per;
  const int i1 = i0 + per < ni ? i0 + per : ni;
  for (int i = i0; i < i1; ++i) {
    __syncthreads();
    for (int m = tid; m < M; m += blockDim.x)
      sx[m] = D == 3 ? I.sn[m] * I.ax[0].X[(size_t)m * ni + i] : I.sn[m];
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    for (int m = 0; m < M; ++m) {
      const double s = sx[m];
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = ys[m * 64 + ty * 4 + r] * s;
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = zs[m * 64 + tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + ty * 4 + r;
      if (j >= nj) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int l = l0 + tx + 16 * c;
        if (l < nl) out[((size_t)i * nj + j) * nl + l] = (T)acc[r][c];
      }
    }
  }
}

size_t reconstruct_tile_lds(int M) { return sizeof(double) * ((size_t)M * 128 + M); }

// MFMA reconstruction (the contraction over modes as a GEMM per slab of the
// first axis): u[i, j, l] = sum_m (Y[j, m] s_m) Z[l, m] with s_m = sn_m X0[i, m]
// (s_m = sn_m in 2D).  A workgroup owns a 64 x 64 (j, l) tile; its four
// waves each compute a 32 x 32 quarter as 2 x 2 MFMA blocks of 16 x 16 with
// K = modes (padded to 4 with zero rows).  Both factor tiles are staged in
// LDS once (mode-major, rows padded so the four modes of a k-step fall in
// distinct banks) in the arithmetic type T: FP32 MFMA with FP32 accumulation
// for FP32 output, FP64 MFMA for FP64 output.
template <class T>
__host__ __device__ constexpr int recon_stride() { return 64 + (sizeof(T) == 4 ? 16 : 8); }

template <class T>
size_t reconstruct_mfma_lds(int M) {
  const size_t Mp = (size_t)(M + 31) / 32 * 32;
  return sizeof(T) * (2 * Mp * recon_stride<T>() + Mp);
}

template <class T>
__global__ __launch_bounds__(256) void k_reconstruct_mfma(DevInst I, int M, T* out) {
  typedef typename Vec4<T>::type V;
  constexpr int RS = recon_stride<T>();
  const int D = I.dim;
  const DevAxis& AY = I.ax[D - 2];
  const DevAxis& AZ = I.ax[D - 1];
  const int nj = AY.n, nl = AZ.n;
  const int ni = D == 3 ? I.ax[0].n : 1;
  const int Mp = (M + 31) / 32 * 32;   // k-steps in blocks of 8 (zero rows past M)
  extern __shared__ unsigned char smr[];
  T* ys = (T*)smr;            // Mp x RS
  T* zs = ys + Mp * RS;       // Mp x RS
  T* sx = zs + Mp * RS;       // Mp
  const int j0 = blockIdx.y * 64, l0 = blockIdx.x * 64;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int idx = tid; idx < Mp * 64; idx += blockDim.x) {
    const int m = idx >> 6, c = idx & 63;
    ys[m * RS + c] = (m < M && j0 + c < nj) ? (T)AY.X[(size_t)m * nj + j0 + c] : (T)0;
    zs[m * RS + c] = (m < M && l0 + c < nl) ? (T)AZ.X[(size_t)m * nl + l0 + c] : (T)0;
  }
  const int wj = (w >> 1) * 32, wl = (w & 1) * 32;   // this wave's quarter
  const int per = (ni + (int)gridDim.z - 1) / (int)gridDim.z;
  const int i0 = blockIdx.z * per;
  const int i1 = i0 + per < ni ? i0 + per : ni;
  // mode weights of slab i, fetched one slab ahead into registers (up to 4
  // modes per thread: M <= 1024 here)
  const double* X0 = I.ax[0].X;
  auto weight = [&](int m, int i) -> T {
    const int mc = m < M ? m : M - 1;
    const double v = I.sn[mc] * (D == 3 ? X0[(size_t)mc * ni + i] : 1.0);
    return m < M ? (T)v : (T)0;
  };
  T wr[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) wr[u] = i0 < i1 ? weight(tid + 256 * u, i0) : (T)0;
  for (int i = i0; i < i1; ++i) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (tid + 256 * u < Mp) sx[tid + 256 * u] = wr[u];
    __syncthreads();
    if (i + 1 < i1) {
#pragma unroll
      for (int u = 0; u < 4; ++u) wr[u] = weight(tid + 256 * u, i + 1);
    }
    V acc[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = V{0, 0, 0, 0};
    // blocks of 8 k-steps, unrolled (a runtime trip count per k-step makes
    // the compiler shuffle the accumulators between iterations)
    for (int kb = 0; kb < Mp / 32; ++kb) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int m = 32 * kb + 4 * kk + (l >> 4);
        const T sm = sx[m];
        const T* yr = ys + m * RS + wj + (l & 15);
        const T* zr = zs + m * RS + wl + (l & 15);
        const T a0 = yr[0] * sm, a1 = yr[16] * sm;
        const T b0 = zr[0], b1 = zr[16];
        acc[0][0] = mfma16(a0, b0, acc[0][0]);
        acc[0][1] = mfma16(a0, b1, acc[0][1]);
        acc[1][0] = mfma16(a1, b0, acc[1][0]);
        acc[1][1] = mfma16(a1, b1, acc[1][1]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int lc = l0 + wl + cb * 16 + (l & 15);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int j = j0 + wj + rb * 16 + mfma_row<T>(l, k);
          if (j < nj && lc < nl) out[((size_t)i * nj + j) * nl + lc] = acc[rb][cb][k];
        }
      }
  }
}

hipError_t launch_reconstruct(const DevInst& I, int M, void* out, int dtype,
                              hipStream_t st) {
  size_t total = 1;
  for (int d = 0; d < I.dim; ++d) total *= (size_t)I.ax[d].n;
  const size_t mlds = dtype == CTD_DTYPE_F32 ? reconstruct_mfma_lds<float>(M) : reconstruct_mfma_lds<double>(M);
  if (M >= 1 && M <= 1024 && mlds <= (size_t)max_lds_bytes()) {
    const int nj = I.ax[I.dim - 2].n, nl = I.ax[I.dim - 1].n;
    const int ni = I.dim == 3 ? I.ax[0].n : 1;
    const int tiles = ((nl + 63) / 64) * ((nj + 63) / 64);
    int zs = std::max(1, std::min(ni, (4 * num_cus() + tiles - 1) / tiles));
    dim3 grid((nl + 63) / 64, (nj + 63) / 64, zs);
    if (dtype == CTD_DTYPE_F32) k_reconstruct_mfma<float><<<grid, 256, mlds, st>>>(I, M, (float*)out);
    else k_reconstruct_mfma<double><<<grid, 256, mlds, st>>>(I, M, (double*)out);
    return hipGetLastError();
  }
  if (M >= 1 && reconstruct_tile_lds(M) <= (size_t)max_lds_bytes()) {
    const int nj = I.ax[I.dim - 2].n, nl = I.ax[I.dim - 1].n;
    const int ni = I.dim == 3 ? I.ax[0].n : 1;
    const int tiles = ((nl + 63) / 64) * ((nj + 63) / 64);
    int zs = std::max(1, std::min(ni, (4 * num_cus() + tiles - 1) / tiles));
    dim3 grid((nl + 63) / 64, (nj + 63) / 64, zs);
    const size_t shm = reconstruct_tile_lds(M);
    if (dtype == CTD_DTYPE_F32) k_reconstruct_tile<float><<<grid, 256, shm, st>>>(I, M, (float*)out);
    else k_reconstruct_tile<double><<<grid, 256, shm, st>>>(I, M, (double*)out);
    return hipGetLastError();
  }
  // very many modes: node-parallel form
  const int blocks = (int)((total + 255) / 256);
  if (dtype == CTD_DTYPE_F32) k_reconstruct<float><<<blocks, 256, 0, st>>>(I, M, (float*)out);
  else k_reconstruct<double><<<blocks, 256, 0, st>>>(I, M, (double*)out);
  return hipGetLastError();
}

// ------------------------------------------------------------ lockstep batch
// Multi-instance launches: one launch serves a group of 2D instances at the
// same phase of their own step (each with its own mode count, sweep number
// and sizes).  blockIdx.z selects the group entry (LsArg); the grid covers
// the largest instance of the group and the blocks an instance does not need
// return at once.  Each instance's arithmetic is that of its own launches.
__global__ void k_reset_scalars_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args) {
  DevScalars* sc = insts[args[blockIdx.z].inst].sc;
  if (threadIdx.x == 0) {
    sc->done = 0;
    sc->converged = 0;
    sc->zero = 0;
    sc->nonfinite = 0;
    sc->change = -1.0;
    sc->sigma_prev = 0.0;
  }
}

__global__ void k_append_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args) {
  const LsArg& a = args[blockIdx.z];
  if (!a.flag) return;
  append_body(insts[a.inst], a.M - 1);
}

__global__ void k_init_mode_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args) {
  const LsArg& a = args[blockIdx.z];
  const DevInst& I = insts[a.inst];
  const int d = blockIdx.y;
  if ((int)blockIdx.x * (int)blockDim.x >= I.ax[d].n) return;
  init_mode_body(I, (uint64_t)a.step, a.mode, a.warm, blockIdx.x, d);
}

template <int B>
__global__ __launch_bounds__(1024) void k_finalize_init_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args) {
  __shared__ double red[96];
  extern __shared__ double ul[];
  const DevInst& I = insts[args[blockIdx.z].inst];
  finalize_body<B>(I, (int)blockIdx.x, 0, 1, red, ul, 0);
}

// d < 0: every direction (the initial guesses), direction blockIdx.y
__global__ void k_signature_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args, int d, int need_flag) {
  const LsArg& a = args[blockIdx.z];
  if (need_flag && !a.flag) return;
  const DevInst& I = insts[a.inst];
  const int ndot = (2 * a.M + I.Mk + 3) / 4;
  if ((int)blockIdx.x >= ndot) return;
  signature_body(I, d, a.M, ndot, 0, blockIdx.x, blockIdx.y);
}

// One workgroup per (row block, column chunk) of every entry, packed: the
// entries' workgroups follow each other (boff), so the grid holds no idle
// workgroups however uneven the instances; a workgroup finds its entry by
// binary search over the offsets.
__global__ __launch_bounds__(256) void k_rhs_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args,
                                               int count, int d) {
  const int b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (args[mid].boff[d] <= b) lo = mid;
    else hi = mid - 1;
  }
  const LsArg& a = args[lo];
  const DevInst& I = insts[a.inst];
  const int rb = (I.ax[d].n + 63) / 64;
  const int local = b - a.boff[d];
  rhs_body(I, d, a.M, 0, a.nlin, local % rb, local / rb);
}

template <int B, int MODE>
__global__ __launch_bounds__(64 * bcr_max_waves(B)) void k_solve_bcr_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args, int d) {
  extern __shared__ double lds[];
  const LsArg& a = args[blockIdx.z];
  const DevInst& I = insts[a.inst];
  double* gws = MODE == 0 ? nullptr : I.bcr_ws;
  BcrMem<B, MODE> mem{MODE == 1 ? gws : lds, MODE == 2 ? gws : nullptr};
  double* sm = MODE == 1 ? gws : lds;
  __shared__ double red[96];
  __shared__ double ab[2];
  const DevAxis& A = I.ax[d];
  if (threadIdx.x == 0) {
    directional_coeffs(I, d, ab[0], ab[1]);
    I.sc->alpha[d] = ab[0];
    I.sc->beta[d] = ab[1];
  }
  __syncthreads();
  bcr_solve_par<B, MODE>(A.n, A.Mb, A.Kb, ab[0], ab[1], A.rpart, a.nlin + a.nld[d] - 1, A.u, mem);
  finalize_body<B>(I, d, a.sweep, 0, red, sm);
}

__global__ void k_gather_scalars_m(const DevInst* __restrict__ insts, const LsArg* __restrict__ args, DevScalars* out) {
  const LsArg& a = args[blockIdx.z];
  const int* src = (const int*)insts[a.inst].sc;
  int* dst = (int*)(out + blockIdx.z);
  for (int k = threadIdx.x; k < (int)(sizeof(DevScalars) / sizeof(int)); k += blockDim.x) dst[k] = src[k];
}

hipError_t launch_multi(int kind, DevInst* insts, const LsArg* args, int count, const LsGrid& g,
                        hipStream_t st, int d, DevScalars* out) {
  if (count <= 0) return hipSuccess;
  switch (kind) {
    case kLsReset: k_reset_scalars_m<<<dim3(1, 1, count), 64, 0, st>>>(insts, args); break;
    case kLsAppend: k_append_m<<<dim3(1, 1, count), 256, 0, st>>>(insts, args); break;
    case kLsInit: k_init_mode_m<<<dim3((g.nmax + 255) / 256, 2, count), 256, 0, st>>>(insts, args); break;
    case kLsFinalizeInit: {
      // g.threads: the workgroup size of the instances' own launch (the
      // reductions' order depends on it), g.nmax: their largest axis
      const size_t shm = sizeof(double) * 3 * (size_t)g.nmax;
      const int nt = g.threads;
      if (nt < 64 || nt > 1024 || nt < (g.nmax >= 1024 ? 1024 : (g.nmax + 63) / 64 * 64))
        return hipErrorInvalidValue;
      switch (g.B) {
        case 3: k_finalize_init_m<3><<<dim3(2, 1, count), nt, shm, st>>>(insts, args); break;
        case 5: k_finalize_init_m<5><<<dim3(2, 1, count), nt, shm, st>>>(insts, args); break;
        case 7: k_finalize_init_m<7><<<dim3(2, 1, count), nt, shm, st>>>(insts, args); break;
        default: return hipErrorInvalidValue;
      }
      break;
    }
    case kLsSignatureAll:
      k_signature_m<<<dim3(g.ndot, 2, count), 256, 0, st>>>(insts, args, -1, 0);
      break;
    case kLsSignature: k_signature_m<<<dim3(g.ndot, 1, count), 256, 0, st>>>(insts, args, d, 0); break;
    case kLsSignatureFlag: k_signature_m<<<dim3(g.ndot, 1, count), 256, 0, st>>>(insts, args, d, 1); break;
    case kLsRhs:
      if (g.nblk <= 0) return hipErrorInvalidValue;
      k_rhs_m<<<g.nblk, 256, 0, st>>>(insts, args, count, d);
      break;
    case kLsSolve: {
#define SOLVE_M(BW)                                                                                   \
  (g.mode == 0 ? k_solve_bcr_m<BW, 0><<<dim3(1, 1, count), g.threads, g.shm, st>>>(insts, args, d)    \
               : g.mode == 2 ? k_solve_bcr_m<BW, 2><<<dim3(1, 1, count), g.threads, g.shm, st>>>(insts, args, d) \
                             : k_solve_bcr_m<BW, 1><<<dim3(1, 1, count), g.threads, 0, st>>>(insts, args, d))
      switch (g.B) {
        case 3: SOLVE_M(3); break;
        case 5: SOLVE_M(5); break;
        case 7: SOLVE_M(7); break;
        default: return hipErrorInvalidValue;
      }
#undef SOLVE_M
      break;
    }
    case kLsGather: k_gather_scalars_m<<<dim3(1, 1, count), 64, 0, st>>>(insts, args, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// BCR launch class of an axis: storage mode (0 LDS, 2 split, 1 workspace),
// threads and dynamic LDS bytes
void bcr_launch_class(int n, int B, int& mode, int& threads, size_t& shm) {
  const bool fits = bcr_fits(n, B);
  const bool split = !fits && bcr_split_fits(n, B);
  mode = fits ? 0 : (split ? 2 : 1);
  threads = bcr_threads(n, B);
  shm = fits ? bcr_lds_bytes(n, B) : (split ? bcr_split_lds_bytes(n, B) : 0);
}

// Strided placement of a C-ordered nodal grid (caller layouts of
// ctd_reconstruct): one element per lane, reads coalesced.
template <class T>
__global__ void k_scatter_strided(const T* __restrict__ src, T* __restrict__ dst, int64_t total,
                                  int64_t n1, int64_t n2, int64_t s0, int64_t s1, int64_t s2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  const int64_t i2 = k % n2, r = k / n2, i1 = r % n1, i0 = r / n1;
  dst[i0 * s0 + i1 * s1 + i2 * s2] = src[k];
}

hipError_t launch_scatter_strided(const void* src, void* dst, int esz, int dim, const int64_t* n,
                                  const int64_t* strides, hipStream_t st) {
  // view as three axes (leading unit axes for 2D)
  int64_t nn[3] = {1, 1, 1}, ss[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) { nn[3 - dim + d] = n[d]; ss[3 - dim + d] = strides[d]; }
  const int64_t total = nn[0] * nn[1] * nn[2];
  if (total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (esz == 4)
    k_scatter_strided<float><<<blocks, 256, 0, st>>>((const float*)src, (float*)dst, total, nn[1], nn[2],
                                                     ss[0], ss[1], ss[2]);
  else
    k_scatter_strided<double><<<blocks, 256, 0, st>>>((const double*)src, (double*)dst, total, nn[1],
                                                      nn[2], ss[0], ss[1], ss[2]);
  return hipGetLastError();
}

}  // namespace ctd

namespace ctd {
static int g_max_lds = 65536;
static int g_num_cus = 256;
// Kernels whose dynamic LDS can exceed 64 KiB (the banded solve stages the
// whole band; the FP64 cubic h kernel stages a 64 x Mkp tile plus an S tile).
hipError_t configure_kernels() {
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lock(mu);
  if (done) return hipSuccess;
  int dev = 0, lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  g_max_lds = lds;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    g_num_cus = ncu;
  // Raising the limit is best effort: launches check their own LDS needs.
  const void* ks[] = {(const void*)k_solve_bcr<3, 0>, (const void*)k_solve_bcr<5, 0>,
                      (const void*)k_solve_bcr<7, 0>, (const void*)k_band_solve_bcr<3, 0>,
                      (const void*)k_band_solve_bcr<5, 0>, (const void*)k_band_solve_bcr<7, 0>,
                      (const void*)k_solve_bcr<3, 2>, (const void*)k_solve_bcr<5, 2>,
                      (const void*)k_solve_bcr<7, 2>, (const void*)k_band_solve_bcr<3, 2>,
                      (const void*)k_band_solve_bcr<5, 2>, (const void*)k_band_solve_bcr<7, 2>,
                      (const void*)k_cubic_h<double>,
                      (const void*)k_cubic_h32, (const void*)k_reconstruct_tile<float>,
                      (const void*)k_reconstruct_tile<double>, (const void*)k_reconstruct_mfma<float>,
                      (const void*)k_reconstruct_mfma<double>,
                      (const void*)k_solve_bcr_m<3, 0>, (const void*)k_solve_bcr_m<5, 0>,
                      (const void*)k_solve_bcr_m<7, 0>, (const void*)k_solve_bcr_m<3, 2>,
                      (const void*)k_solve_bcr_m<5, 2>, (const void*)k_solve_bcr_m<7, 2>,
                      (const void*)k_finalize_init_m<3>, (const void*)k_finalize_init_m<5>,
                      (const void*)k_finalize_init_m<7>, (const void*)k_finalize<3>,
                      (const void*)k_finalize<5>, (const void*)k_finalize<7>,
                      (const void*)k_finalize_sig<3>, (const void*)k_finalize_sig<5>,
                      (const void*)k_finalize_sig<7>};
  for (const void* k : ks)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipGetLastError();
  done = true;
  return hipSuccess;
}

int max_lds_bytes() { return g_max_lds; }
int num_cus() { return g_num_cus; }
}  // namespace ctd
