// HIP kernels of the CTD step for gfx950.
//
// Notation (Sec. 3.3 / App. D): for the directional solve in direction d the
// other directions' factors u_e are fixed; c = 1/dt + alpha L, lam = L kappa,
// omega = 4 a0 L.  Quadrature tables: Phi_d (nq x n, SW = 2s+2 nonzeros per
// row starting at column st(e)), weights W_d.  u^k = sum_j sk_j prod_d X^k_d[:,j]
// and its Gauss-point tables Xh_d = Phi_d X^k_d diag(sk^(1/D)).
#include "ctd_internal.h"

#include <cmath>

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
                            double pw, int mixed) {
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
  if (mixed) A.Xhf[idx] = (float)val;
}

hipError_t launch_quad_eval(const DevInst& I, int d, hipStream_t st) {
  const DevAxis& A = I.ax[d];
  size_t total = (size_t)A.nq * I.Mkp;
  int blocks = (int)((total + 255) / 256);
  if (blocks == 0) return hipSuccess;
  k_quad_eval<<<blocks, 256, 0, st>>>(A, I.Mk, I.Mkp, I.sk, 1.0 / I.dim, I.mixed);
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

__global__ void k_init_mode(DevInst I, uint64_t step, int mode, int warm) {
  const int d = blockIdx.y;
  const DevAxis& A = I.ax[d];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
__device__ void finalize_body(DevInst& I, int d, int sweep, int from_init, double* red) {
  DevAxis& A = I.ax[d];
  DevScalars* sc = I.sc;
  const int n = A.n;
  double s2 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double mu = band_row(A.Mb, n, A.B, A.u, i);
    double ku = band_row(A.Kb, n, A.B, A.u, i);
    A.Mu[i] = mu;
    A.Ku[i] = ku;
    s2 += A.u[i] * mu;
  }
  s2 = block_sum(s2, red);
  const double sigma = sqrt(s2);
  const bool bad = !(sigma == sigma) || isinf(sigma);
  const bool zero = sigma == 0.0;
  const double inv = (bad || zero) ? 0.0 : 1.0 / sigma;
  double m = 0, k = 0, uu = 0, uup = 0, upup = 0, um = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double u = A.u[i] * inv;
    double mu = A.Mu[i] * inv, ku = A.Ku[i] * inv;
    double up = A.up[i];
    m += u * mu;
    k += u * ku;
    uu += u * u;
    uup += u * up;
    upup += up * up;
    um = fmax(um, fabs(u));
  }
  m = block_sum(m, red);
  k = block_sum(k, red);
  uu = block_sum(uu, red);
  uup = block_sum(uup, red);
  upup = block_sum(upup, red);
  um = block_max(um, red);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double u = A.u[i] * inv;
    A.u[i] = u;
    A.up[i] = u;
    A.Mu[i] *= inv;
    A.Ku[i] *= inv;
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
        if (sweep >= 2) {
          double puu = 1.0, pupup = 1.0, puup = 1.0;
          for (int e = 0; e < I.dim; ++e) {
            puu *= sc->uu[e];
            pupup *= sc->upup[e];
            puup *= sc->uup[e];
          }
          const double nn = sigma * sigma * puu;
          const double oo = sc->sigma_prev * sc->sigma_prev * pupup;
          const double no = sigma * sc->sigma_prev * puup;
          double r2 = nn + oo - 2.0 * no;
          r2 = r2 > 0.0 ? r2 : 0.0;
          double r = nn > 0.0 ? sqrt(r2 / nn) : 0.0;
          sc->change = r;
          sc->converged = r <= I.fp_tol ? 1 : 0;
        }
        sc->sigma_prev = sigma;
      }
    }
  }
}

__global__ void k_finalize(DevInst I, int d, int sweep, int from_init) {
  __shared__ double red[16];
  finalize_body(I, d, sweep, from_init, red);
}

hipError_t launch_finalize(const DevInst& I, int d, int sweep, int from_init,
                           hipStream_t st) {
  k_finalize<<<1, 256, 0, st>>>(I, d, sweep, from_init);
  return hipGetLastError();
}

// ------------------------------------------------------------ signature
// Grams of the freshly solved factor u_d against the stored columns
// (gm = X^T M u, gk = X^T K u over the M modes of u^{k+1}, gmk = X^kT M u)
// and v = W * (Phi u) at the Gauss points (3D cubic route).
__global__ void k_signature(DevInst I, int d, int M, int ndot_blocks, int want_v) {
  DevAxis& A = I.ax[d];
  const int n = A.n;
  if ((int)blockIdx.x < ndot_blocks) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + w;
    const int total = 2 * M + I.Mk;
    if (idx >= total) return;
    const double* col;
    double* out;
    if (idx < M) { col = A.MX + (size_t)idx * n; out = A.gm + idx; }
    else if (idx < 2 * M) { col = A.KX + (size_t)(idx - M) * n; out = A.gk + (idx - M); }
    else { col = A.MXk + (size_t)(idx - 2 * M) * n; out = A.gmk + (idx - 2 * M); }
    double s = 0.0;
    for (int i = l; i < n; i += 64) s += col[i] * A.u[i];
    s = wave_sum(s);
    if (l == 0) *out = s;
    return;
  }
  if (!want_v) return;
  const int q = (blockIdx.x - ndot_blocks) * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  const int st = elem_start(q / A.ng, A.s, n, A.SW);
  const double* ph = A.phi + (size_t)q * A.SW;
  double val = 0.0;
  for (int j = 0; j < A.SW; ++j) val += ph[j] * A.u[st + j];
  val *= A.w[q];
  A.v[q] = val;
  if (I.mixed) A.vf[q] = (float)val;
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

// ------------------------------------------------------------ rhs
// Right-hand side of the directional system (eq. KxQx and its 3D analogue):
//   Q_d = ck MXk (sk * a^k) - MX (sn (c a + lam b)) - lam KX (sn a) - F_d,
// ck = c with the 2D M_xy load (which contains the full w), ck = c + omega
// with the 3D cubic load F_d = omega Phi^T W h.  Also alpha_d, beta_d of
// K_d = alpha_d M_d + beta_d K_d.
__global__ void k_rhs(DevInst I, int d, int M, int load_only) {
  extern __shared__ double sm[];
  double* ak = sm;                  // Mk
  double* cX = ak + I.Mk;           // M
  double* cK = cX + M;              // M
  double* part = cK + M;            // 4 x 64
  DevAxis& A = I.ax[d];
  const int n = A.n;
  const int tid = threadIdx.x;
  for (int j = tid; j < I.Mk; j += blockDim.x) {
    double v = I.sk[j];
    for (int e = 0; e < I.dim; ++e)
      if (e != d) v *= I.ax[e].gmk[j];
    ak[j] = v;
  }
  for (int m = tid; m < M; m += blockDim.x) {
    double am = 1.0, bm = 0.0;
    for (int e = 0; e < I.dim; ++e) {
      if (e == d) continue;
      am *= I.ax[e].gm[m];
      double t = I.ax[e].gk[m];
      for (int f = 0; f < I.dim; ++f)
        if (f != d && f != e) t *= I.ax[f].gm[m];
      bm += t;
    }
    cX[m] = I.sn[m] * (I.c * am + I.lam * bm);
    cK[m] = I.lam * I.sn[m] * am;
  }
  if (blockIdx.x == 0 && tid == 0) {
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
    I.sc->alpha[d] = I.c * pm + I.lam * grad;
    I.sc->beta[d] = I.lam * pm;
  }
  __syncthreads();
  const int w = tid >> 6, l = tid & 63;
  const int i = blockIdx.x * 64 + l;
  const double ck = load_only ? (I.dim == 3 ? -I.omega : 0.0)
                              : (I.dim == 3 ? I.c + I.omega : I.c);
  double acc = 0.0;
  if (i < n && !load_only) {
    for (int j = w; j < I.Mk; j += 4) acc += ck * A.MXk[(size_t)j * n + i] * ak[j];
    for (int m = w; m < M; m += 4)
      acc -= A.MX[(size_t)m * n + i] * cX[m] + A.KX[(size_t)m * n + i] * cK[m];
  } else if (i < n && I.dim == 3) {
    // load only, 3D: linear part -omega M X^k (sk * a^k) of the full load
    for (int j = w; j < I.Mk; j += 4) acc += ck * A.MXk[(size_t)j * n + i] * ak[j];
  }
  part[w * 64 + l] = acc;
  __syncthreads();
  if (w == 0 && i < n) {
    double q = part[l] + part[64 + l] + part[128 + l] + part[192 + l];
    double F;
    if (I.dim == 3) {
      F = 0.0;
      const int ne = n - 1;
      int e0 = i - A.SW;
      e0 = e0 < 0 ? 0 : e0;
      int e1 = i + A.SW;
      e1 = e1 > ne - 1 ? ne - 1 : e1;
      for (int e = e0; e <= e1; ++e) {
        const int st = elem_start(e, A.s, n, A.SW);
        const int jj = i - st;
        if (jj < 0 || jj >= A.SW) continue;
        for (int g = 0; g < A.ng; ++g) {
          const int qq = e * A.ng + g;
          double h = 0.0;
          for (int sp = 0; sp < I.nsplit_h; ++sp) h += I.hpart[(size_t)sp * A.nq + qq];
          F += A.phi[(size_t)qq * A.SW + jj] * A.w[qq] * h;
        }
      }
      F *= I.omega;
    } else {
      F = A.F[i];
    }
    A.rhs[i] = load_only ? q + F : q - F;
  }
}

hipError_t launch_rhs(const DevInst& I, int d, int M, hipStream_t st, int load_only) {
  const int n = I.ax[d].n;
  size_t shm = sizeof(double) * (I.Mk + 2 * M + 256);
  k_rhs<<<(n + 63) / 64, 256, shm, st>>>(I, d, M, load_only);
  return hipGetLastError();
}

// ------------------------------------------------------------ band solve
// SPD banded solve (alpha M + beta K) x = b by LDL^T, half-bandwidth B.
// The band and the right-hand side are staged in LDS; one thread runs the
// factorisation with forward substitution fused, keeping the active
// (B+1) x (B+1) window in registers, then the back substitution.
template <int B>
__device__ void ldlt_lds(int n, double* band, double* x) {
  // band: (B+1) x n in LDS, [t*n + j] = A[j+t][j]; overwritten by L (t>=1)
  // and D (t=0).  x: LDS rhs in, solution out.
  double w[B + 1][B + 1];
  double bw[B + 1];
#pragma unroll
  for (int r = 0; r <= B; ++r) {
#pragma unroll
    for (int c = 0; c <= r; ++c)
      w[r][c] = (r < n) ? band[(r - c) * n + c] : (r == c ? 1.0 : 0.0);
    bw[r] = r < n ? x[r] : 0.0;
  }
  for (int j = 0; j < n; ++j) {
    // prefetch the row entering the window
    const int inew = j + 1 + B;
    double nr[B + 1];
    double nb;
    if (inew < n) {
#pragma unroll
      for (int c = 0; c <= B; ++c) nr[c] = band[(B - c) * n + (j + 1 + c)];
      nb = x[inew];
    } else {
#pragma unroll
      for (int c = 0; c <= B; ++c) nr[c] = (c == B) ? 1.0 : 0.0;
      nb = 0.0;
    }
    const double dj = w[0][0];
    const double rd = 1.0 / dj;
    double l[B + 1];
#pragma unroll
    for (int t = 1; t <= B; ++t) l[t] = w[t][0] * rd;
    const double yj = bw[0];
    band[j] = dj;
#pragma unroll
    for (int t = 1; t <= B; ++t) band[t * n + j] = l[t];
    x[j] = yj * rd;
#pragma unroll
    for (int r = 0; r < B; ++r) {
#pragma unroll
      for (int c = 0; c <= r; ++c) w[r][c] = w[r + 1][c + 1] - w[r + 1][0] * l[c + 1];
      bw[r] = bw[r + 1] - l[r + 1] * yj;
    }
#pragma unroll
    for (int c = 0; c <= B; ++c) w[B][c] = nr[c];
    bw[B] = nb;
  }
  double xw[B];
#pragma unroll
  for (int t = 0; t < B; ++t) xw[t] = 0.0;
  for (int j = n - 1; j >= 0; --j) {
    double s = x[j];
#pragma unroll
    for (int t = 1; t <= B; ++t) s -= band[t * n + j] * xw[t - 1];
    x[j] = s;
#pragma unroll
    for (int t = B - 1; t > 0; --t) xw[t] = xw[t - 1];
    xw[0] = s;
  }
}

__device__ void run_ldlt(int B, int n, double* band, double* x) {
  switch (B) {
    case 3: ldlt_lds<3>(n, band, x); break;
    case 5: ldlt_lds<5>(n, band, x); break;
    case 7: ldlt_lds<7>(n, band, x); break;
    default: break;
  }
}

int max_lds_bytes();
int solve_lds_max_n(int B) {
  const size_t budget = (size_t)max_lds_bytes() - 1024;
  return (int)(budget / (sizeof(double) * (B + 2)));
}

__global__ __launch_bounds__(256) void k_solve(DevInst I, int d, int sweep) {
  extern __shared__ double sm[];
  __shared__ double red[16];
  DevAxis& A = I.ax[d];
  const int n = A.n, B = A.B;
  double* band = sm;
  double* x = sm + (size_t)(B + 1) * n;
  const double al = I.sc->alpha[d], be = I.sc->beta[d];
  for (int idx = threadIdx.x; idx < (B + 1) * n; idx += blockDim.x)
    band[idx] = al * A.Mb[idx] + be * A.Kb[idx];
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = A.rhs[i];
  __syncthreads();
  if (threadIdx.x == 0) run_ldlt(B, n, band, x);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) A.u[i] = x[i];
  __syncthreads();
  finalize_body(I, d, sweep, 0, red);
}

hipError_t launch_solve(const DevInst& I, int d, int sweep, hipStream_t st) {
  const DevAxis& A = I.ax[d];
  size_t shm = sizeof(double) * ((size_t)(A.B + 2) * A.n);
  k_solve<<<1, 256, shm, st>>>(I, d, sweep);
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_band_solve_batch(int n, int B, const double* Mb, const double* Kb,
                                   const double* alpha, const double* beta,
                                   const double* b, double* x) {
  extern __shared__ double sm[];
  const int k = blockIdx.x;
  double* band = sm;
  double* xs = sm + (size_t)(B + 1) * n;
  const double al = alpha[k], be = beta[k];
  for (int idx = threadIdx.x; idx < (B + 1) * n; idx += blockDim.x)
    band[idx] = al * Mb[idx] + be * Kb[idx];
  for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = b[(size_t)k * n + i];
  __syncthreads();
  if (threadIdx.x == 0) run_ldlt(B, n, band, xs);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[(size_t)k * n + i] = xs[i];
}

hipError_t launch_band_solve_batch(int n, int bw, const double* Mb,
                                   const double* Kb, const double* alpha,
                                   const double* beta, const double* b,
                                   double* x, int count, hipStream_t st) {
  size_t shm = sizeof(double) * ((size_t)(bw + 2) * n);
  k_band_solve_batch<<<count, 64, shm, st>>>(n, bw, Mb, Kb, alpha, beta, b, x);
  return hipGetLastError();
}

// ------------------------------------------------------------ append
// Append the converged rank-one term as mode M and take the enrichment
// decision: stop when its nodal max sigma * prod max|u_d| <= enrich_tol, or
// at the mode cap.
__global__ void k_append(DevInst I, int M) {
  const double sigma = I.sc->sigma[I.dim - 1];
  for (int d = 0; d < I.dim; ++d) {
    DevAxis& A = I.ax[d];
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

hipError_t launch_append(const DevInst& I, int M, hipStream_t st) {
  k_append<<<1, 256, 0, st>>>(I, M);
  return hipGetLastError();
}

__global__ void k_reset_scalars(DevScalars* sc) {
  if (threadIdx.x == 0) {
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

template <class T>
__global__ __launch_bounds__(256) void k_cubic_g(DevInst I, int d) {
  typedef typename Vec4<T>::type V;
  const DevAxis& A = I.ax[d];
  const T* Y = (const T*)(sizeof(T) == 4 ? (const void*)A.Xhf : (const void*)A.Xh);
  const T* vq = (const T*)(sizeof(T) == 4 ? (const void*)A.vf : (const void*)A.v);
  const int ldh = I.Mkp;
  const int t = blockIdx.x, split = blockIdx.y;
  const int4 tr = I.tri[t];
  const int A0 = tr.x * kTile, B0 = tr.y * kTile, C0 = tr.z * kTile;
  const int nq = A.nq;
  const int per = ((nq + I.nsplit_g - 1) / I.nsplit_g + kGChunk - 1) / kGChunk * kGChunk;
  const int qbeg = split * per;
  const int qend = qbeg + per < nq ? qbeg + per : nq;
  __shared__ T ya[kGChunk][kTile];
  __shared__ T yb[kGChunk][kTile];
  __shared__ T yc[kGChunk][kTile];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  V acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = V{0, 0, 0, 0};
  for (int q0 = qbeg; q0 < qend; q0 += kGChunk) {
    for (int idx = tid; idx < kGChunk * kTile; idx += 256) {
      const int qq = idx / kTile, cc = idx % kTile, q = q0 + qq;
      T va = 0, vb = 0, vc = 0;
      if (q < qend) {
        const T* row = Y + (size_t)q * ldh;
        va = row[A0 + cc];
        vb = row[B0 + cc];
        vc = row[C0 + cc] * vq[q];
      }
      ya[qq][cc] = va;
      yb[qq][cc] = vb;
      yc[qq][cc] = vc;
    }
    __syncthreads();
#pragma unroll 4
    for (int ks = 0; ks < kGChunk / 4; ++ks) {
      const int qq = ks * 4 + (l >> 4);
      const T bval = yc[qq][l & 15];
      const T ybv = yb[qq][l & 15];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T aval = ya[qq][w * 4 + r] * ybv;
        acc[r] = mfma16(aval, bval, acc[r]);
      }
    }
    __syncthreads();
  }
  T* out = (T*)I.gpart + ((size_t)split * I.ntri + t) * (kTileSq * kTile);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int al = w * 4 + r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = mfma_row<T>(l, k), j = l & 15;
      out[(al * kTile + i) * kTile + j] = acc[r][k];
    }
  }
}

template <class T>
__global__ void k_cubic_gred(DevInst I, int d, int e_other) {
  const size_t per = (size_t)kTileSq * kTile;
  const size_t total = (size_t)I.ntri * per;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const T* gp = (const T*)I.gpart;
  double s = 0.0;
  for (int sp = 0; sp < I.nsplit_g; ++sp) s += (double)gp[(size_t)sp * total + idx];
  T* g = (T*)I.ax[d].g;
  g[idx] = (T)s;
  if (e_other >= 0) {
    const int t = (int)(idx / per);
    const T* go = (const T*)I.ax[e_other].g;
    ((T*)I.S)[idx] = (T)((double)I.tri[t].w * s * (double)go[idx]);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_cubic_h(DevInst I, int d) {
  typedef typename Vec4<T>::type V;
  extern __shared__ unsigned char smraw[];
  const DevAxis& A = I.ax[d];
  const T* X = (const T*)(sizeof(T) == 4 ? (const void*)A.Xhf : (const void*)A.Xh);
  const int ldh = I.Mkp;
  const int nq = A.nq;
  T* xs = (T*)smraw;                       // 64 x ldh
  T* ss = xs + 64 * ldh;                   // 256 x 16
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int q0 = blockIdx.x * 64;
  const int split = blockIdx.y;
  const int per = (I.ntri + I.nsplit_h - 1) / I.nsplit_h;
  const int t0 = split * per;
  const int t1 = t0 + per < I.ntri ? t0 + per : I.ntri;
  for (int idx = tid; idx < 64 * ldh; idx += 256) {
    const int qq = idx / ldh, c = idx % ldh, q = q0 + qq;
    xs[idx] = q < nq ? X[(size_t)q * ldh + c] : (T)0;
  }
  const int rowA = w * 16 + (l & 15);     // A-operand row (q) of this lane
  double hq[4] = {0, 0, 0, 0};
  V acc = V{0, 0, 0, 0};
  int curC = -1;
  for (int t = t0; t < t1; ++t) {
    const int4 tr = I.tri[t];
    if (tr.z != curC) {
      if (curC >= 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = w * 16 + mfma_row<T>(l, r);
          double v = (double)acc[r] * (double)xs[row * ldh + curC * kTile + (l & 15)];
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
    __syncthreads();
    const T* St = (const T*)I.S + (size_t)t * (kTileSq * kTile);
    for (int idx = tid; idx < kTileSq * kTile; idx += 256) ss[idx] = St[idx];
    __syncthreads();
    const int A0 = tr.x * kTile, B0 = tr.y * kTile;
    T xa[kTile], xb[4];
#pragma unroll
    for (int a = 0; a < kTile; ++a) xa[a] = xs[rowA * ldh + A0 + a];
#pragma unroll
    for (int m = 0; m < 4; ++m) xb[m] = xs[rowA * ldh + B0 + 4 * m + (l >> 4)];
#pragma unroll
    for (int ks = 0; ks < kTileSq / 4; ++ks) {
      const T aval = xa[ks >> 2] * xb[ks & 3];
      const T bval = ss[(4 * ks + (l >> 4)) * kTile + (l & 15)];
      acc = mfma16(aval, bval, acc);
    }
  }
  if (curC >= 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + mfma_row<T>(l, r);
      double v = (double)acc[r] * (double)xs[row * ldh + curC * kTile + (l & 15)];
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
  dim3 grid(I.ntri, I.nsplit_g);
  if (I.mixed) k_cubic_g<float><<<grid, 256, 0, st>>>(I, d);
  else k_cubic_g<double><<<grid, 256, 0, st>>>(I, d);
  return hipGetLastError();
}

hipError_t launch_cubic_gred(const DevInst& I, int d, int e_other, hipStream_t st) {
  size_t total = (size_t)I.ntri * kTileSq * kTile;
  int blocks = (int)((total + 255) / 256);
  if (I.mixed) k_cubic_gred<float><<<blocks, 256, 0, st>>>(I, d, e_other);
  else k_cubic_gred<double><<<blocks, 256, 0, st>>>(I, d, e_other);
  return hipGetLastError();
}

hipError_t launch_cubic_h(const DevInst& I, int d, hipStream_t st) {
  const int nq = I.ax[d].nq;
  dim3 grid((nq + 63) / 64, I.nsplit_h);
  if (I.mixed) {
    size_t shm = sizeof(float) * (64 * I.Mkp + kTileSq * kTile);
    k_cubic_h<float><<<grid, 256, shm, st>>>(I, d);
  } else {
    size_t shm = sizeof(double) * (64 * I.Mkp + kTileSq * kTile);
    k_cubic_h<double><<<grid, 256, shm, st>>>(I, d);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ M_xy (2D)
// Full integration of M_xy = int N~_x^T N~_y L w(u^k) (eq. KxxMxx) on the
// tensor Gauss grid: U = Xh_0 Xh_1^T, G = omega (U^3 - U) W_0 W_1,
// T1 = Phi_0^T G (gathered per node), M_xy = T1 Phi_1.
template <class T>
__global__ void k_mxy_t1(DevInst I) {
  const DevAxis& X = I.ax[0];
  const DevAxis& Yx = I.ax[1];
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nqy = Yx.nq;
  if (idx >= (size_t)X.n * nqy) return;
  const int i = (int)(idx / nqy), qy = (int)(idx % nqy);
  const int ldh = I.Mkp;
  const T* Xh = (const T*)(sizeof(T) == 4 ? (const void*)X.Xhf : (const void*)X.Xh);
  const T* Yh = (const T*)(sizeof(T) == 4 ? (const void*)Yx.Xhf : (const void*)Yx.Xh);
  const T* yrow = Yh + (size_t)qy * ldh;
  const int n = X.n, ne = n - 1;
  int e0 = i - X.SW;
  e0 = e0 < 0 ? 0 : e0;
  int e1 = i + X.SW;
  e1 = e1 > ne - 1 ? ne - 1 : e1;
  double acc = 0.0;
  for (int e = e0; e <= e1; ++e) {
    const int st = elem_start(e, X.s, n, X.SW);
    const int jj = i - st;
    if (jj < 0 || jj >= X.SW) continue;
    for (int g = 0; g < X.ng; ++g) {
      const int qx = e * X.ng + g;
      const T* xrow = Xh + (size_t)qx * ldh;
      T u = 0;
      for (int a = 0; a < I.Mk; ++a) u += xrow[a] * yrow[a];
      const double ud = (double)u;
      acc += X.phi[(size_t)qx * X.SW + jj] * X.w[qx] * (ud * ud * ud - ud);
    }
  }
  I.T1[idx] = acc * I.omega * Yx.w[qy];
}

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
  const size_t t1 = (size_t)I.ax[0].n * I.ax[1].nq;
  const size_t t2 = (size_t)I.ax[0].n * I.ax[1].n;
  if (I.mixed) {
    k_mxy_t1<float><<<(int)((t1 + 255) / 256), 256, 0, st>>>(I);
    k_mxy_t2<float><<<(int)((t2 + 255) / 256), 256, 0, st>>>(I);
  } else {
    k_mxy_t1<double><<<(int)((t1 + 255) / 256), 256, 0, st>>>(I);
    k_mxy_t2<double><<<(int)((t2 + 255) / 256), 256, 0, st>>>(I);
  }
  return hipGetLastError();
}

// F_0 = M_xy u_1 (d = 0) or F_1 = M_xy^T u_0 (d = 1): one wave per row.
template <class T>
__global__ void k_gemv(DevInst I, int d) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  const int nrows = I.ax[d].n, ncols = I.ax[1 - d].n;
  if (row >= nrows) return;
  const T* Mat = (const T*)(d == 0 ? I.Mxy : I.MxyT) + (size_t)row * ncols;
  const double* x = I.ax[1 - d].u;
  double s = 0.0;
  for (int j = l; j < ncols; j += 64) s += (double)Mat[j] * x[j];
  s = wave_sum(s);
  if (l == 0) I.ax[d].F[row] = s;
}

hipError_t launch_gemv(const DevInst& I, int d, hipStream_t st) {
  const int blocks = (I.ax[d].n + 3) / 4;
  if (I.mixed) k_gemv<float><<<blocks, 256, 0, st>>>(I, d);
  else k_gemv<double><<<blocks, 256, 0, st>>>(I, d);
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

hipError_t launch_reconstruct(const DevInst& I, int M, void* out, int dtype,
                              hipStream_t st) {
  size_t total = 1;
  for (int d = 0; d < I.dim; ++d) total *= (size_t)I.ax[d].n;
  const int blocks = (int)((total + 255) / 256);
  if (dtype == CTD_DTYPE_F32) k_reconstruct<float><<<blocks, 256, 0, st>>>(I, M, (float*)out);
  else k_reconstruct<double><<<blocks, 256, 0, st>>>(I, M, (double*)out);
  return hipGetLastError();
}

}  // namespace ctd

namespace ctd {
static int g_max_lds = 65536;
// Kernels whose dynamic LDS can exceed 64 KiB (the banded solve stages the
// whole band; the FP64 cubic h kernel stages a 64 x Mkp tile plus an S tile).
hipError_t configure_kernels() {
  static bool done = false;
  if (done) return hipSuccess;
  int dev = 0, lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  g_max_lds = lds;
  // Raising the limit is best effort: launches check their own LDS needs.
  const void* ks[] = {(const void*)k_solve, (const void*)k_band_solve_batch,
                      (const void*)k_cubic_h<double>, (const void*)k_cubic_h<float>};
  for (const void* k : ks)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipGetLastError();
  done = true;
  return hipSuccess;
}

int max_lds_bytes() { return g_max_lds; }
}  // namespace ctd
