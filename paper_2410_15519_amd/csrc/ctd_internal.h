// Internal declarations shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ctd.h"

namespace ctd {

constexpr int kMaxDim = 3;
constexpr int kTile = 16;          // mode tile of the cubic contractions
constexpr int kTileSq = kTile * kTile;

// Host FP64 tables of one axis (built by build_axis).
struct AxisTables {
  int n = 0, ne = 0, ng = 0, nq = 0, s = 0, p = 0, SW = 0, B = 0;
  double a = 0, lo = 0, hi = 0, h = 0;
  std::vector<double> phi, dphi;  // nq x SW
  std::vector<double> w;          // nq
  std::vector<double> Mb, Kb;     // (B+1) x n lower band
};

int build_axis(int64_t n, double lo, double hi, int s, int p, double a, int ng,
               AxisTables& ax, std::string& err);
void gauss_legendre(int ng, std::vector<double>& x, std::vector<double>& w);

// Generalised eigenvectors of (K, M) of an axis: V^T M V = I, V^T K V =
// diag(mu); V row-major n x n (V[i*n + k] = entry i of eigenvector k).
struct FastDiag {
  std::vector<double> V, mu;
};
bool fast_diag(const AxisTables& T, std::vector<double>& V, std::vector<double>& mu, std::string& err);
std::shared_ptr<const FastDiag> fast_diag_cached(const AxisTables& T, std::string& err);

// Device buffers of one axis of one instance.
struct DevAxis {
  int n, nq, ng, SW, B, s;
  double* phi;      // nq x SW
  float* phif;
  double* w;        // nq
  double* Mb;       // (B+1) x n
  double* Kb;
  double* Xk;       // n x Mcap, factors of u^k
  double* MXk;      // n x Mcap, M X^k
  double* Xh;       // nq x ldh, Phi X^k sigma^(1/D) (row-major)
  float* Xhf;       // FP32 copy, tile-major: [a / 16][q][slot] (3D h contraction)
  float* Xhg;       // FP32 copy for the 3D g contraction: [a / 16][q / 4][a % 16][q % 4]
  double* X;        // n x Mcap, factors of u^{k+1}
  double* MX;
  double* KX;
  double* u;        // n, current mode factor (unit M-norm after finalize)
  double* up;       // n, same factor one sweep earlier
  double* Mu;       // n
  double* Ku;       // n
  double* rhs;      // n
  double* rpart;    // (chunks + 1) x n partial right-hand sides
  double* v;        // nq, W * (Phi u)
  float* vf;
  double* gm;       // Mcap: u . MX[:, m]
  double* gk;       // Mcap: u . KX[:, m]
  double* gmk;      // Mcap: u . MXk[:, j]
  void* g;          // cubic Gram of u (3D): ntri x 256 x 16 (T)
  // fast-diagonalisation solve (null when the axis uses cyclic reduction)
  const double* fdV;   // n x n row-major generalised eigenvectors
  const double* fdmu;  // n eigenvalues
  double* fdz;         // kFdSplit x n partial projections V^T b
  double* fdu;         // kFdKb x n partial back-projections (split over eigenvectors)
};

// Scalars shared by kernels of one instance (device memory).
struct DevScalars {
  double sigma[kMaxDim];   // amplitude after solving direction d
  double m[kMaxDim];       // u.M.u (=1 after normalisation, up to rounding)
  double k[kMaxDim];       // u.K.u
  double uu[kMaxDim], uup[kMaxDim], upup[kMaxDim];
  double umax[kMaxDim];
  double alpha[kMaxDim], beta[kMaxDim];
  double sigma_prev;
  double change;
  double term_max;
  int32_t converged;
  int32_t zero;
  int32_t nonfinite;
  int32_t nmodes;
  int32_t stop;            // 1 tol, 2 cap
  int32_t done;            // the mode's last sweep has run (set when DevInst::spec_nsw > 0)
};

// Everything a kernel may need about one instance, passed by value.
constexpr int kHsbMax = 64;   // h splits with balanced ranges (more: equal counts)

struct DevInst {
  int dim;
  int Mk;            // modes of u^k
  int Mkp;           // Mk rounded up to kTile (ldh of Xh)
  int nb;            // Mkp / kTile
  int ntri;          // tile triples A <= B <= C
  int Mcap;          // capacity of factor matrices
  int mixed;
  // speculative sweeps: with spec_nsw > 0 the finalisation of the last
  // direction sets sc->done when the sweep ends the mode (zero amplitude,
  // non-finite, converged, or sweep spec_nsw); a launch with spec_check set
  // returns at once when sc->done is set
  int spec_nsw;
  int spec_check;
  // 3D field state (adaptive algorithm, after a full solve): u^k is the
  // nodal tensor, the load of a directional solve is fparts chunks of the
  // contraction of R3 (0: u^k is separated)
  int fparts;
  const double* R3;
  double c, lam, omega, a0, kappa;
  // 2D reduced integration domain (eq. MxyRD): elements with max |w| <=
  // rd_tol are left out of M_xy; rd_count counts them (rd_tol > 0)
  double rd_tol;
  unsigned long long* rd_count;
  double fp_tol, enrich_tol;
  int max_modes;
  uint64_t seed;
  double* sk;        // sigma of u^k (Mcap)
  double* sn;        // sigma of u^{k+1} (Mcap)
  DevScalars* sc;
  DevAxis ax[kMaxDim];
  // cubic route (3D)
  const int4* tri;   // (A, B, C, weight) per triple, C-major order (g, S)
  // the h contraction's view of the triples, C-groups kept and each sorted
  // by column tile: (first, second, column tile, pair skip); (b <= c) pairs
  // for A < B = C, (a <= b) pairs when A = B, all 256 pairs otherwise
  const int4* trih;
  const int2* trimap; // per triple of tri: (position in trih, 1 if h takes it transposed)
  const int* thinv;   // per position of trih: the triple of tri
  // FP32 g by triple class: tlist holds the triples with three distinct
  // tiles (16 chains of 16 x 16 outputs) in C-major order, then those with
  // a repeated tile (9 blocks of 16 mode pairs x 16 outputs); trank[t] =
  // (class: 0 distinct, 1 A = B < C, 2 A < B = C, 3 A = B = C; rank in its list)
  const int* tlist;          // distinct-tile triples (all mode tiles of the handle)
  const int* tlist_p;        // repeated-tile triples (a prefix serves fewer tiles)
  const int2* trank;
  int ntri_d, ntri_p;        // distinct / repeated-tile triples of the current M_k
  int nsplit_p;              // point splits of a repeated-tile triple (nsplit_g: distinct)
  void* gpart;       // split-K partials of g: FP64 nsplit_g x ntri x 4096; FP32 by
                     // class: [rank][split][4096] distinct, then [rank][split][2304]
  void* S;           // ntri x 4096 (T), weighted g_e * g_f
  double* hpart;     // nsplit_h x nqmax
  // h splits of about equal MFMA work (a triple whose pair tiles coincide
  // runs 40 of the 64 k-steps): when hsb_n == nsplit_h, split s takes the
  // positions [hsb[s], hsb[s + 1]) of the h order, else ranges of equal
  // triple counts
  int hsb_n;
  int16_t hsb[kHsbMax + 1];
  double* bcr_ws;    // cyclic-reduction block data in HBM for axes too large for LDS (else null)
  int nsplit_g, nsplit_h;
  // 2D route
  double* T1;        // n0 x nq1
  double* Gq;        // Gauss-grid strip of omega (u^3 - u) W_0 W_1: gq_rows x nq1
  int gq_rows;       // rows of the strip (whole elements of axis 0)
  void* Mxy;         // n0 x n1 (T), row-major
  void* MxyT;        // n1 x n0 (T)
};

// ---------------------------------------------------------------- kernels
// (defined in kernels.hip; host wrappers launch them on a stream)
hipError_t launch_quad_eval(const DevInst& I, int d, hipStream_t st);
hipError_t launch_band_mv(const DevAxis& A, const double* band, const double* X,
                          double* Y, int ncols, hipStream_t st);
hipError_t launch_init_mode(const DevInst& I, int64_t step, int mode, int warm,
                            hipStream_t st);
hipError_t launch_finalize(const DevInst& I, int d, int sweep, int from_init,
                           hipStream_t st, int nparts = 0);
// normalisation of the initial guesses of every direction in one launch
// (one workgroup per direction; all axes share the band width)
hipError_t launch_finalize_init(const DevInst& I, hipStream_t st);
hipError_t launch_signature(const DevInst& I, int d, int M, hipStream_t st);
// launch_finalize (sweep, fast-diagonalisation partials) and launch_signature
// of the same direction in one launch, with the same results
hipError_t launch_finalize_sig(const DevInst& I, int d, int sweep, int M, hipStream_t st, int nparts);
hipError_t launch_signature_all(const DevInst& I, int M, hipStream_t st);   // every direction, one launch
hipError_t launch_rhs(const DevInst& I, int d, int M, hipStream_t st, int load_only = 0);
hipError_t launch_rhs_sum(const DevInst& I, int d, int M, int load_only, hipStream_t st);
// index of the last RHS partial chunk of direction d (consumers add chunks
// 0 ..= this one); load chunks: 2D ceil(n_other / 64), 3D one
int rhs_chunks(const DevInst& I, int d, int M, int load_only);
int rhs_load_chunks(const DevInst& I, int d);
hipError_t launch_append(const DevInst& I, int M, hipStream_t st);
// g_d as split-K partials, then their reduction into g_d and S = w g_d g_other
hipError_t launch_cubic_g(const DevInst& I, int d, hipStream_t st);
hipError_t launch_cubic_gred(const DevInst& I, int d, int e_other, hipStream_t st);
size_t cubic_h_lds(const DevInst& I);   // dynamic LDS bytes of the h kernel
size_t cubic_h_lds_total(const DevInst& I);   // dynamic + static LDS bytes of the h kernel
int cubic_h_rows(const DevInst& I);     // Gauss points per workgroup of the h kernel
int cubic_h_blocks_per_cu(const DevInst& I);   // resident h workgroups per CU
hipError_t launch_cubic_h(const DevInst& I, int d, hipStream_t st);
hipError_t launch_mxy_build(const DevInst& I, hipStream_t st);
hipError_t launch_reset_scalars(const DevInst& I, hipStream_t st);
hipError_t launch_energy(const DevInst& I, double* partial, int* npartial,
                         hipStream_t st);
hipError_t launch_energy_grams(const DevInst& I, int M, double* partial,
                               hipStream_t st);
// dst[sum_d i_d strides[d]] = src[C-order index of i], elements of esz bytes
hipError_t launch_scatter_strided(const void* src, void* dst, int esz, int dim, const int64_t* n,
                                  const int64_t* strides, hipStream_t st);
hipError_t launch_reconstruct(const DevInst& I, int M, void* out, int dtype,
                              hipStream_t st);
hipError_t launch_band_solve_batch(int n, int bw, const double* Mb,
                                   const double* Kb, const double* alpha,
                                   const double* beta, const double* b,
                                   double* x, int count, hipStream_t st);
// device workspace the batched banded solve needs (0 when the block data of
// a system fit in LDS), and the launch on a caller-provided workspace
size_t band_solve_workspace_bytes(int n, int bw, int count);
hipError_t launch_band_solve_batch_ws(int n, int bw, const double* Mb, const double* Kb,
                                      const double* alpha, const double* beta, const double* b,
                                      double* x, int count, double* gws, hipStream_t st);
hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st);
constexpr int kFdSplit = 32;   // row splits of the projection V^T b
constexpr int kFdKb = 8;      // eigenvector splits of the back-projection V z
// x = V diag(1 / (alpha + beta mu)) V^T b into ax[d].u, alpha/beta from the
// fixed factors (two launches; the normalisation follows separately)
hipError_t launch_solve_fd(const DevInst& I, int d, int M, hipStream_t st);
bool bcr_fits(int n, int B);                       // block data fit in LDS
__host__ __device__ size_t bcr_lds_bytes(int n, int B);   // block data bytes of one system
hipError_t launch_solve_bcr(const DevInst& I, int d, int sweep, int M, hipStream_t st);
// Dense FP64 product C = op(A diag(ks) B) on MFMA (actd.hip): A(i, k) =
// A[i a_i + k a_k], B(k, j) = B[k b_k + j b_j], C(i, j) = C[i c_i + j c_j];
// i < m, j < n, k < K.  Epilogues: store; alpha acc - D(i, j) (D FP64 or
// FP32); acc / (c + lam (mu0_i + mu1_j)); or no store and one partial sum
// per workgroup of w0_i w1_j acc^4 into part (gemm64_blocks(m, n) values);
// or alpha w0_i w1_j (acc^3 - acc).
enum { kEpiStore = 0, kEpiAxpby = 1, kEpiFdDiv = 2, kEpiU4 = 3, kEpiCubic = 4 };
struct GemmArgs {
  int m = 0, n = 0, K = 0, epi = kEpiStore;
  const double* A = nullptr;
  int64_t a_i = 0, a_k = 0;
  const double* B = nullptr;
  int64_t b_k = 0, b_j = 0;
  const double* ks = nullptr;
  double* C = nullptr;
  int64_t c_i = 0, c_j = 0;
  double alpha = 1.0;
  const void* D = nullptr;
  int d_f32 = 0;
  int64_t d_i = 0, d_j = 0;
  const double* mu0 = nullptr;
  const double* mu1 = nullptr;
  double c = 0.0, lam = 0.0;
  const double* w0 = nullptr;
  const double* w1 = nullptr;
  double* part = nullptr;
};
hipError_t launch_gemm64(const GemmArgs& g, hipStream_t st);
int gemm64_blocks(int m, int n);
hipError_t launch_unit_columns(double* X, int n, int ncols, hipStream_t st);   // X[:, m] = e_m
// 3D field state (actd.hip): passes of a row-major (d0, d1, d2) tensor along
// one axis -- Phi (nodes to Gauss points), Phi^T, a banded symmetric matrix,
// the eigenvector products of the full solve -- and the pointwise steps.
hipError_t launch_field_phi(const double* in, double* out, const int* dims, int a, const DevAxis& A,
                            hipStream_t st);
hipError_t launch_field_phit(const double* in, double* out, const int* dims, int a, const DevAxis& A,
                             hipStream_t st);
hipError_t launch_field_band(const double* in, double* out, const int* dims, int a, const double* band,
                             int n, int B, hipStream_t st);
hipError_t launch_field_integrand(double* G, const int* qdims, const double* w0, const double* w1,
                                  const double* w2, double omega, double a0, double* part,
                                  hipStream_t st);
int64_t field_partials(int64_t total);
hipError_t launch_field_axpby(double* R, const double* MU, const double* T, double c, int64_t total,
                              hipStream_t st);
hipError_t launch_field_dot(const double* x, const double* y, int64_t total, double* part, hipStream_t st);
hipError_t launch_field_fd_div(double* T, const int* dims, const double* mu0, const double* mu1,
                               const double* mu2, double c, double lam, hipStream_t st);
// skip: a device flag; the launch returns at once when it is set (nullptr: never)
hipError_t launch_field_contract(const double* R, const int* dims, int d, const double* u0, const double* u1,
                                 const double* u2, int P, double* out, const int* skip, hipStream_t st);
hipError_t launch_field_eig(const double* X, double* Y, const int* dims, int a, const double* V, int forward,
                            hipStream_t st);
hipError_t launch_field_to_f32(const double* X, float* Y, int64_t total, hipStream_t st);
constexpr int kLoadSub = 4;      // 3D cubic load: RHS chunks of 16-row sub-blocks of a 64-row block
constexpr int kFieldParts = 8;   // load chunks of a directional solve from a 3D field state
hipError_t launch_fill(double* x, int n, double v, hipStream_t st);
// Separated integration of the 2D M_xy (wsep.hip, Sec. 3.3 eq. MxySep):
// W = L w(u^k) on the Gauss grid (nq0 x nq1, row-major) and W^T, the Q
// greedy rank-one terms (A: nq0 x Q, B: nq1 x Q, column-major), all at the
// even strides of wsep_ld, their 1D
// integrals (Pa: n0 x Q, Pb: n1 x Q), Q + 1 dot products, a unit vector of
// max(nq0, nq1) weights.
constexpr int kWsepMaxRank = 256;
// even stride of the rows of W (of W^T) and of the columns of B (of A)
inline size_t wsep_ld(size_t n) { return (n + 1) & ~(size_t)1; }
struct WsepBufs {
  int rank = 0, iters = 0;
  double *W = nullptr, *Wt = nullptr, *A = nullptr, *B = nullptr;
  double *Pa = nullptr, *Pb = nullptr, *dots = nullptr, *ones = nullptr;
};
hipError_t launch_mxy_separated(const DevInst& I, const WsepBufs& B, hipStream_t st);
hipError_t configure_kernels();
int max_lds_bytes();
int num_cus();

// Lockstep batch (2D): per-instance arguments of a multi-instance launch,
// launch kinds and the group's grid bounds.
struct LsArg {
  int inst;       // index into the device DevInst array
  int M;          // modes of u^{k+1} built so far (append: the count after it)
  int sweep;      // sweep number of the current mode (1-based)
  int mode;       // current mode index
  int warm;       // initial guess: mode m of u^k
  int flag;       // append pending / leading signature of a continued sweep
  int nlin;       // linear RHS column chunks for M
  int nld[2];     // load chunks of the RHS of direction 0, 1
  int boff[2];    // first workgroup of this entry in the RHS launch of direction 0, 1
  int pad[2];
  int64_t step;   // time-step index (keys the counter-based guess)
};
enum { kLsReset = 0, kLsAppend, kLsInit, kLsFinalizeInit, kLsSignatureAll, kLsSignature,
       kLsSignatureFlag, kLsRhs, kLsSolve, kLsGather };
struct LsGrid {
  int nmax = 0;      // largest node count of the launched axis / instance
  int ndot = 0;      // signature dot blocks
  int nchunk = 0;    // RHS chunks (linear + load)
  int B = 0;         // band half-width shared by the group
  int nblk = 0;      // workgroups of the RHS launch (sum over the entries)
  int mode = 0, threads = 0;   // BCR storage class and threads
  size_t shm = 0;
};
hipError_t launch_multi(int kind, DevInst* insts, const LsArg* args, int count, const LsGrid& g,
                        hipStream_t st, int d = 0, DevScalars* out = nullptr);
void bcr_launch_class(int n, int B, int& mode, int& threads, size_t& shm);

// Lockstep execution of 2D instances (solver.hip): adaptive, cyclic-reduction
// solves, one band width; results equal the instances' own ctd_step.
bool lockstep_eligible(const ctd_solver* s);
int band_halfwidth(const ctd_solver* s);
// The engine behind it: instances join (add) between rounds and leave when
// their steps are done; one round is one sweep of every instance in a mode
// (with the initialisation of those starting one) and one read-back.
class Lockstep {
 public:
  explicit Lockstep(hipStream_t st);
  ~Lockstep();
  Lockstep(const Lockstep&) = delete;
  Lockstep& operator=(const Lockstep&) = delete;
  // the instance runs `nsteps` steps from its next one, on the engine's stream
  int add(ctd_solver* s, int nsteps, int* slot, std::string& err);
  // one round: `steps` gets (slot, record) of every step that ended in it,
  // `finished` the slots whose steps are all done (they leave the engine).
  // An instance that fails (non-finite amplitude) leaves the engine with its
  // (slot, error) in `failed` when given, else the round returns the error.
  int round(std::vector<std::pair<int, ctd_step_info>>& steps, std::vector<int>& finished,
            std::string& err, std::vector<std::pair<int, int>>* failed = nullptr);
  bool empty() const;
  int band() const;   // band half-width of the instances (0 before the first)
 private:
  struct Impl;
  Impl* p;
};
int lockstep_steps(std::vector<ctd_solver*>& S, int nsteps, ctd_step_info* info, hipStream_t st,
                   std::string& err);

// Instance plumbing for the executors (batch, server).
void solver_bind_stream(ctd_solver* s, hipStream_t st);   // between ctd_step calls
size_t solver_device_bytes(const ctd_solver* s);

}  // namespace ctd
