// Host orchestration of the CTD step and the C-ABI entry points.
//
// One time step (Sec. 3.3): freeze u^k (Gauss-point tables, 2D: M_xy), then
// for each new mode: initialise, sweep the directions with the directional
// solves of eq. (ux)/(KxQx) (3D analogue), test the fixed point, append, test
// the enrichment stop.  All arithmetic runs in the kernels of kernels.hip; the
// host sequences launches on the handle's stream and reads back a few scalars
// per sweep to take the threshold decisions (adaptive schedule) or follows a
// given decision log (replay schedule).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <limits>
#include <string>
#include <tuple>
#include <vector>

#include "ctd_internal.h"

using namespace ctd;

namespace {

thread_local std::string g_init_error = "no error";

// Device memory of one instance: from the caller's allocator hooks when the
// problem has them, else stream-ordered hipMallocAsync.  Buffers are cleared
// on the instance's stream; in the dry mode only the byte count is kept
// (footprint queries).
struct DeviceArena {
  std::vector<std::pair<void*, size_t>> ptrs;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  bool dry = false;
  ctd_dev_alloc_fn hook_alloc = nullptr;
  ctd_dev_free_fn hook_free = nullptr;
  void* hook_ctx = nullptr;
  hipError_t raw_alloc(void** p, size_t n) {
    if (hook_alloc) {
      *p = hook_alloc((uint64_t)n, (void*)stream, hook_ctx);
      return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    // stream-ordered: no device-wide synchronisation when other instances'
    // work is in flight on other streams
    return hipMallocAsync(p, n, stream);
  }
  // returns memory of raw_alloc; with hooks only after the stream is idle
  void raw_free(void* p, size_t n) {
    if (hook_free) {
      (void)hipStreamSynchronize(stream);
      hook_free(p, (uint64_t)n, (void*)stream, hook_ctx);
    } else {
      (void)hipFreeAsync(p, stream);
    }
  }
  hipError_t alloc(void** p, size_t n) {
    if (n == 0) n = 8;
    n = (n + 255) / 256 * 256;
    if (dry) {
      *p = nullptr;
      bytes += n;
      return hipSuccess;
    }
    hipError_t e = raw_alloc(p, n);
    if (e == hipSuccess) {
      ptrs.push_back({*p, n});
      bytes += n;
      e = hipMemsetAsync(*p, 0, n, stream);
    }
    return e;
  }
  void release() {
    if (ptrs.empty()) return;
    (void)hipStreamSynchronize(stream);
    for (auto& pn : ptrs) raw_free(pn.first, pn.second);
    if (!hook_free) (void)hipStreamSynchronize(stream);
    ptrs.clear();
  }
};

// Launch timing with HIP events on the handle's stream.
struct Profiler {
  bool on = false;
  uint32_t mask = ~0u;   // kernel classes bracketed with events
  struct Pending { int id; int ev; double flops, bytes; int64_t tag; };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  int used = 0;
  int64_t tag = 0;       // launches of a speculative sweep carry its serial number
  int64_t launches[CTD_K_COUNT] = {};
  double ms[CTD_K_COUNT] = {}, flops[CTD_K_COUNT] = {}, bytes[CTD_K_COUNT] = {};
  hipError_t event_pair(int& idx) {
    while ((int)pool.size() < used + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      pool.push_back(e);
    }
    idx = used;
    used += 2;
    return hipSuccess;
  }
  // after a stream synchronisation: fold pending launches into the totals
  hipError_t collect() {
    for (const Pending& p : pending) {
      float t = 0.f;
      hipError_t r = hipEventElapsedTime(&t, pool[p.ev], pool[p.ev + 1]);
      if (r != hipSuccess) return r;
      launches[p.id] += 1;
      ms[p.id] += t;
      flops[p.id] += p.flops;
      bytes[p.id] += p.bytes;
    }
    pending.clear();
    used = 0;
    return hipSuccess;
  }
  // a speculative sweep whose mode had ended: its launches returned at once
  // on the device and are booked apart from the kernels' own classes
  void skipped(int64_t t) {
    for (auto it = pending.rbegin(); it != pending.rend() && it->tag >= t; ++it)
      if (it->tag == t) it->id = CTD_K_SKIPPED;
  }
  void reset() {
    pending.clear();
    used = 0;
    for (int i = 0; i < CTD_K_COUNT; ++i) { launches[i] = 0; ms[i] = flops[i] = bytes[i] = 0; }
  }
  void release() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

int tri_count(int nb) { return nb * (nb + 1) * (nb + 2) / 6; }

int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

struct ctd_solver {
  ctd_problem P{};
  int dim = 0;
  double L = 0, kappa = 0, a0 = 0, alpha = 0;
  double c = 0, lam = 0, omega = 0;
  hipStream_t stream = nullptr;
  AxisTables ax[kMaxDim];
  DeviceArena arena;
  DevInst I{};
  DevScalars* sc_host = nullptr;   // pinned, two slots (slot 0: the last scalars read)
  hipEvent_t sc_ev[2] = {};        // completion of the scalar copy into each slot
  int64_t spec_serial = 0;         // tag of the launches of speculative sweeps (profiling)
  double* KXk[kMaxDim] = {};       // K X^k (energy of u^k)
  int Mk = 0, Mcap = 0, Mkp_max = 0, ntri_max = 0;
  int Mcap_ctd = 0;                // modes of a CTD state (max_modes, initial count)
  bool actd = false;               // full CFE solve past the mode cap (2D and 3D)
  // 3D field state of actd: u^k is the nodal tensor U3 (row-major n0 x n1 x
  // n2), R3 the step's right-hand-side tensor c (M0 (x) M1 (x) M2) U3 minus
  // the integrated w, G3a / G3b Gauss-grid work buffers, energy_field the
  // energy of the field state (computed with R3)
  bool field3 = false;
  double* U3 = nullptr;
  double* R3 = nullptr;
  double* G3a = nullptr;
  double* G3b = nullptr;
  double energy_field = std::numeric_limits<double>::quiet_NaN();
  WsepBufs wsep;                   // separated 2D M_xy (w_rank > 0)
  double* fsQ = nullptr;           // n0 x n1 temporaries of the full solve
  double* fsT = nullptr;
  int nsplit_g_cap = 0;
  // MFMA k-steps of the first t triples of the h order (t = 0 .. ntri_max)
  std::vector<int> hcost;
  int64_t step_index = 0;
  std::vector<int32_t> decisions_last, decisions_next;
  std::string err = "no error";
  double energy_prev = std::numeric_limits<double>::quiet_NaN();
  double* energy_partial = nullptr;
  size_t energy_partial_cap = 0;
  std::vector<double> host_tmp;
  bool use_fd[kMaxDim] = {};                            // fast-diagonalisation solve per axis
  std::shared_ptr<const FastDiag> fd[kMaxDim];          // host eigenvectors (process cache)
  Profiler prof;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* where) {
    err = std::string("HIP error in ") + where + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CTD_ENOMEM : CTD_EDEVICE;
  }
};

#define HIPCHK(s, expr)                                   \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return (s)->hip_fail(_e, #expr); \
  } while (0)

// Launch `expr` (a hipError_t-returning launcher); when profiling, bracket it
// with events and book it under kernel class `id` with algorithmic work.
#define LAUNCH_ON(s, st, id, fl, by, expr)                                   \
  do {                                                                       \
    if ((s)->prof.on && (((s)->prof.mask >> (id)) & 1u)) {                   \
      int _ev = 0;                                                           \
      HIPCHK(s, (s)->prof.event_pair(_ev));                                  \
      HIPCHK(s, hipEventRecord((s)->prof.pool[_ev], (st)));                  \
      HIPCHK(s, expr);                                                       \
      HIPCHK(s, hipEventRecord((s)->prof.pool[_ev + 1], (st)));              \
      (s)->prof.pending.push_back({(id), _ev, (double)(fl), (double)(by), (s)->prof.tag}); \
    } else {                                                                 \
      HIPCHK(s, expr);                                                       \
    }                                                                        \
  } while (0)
#define LAUNCH(s, id, fl, by, expr) LAUNCH_ON(s, (s)->stream, id, fl, by, expr)

namespace {

hipError_t sync_collect(ctd_solver* s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess && s->prof.on) e = s->prof.collect();
  return e;
}

// Copy ordered on the instance's stream, complete on return (host buffers
// may be pageable temporaries).
hipError_t copy_sync(ctd_solver* s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (s->arena.dry || bytes == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  return e;
}

// Algorithmic work of each launch (minimal operation counts from shapes).
struct Work { double flops, bytes; };
double tsz(const ctd_solver* s) { return s->I.mixed ? 4.0 : 8.0; }
double symT(int M) { return (double)M * (M + 1) * (M + 2) / 6.0; }
Work w_cubic(const ctd_solver* s, int d) {   // g or h: one FMA per (q, a<=b<=c)
  const double nq = s->I.ax[d].nq, M = s->I.Mk;
  return {2.0 * nq * symT(s->I.Mk), tsz(s) * (nq * M + symT(s->I.Mk)) + 8.0 * nq};
}
Work w_gred(const ctd_solver* s, bool with_s) {   // read partials (+ g_other), write g (+ S)
  const double tiles = (double)s->I.ntri * kTileSq * kTile;
  return {0.0, tsz(s) * tiles * (s->I.nsplit_g + 1 + (with_s ? 2 : 0))};
}
Work w_rhs(const ctd_solver* s, int d, int M) {
  const double n = s->I.ax[d].n, c = s->I.Mk + 2.0 * M;
  return {2.0 * n * c, 8.0 * n * (c + 2)};
}
Work w_solve(const ctd_solver* s, int d) {
  const double n = s->I.ax[d].n, B = s->I.ax[d].B;
  // fast diagonalisation: two dense n x n products over the eigenvectors
  if (s->use_fd[d]) return {4.0 * n * n, 8.0 * (2.0 * n * n + 4.0 * n)};
  return {n * (B * B + 6 * B + 8 * B), 8.0 * n * (2 * (B + 1) + 6)};
}
Work w_sig(const ctd_solver* s, int d, int M) {
  const double n = s->I.ax[d].n, nq = s->I.ax[d].nq, c = s->I.Mk + 2.0 * M;
  const double v = s->dim == 3 ? nq : 0.0;
  return {2.0 * n * c + 2.0 * v * s->I.ax[d].SW, 8.0 * n * (c + 1) + 8.0 * v};
}
Work w_load2d(const ctd_solver* s, int d) {
  const double a = s->I.ax[d].n, b = s->I.ax[1 - d].n;
  return {2.0 * a * b, tsz(s) * a * b};
}
Work w_mxy(const ctd_solver* s) {
  const double q0 = s->I.ax[0].nq, q1 = s->I.ax[1].nq, n0 = s->I.ax[0].n, n1 = s->I.ax[1].n;
  if (s->P.w_rank > 0) {
    // separated w: W and W^T by the product, then every update reads one of
    // them once (2 products of q0 q1 flops per update)
    const double upd = 2.0 * s->P.w_rank * s->P.w_iters;
    return {4.0 * q0 * q1 * s->I.Mk + upd * 2.0 * q0 * q1, (upd + 2.0) * 8.0 * q0 * q1 + 2.0 * tsz(s) * n0 * n1};
  }
  return {2.0 * q0 * q1 * (s->I.Mk + 2.0 * s->I.ax[0].SW), 2.0 * tsz(s) * n0 * n1};
}
Work w_quad(const ctd_solver* s, int d) {
  const double nq = s->I.ax[d].nq, n = s->I.ax[d].n, M = s->I.Mk;
  return {2.0 * nq * s->I.ax[d].SW * M, 8.0 * n * M + (8.0 + (s->I.mixed ? 4.0 : 0.0)) * nq * M};
}

int validate(const ctd_problem* p, std::string& err) {
  if (!p) { err = "problem is NULL"; return CTD_EINVAL; }
  if (p->abi_version != CTD_ABI_VERSION) { err = "abi_version mismatch"; return CTD_EINVAL; }
  if (p->dim != 2 && p->dim != 3) { err = "dim must be 2 or 3"; return CTD_EINVAL; }
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) { err = "dt must be positive"; return CTD_EINVAL; }
  if (p->max_modes < 1 || p->max_modes > 1024) { err = "max_modes must be in [1, 1024]"; return CTD_EINVAL; }
  if (p->fp_max_iter < 0 || p->fp_tol < 0.0) { err = "negative fixed-point settings"; return CTD_EINVAL; }
  if (!(p->enrich_tol >= 0.0)) { err = "enrich_tol must be >= 0"; return CTD_EINVAL; }
  if (p->precision != CTD_PREC_FP64 && p->precision != CTD_PREC_MIXED) { err = "bad precision"; return CTD_EINVAL; }
  if (p->schedule != CTD_SCHED_ADAPTIVE && p->schedule != CTD_SCHED_REPLAY) { err = "bad schedule"; return CTD_EINVAL; }
  if (p->init_mode != CTD_INIT_HASH && p->init_mode != CTD_INIT_WARM) { err = "bad init_mode"; return CTD_EINVAL; }
  if ((p->dev_alloc == nullptr) != (p->dev_free == nullptr)) {
    err = "dev_alloc and dev_free must both be set or both be NULL";
    return CTD_EINVAL;
  }
  const bool paper = std::isfinite(p->L) || std::isfinite(p->kappa) || std::isfinite(p->a0) || std::isfinite(p->alpha);
  if (paper) {
    if (!(p->L > 0) || !(p->kappa >= 0) || !(p->a0 >= 0) || !(p->alpha >= 0)) {
      err = "paper-form coefficients must all be given: L > 0, kappa >= 0, a0 >= 0, alpha >= 0";
      return CTD_EINVAL;
    }
  } else {
    if (!(p->eps > 0) || !std::isfinite(p->eps)) { err = "eps must be positive"; return CTD_EINVAL; }
    if (!(p->S >= 0) || !std::isfinite(p->S)) { err = "S must be >= 0"; return CTD_EINVAL; }
  }
  if (p->actd) {
    for (int d = 0; d < p->dim; ++d)
      if (p->nodes[d] > 2048) { err = "actd needs nodes <= 2048 per axis"; return CTD_EUNSUPPORTED; }
    if (p->dim == 3) {
      // the full step and the field state work on the tensor Gauss grid
      const double ng = p->gauss_points > 0 ? p->gauss_points : 5;
      double q = 1.0;
      for (int d = 0; d < 3; ++d) q *= ng * (p->nodes[d] - 1);
      if (q > (double)(1u << 30)) {
        err = "actd in 3D needs at most 2^30 tensor Gauss points (about 200 nodes per axis at 5 points)";
        return CTD_EUNSUPPORTED;
      }
    }
  }
  if (!(p->rd_tol >= 0.0) || !std::isfinite(p->rd_tol)) { err = "rd_tol must be finite and >= 0"; return CTD_EINVAL; }
  if (p->rd_tol > 0.0 && (p->dim != 2 || p->actd)) {
    err = "the reduced integration domain (rd_tol > 0) is defined for the 2D M_xy without actd";
    return CTD_EUNSUPPORTED;
  }
  if (p->w_rank < 0 || p->w_rank > kWsepMaxRank || p->w_iters < 0 || p->w_iters > 100000) {
    err = "need 0 <= w_rank <= 256 and 0 <= w_iters <= 100000";
    return CTD_EINVAL;
  }
  if (p->w_rank > 0 && (p->dim != 2 || p->actd || p->rd_tol > 0.0)) {
    err = "the separated w (w_rank > 0) is defined for the 2D M_xy without actd or rd_tol";
    return CTD_EUNSUPPORTED;
  }
  if (p->patch_s < 1 || p->patch_s > 3) { err = "patch_s must be 1, 2 or 3"; return CTD_EINVAL; }
  if (p->poly_p < 0 || p->poly_p > p->patch_s) { err = "need 0 <= poly_p <= patch_s"; return CTD_EINVAL; }
  for (int d = 0; d < p->dim; ++d) {
    if (p->nodes[d] < 2 * p->patch_s + 2) { err = "need nodes >= 2*patch_s+2 on every axis"; return CTD_EINVAL; }
    if (!(p->hi[d] > p->lo[d])) { err = "need hi > lo on every axis"; return CTD_EINVAL; }
  }
  return CTD_OK;
}

// Tile triples A <= B <= C in C-major order with multiplicities.
std::vector<int4> make_triples(int nb) {
  std::vector<int4> t;
  for (int C = 0; C < nb; ++C)
    for (int B = 0; B <= C; ++B)
      for (int A = 0; A <= B; ++A) {
        int w = (A == B && B == C) ? 1 : ((A == B || B == C) ? 3 : 6);
        t.push_back(int4{A, B, C, w});
      }
  return t;
}

// The h contraction's order of the same triples.  h runs each triple as an
// MFMA product over pairs of modes (first, second tile) against the modes of
// the column tile; where two tiles coincide it takes their pairs once (the
// ordered pairs below the diagonal meet zero weights and are skipped): A = B
// pairs (a <= b) with column C; A < B = C pairs (b <= c) with column A.  The
// C-groups of the C-major order stay in place (a step with fewer mode tiles
// uses a prefix), and inside a group the triples are sorted by column tile so
// that the per-column closing sums run once per column.
// Class lists of the FP32 g contraction (C-major order kept inside each list,
// so a step with fewer mode tiles uses a prefix of both).
void make_g_classes(const std::vector<int4>& tri, std::vector<int>& tlist, std::vector<int2>& trank) {
  const int n = (int)tri.size();
  std::vector<int> d, p;
  trank.assign(n, int2{0, 0});
  for (int i = 0; i < n; ++i) {
    const int4 t = tri[i];
    const int cls = t.x < t.y && t.y < t.z ? 0 : (t.x == t.y && t.y < t.z ? 1 : (t.x < t.y ? 2 : 3));
    if (cls == 0) { trank[i] = int2{0, (int)d.size()}; d.push_back(i); }
    else { trank[i] = int2{cls, (int)p.size()}; p.push_back(i); }
  }
  tlist = d;
  tlist.insert(tlist.end(), p.begin(), p.end());
}

void make_h_order(const std::vector<int4>& tri, std::vector<int4>& trih, std::vector<int2>& map) {
  const int n = (int)tri.size();
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  auto col = [&](int i) { const int4 t = tri[i]; return (t.x < t.y && t.y == t.z) ? t.x : t.z; };
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (tri[a].z != tri[b].z) return tri[a].z < tri[b].z;
    return col(a) < col(b);
  });
  trih.assign(n, int4{0, 0, 0, 0});
  map.assign(n, int2{0, 0});
  for (int p = 0; p < n; ++p) {
    const int4 t = tri[ord[p]];
    const bool p2 = t.x < t.y && t.y == t.z;
    trih[p] = p2 ? int4{t.y, t.z, t.x, 1} : int4{t.x, t.y, t.z, t.x == t.y ? 1 : 0};
    map[ord[p]] = int2{p, p2 ? 1 : 0};
  }
}

// ---- tuning table of the 3D cubic contraction (see ctd_tuning_set)
namespace {
std::mutex g_tune_mu;
// (precision, nb, nq) -> (nsplit_g, nsplit_h)
std::map<std::tuple<int, int, int>, std::pair<int, int>> g_tune;
}  // namespace

bool tuning_lookup(int prec, int nb, int nq, int& ng, int& nh) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({prec, nb, nq});
  if (it == g_tune.end()) return false;
  ng = it->second.first;
  nh = it->second.second;
  return true;
}

// Point splits of the FP32 g contraction by triple class.  A distinct-tile
// triple costs 16 chains per point, a repeated-tile one 9 pair blocks, so the
// latter get about 16/9 as many points per split; the distinct split count is
// the one that minimises the launch length (longest workgroup times the
// rounds of resident workgroups), or the tuning table's entry when it has
// one.  Splits are whole 64-point chunks; the partials stay within what the
// handle allocated.
void fp32_g_splits(ctd_solver* s, int nq, int forced) {
  DevInst& I = s->I;
  const int nb = I.nb;
  int nd = 0;
  for (int C = 0; C < nb; ++C)
    for (int B = 0; B <= C; ++B)
      for (int A = 0; A <= B; ++A) nd += (A < B && B < C) ? 1 : 0;
  I.ntri_d = nd;
  I.ntri_p = I.ntri - nd;
  const int nchunk = (nq + 63) / 64;
  const double slots = (double)num_cus() * 4.0;
  auto plan = [&](int nsd, int& pd, int& pp, int& nsp) {
    pd = (nchunk + nsd - 1) / nsd * 64;
    pp = std::min(nchunk * 64, ((pd * 16 + 8) / 9 + 63) / 64 * 64);
    nsp = (nq + pp - 1) / pp;
  };
  // Split counts that are multiples of 8 keep each XCD's L2 on one eighth of
  // the tables (kernel placement); measured on the 1024^3 workload that is
  // worth about a fifth of the launch length, so such a count is taken when
  // its modelled length is within 25 % of the best.
  int best = 1, best8 = 0;
  double best_cost = 1e300, best8_cost = 1e300;
  for (int nsd = 1; nsd <= nchunk; ++nsd) {
    int pd, pp, nsp;
    plan(nsd, pd, pp, nsp);
    const int nsd_eff = (nq + pd - 1) / pd;
    const double wgs = (double)nd * nsd_eff + (double)I.ntri_p * nsp;
    const double floats = (double)nd * nsd_eff * 4096.0 + (double)I.ntri_p * nsp * 2304.0;
    if (floats > (double)s->nsplit_g_cap * 4096.0) continue;
    const double len = std::max(16.0 * (nd ? pd : 0), 9.0 * (I.ntri_p ? pp : 0));
    const double cost = len * std::ceil(wgs / slots);
    if (forced > 0 ? nsd == std::min(forced, nchunk) : cost < best_cost * 0.999) {
      best = nsd;
      best_cost = cost;
      if (forced > 0) break;
    }
    if (nsd_eff == nsd && nsd % 8 == 0 && cost < best8_cost * 0.999) {
      best8 = nsd;
      best8_cost = cost;
    }
  }
  if (forced <= 0 && best8 > 0 && best % 8 != 0 && best8_cost <= 1.25 * best_cost) best = best8;
  int pd, pp, nsp;
  plan(best, pd, pp, nsp);
  // the kernel spreads each axis' Gauss points over these split counts
  I.nsplit_g = (nq + pd - 1) / pd;
  I.nsplit_p = nsp;
  // a multiple of 8 distinct splits: the repeated-tile triples take the same
  // point ranges, so that each XCD reads one eighth of the tables (kernel
  // placement), when the workgroups still fit one resident round and the
  // partial buffer
  if (I.nsplit_g % 8 == 0 && I.nsplit_g != nsp) {
    const double wgs = (double)nd * I.nsplit_g + (double)I.ntri_p * I.nsplit_g;
    const double floats = (double)nd * I.nsplit_g * 4096.0 + (double)I.ntri_p * I.nsplit_g * 2304.0;
    if (wgs <= slots && floats <= (double)s->nsplit_g_cap * 4096.0) I.nsplit_p = I.nsplit_g;
  }
}

// Split boundaries of the h contraction with about equal MFMA work per
// split: boundary s is the position whose k-step prefix is nearest to s/n of
// the total (ranges may be empty; the kernels then write zero partials).
void h_split_ranges(ctd_solver* s) {
  DevInst& I = s->I;
  const int ns = I.nsplit_h, nt = I.ntri;
  I.hsb_n = 0;
  if (ns > kHsbMax || (int)s->hcost.size() < nt + 1) return;
  const double total = (double)s->hcost[nt];
  int t = 0;
  I.hsb[0] = 0;
  for (int k = 1; k < ns; ++k) {
    const double target = total * k / ns;
    while (t < nt && s->hcost[t + 1] <= target) ++t;
    // s->hcost[t] <= target < s->hcost[t + 1] (or t == nt)
    int b = t;
    if (t < nt && s->hcost[t + 1] - target < target - s->hcost[t]) b = t + 1;
    I.hsb[k] = (int16_t)std::max<int>(b, I.hsb[k - 1]);
  }
  I.hsb[ns] = (int16_t)nt;
  I.hsb_n = ns;
}

void update_view(ctd_solver* s) {
  DevInst& I = s->I;
  I.Mk = s->Mk;
  I.fparts = s->field3 ? kFieldParts : 0;
  I.R3 = s->R3;
  I.Mkp = std::max(kTile, round_up(s->Mk, kTile));
  I.nb = I.Mkp / kTile;
  I.ntri = tri_count(I.nb);
  if (s->dim == 3) {
    int nqmin = 1 << 30;
    for (int d = 0; d < 3; ++d) nqmin = std::min(nqmin, I.ax[d].nq);
    // g: about 1024 workgroups of 64-point chunks; a multiple of 8 splits
    // when there are at least 8 (XCD-aware split mapping in the kernel)
    int ng = std::max(1, std::min((1024 + I.ntri - 1) / I.ntri, (nqmin + 63) / 64));
    if (ng >= 8) ng = ng / 8 * 8;
    // h, triples split by MFMA work: FP32 two rounds of resident workgroups
    // (the second round evens out the workgroups' unequal lengths); FP64
    // one round (measured at 1024^3: 3 splits 175 us, 12 splits 194 us)
    const int nqt = (nqmin + cubic_h_rows(I) - 1) / cubic_h_rows(I);
    const int per_cu = std::max(1, std::min(8, cubic_h_blocks_per_cu(I)));
    const int slots = num_cus() * per_cu;
    int nh = (I.mixed ? 2 : 1) * slots / nqt;
    // a measured table entry for this precision and shape replaces the heuristic
    int tg = 0, th = 0;
    if (tuning_lookup(I.mixed ? CTD_PREC_MIXED : CTD_PREC_FP64, I.nb, nqmin, tg, th)) {
      ng = tg;
      nh = th;
    } else {
      tg = 0;
    }
    ng = std::min(ng, (nqmin + 63) / 64);
    ng = std::min(ng, s->nsplit_g_cap / I.ntri);
    I.nsplit_g = std::max(1, ng);
    I.nsplit_h = std::max(1, std::min(I.ntri, nh));
    h_split_ranges(s);
    if (I.mixed) fp32_g_splits(s, nqmin, tg > 0 ? tg : 0);
  }
}

// Coefficients, defaults and the host CFE tables of every axis.
int setup_host(ctd_solver* s, const ctd_problem* p, void* hip_stream, std::string& err) {
  s->P = *p;
  if (s->P.dilation_a == 0.0) s->P.dilation_a = 12.0;
  if (s->P.gauss_points == 0) s->P.gauss_points = 5;
  if (s->P.fp_tol == 0.0) s->P.fp_tol = 1e-2;
  if (s->P.fp_max_iter == 0) s->P.fp_max_iter = 20;
  if (s->P.w_iters == 0) s->P.w_iters = 30;
  s->dim = p->dim;
  if (std::isfinite(p->L)) {
    s->L = p->L; s->kappa = p->kappa; s->a0 = p->a0; s->alpha = p->alpha;
  } else {
    s->L = 1.0; s->kappa = p->eps * p->eps; s->a0 = 0.25; s->alpha = p->S;
  }
  s->c = 1.0 / p->dt + s->alpha * s->L;
  s->lam = s->L * s->kappa;
  s->omega = 4.0 * s->a0 * s->L;
  s->stream = (hipStream_t)hip_stream;
  s->arena.stream = s->stream;
  s->arena.hook_alloc = p->dev_alloc;
  s->arena.hook_free = p->dev_free;
  s->arena.hook_ctx = p->alloc_ctx;
  for (int d = 0; d < s->dim; ++d) {
    int rc = build_axis(p->nodes[d], p->lo[d], p->hi[d], p->patch_s, p->poly_p,
                        s->P.dilation_a, s->P.gauss_points, s->ax[d], err);
    if (rc) return rc;
  }
  return CTD_OK;
}

int alloc_instance(ctd_solver* s, int m0) {
  DeviceArena& A = s->arena;
  DevInst& I = s->I;
  const bool mixed = s->P.precision == CTD_PREC_MIXED;
  s->actd = s->P.actd != 0;
  s->Mcap_ctd = std::max(s->P.max_modes, m0);
  // a 2D field state from the full solve holds one mode per node of axis 1
  // (a 3D one is held as a tensor)
  s->Mcap = s->actd && s->dim == 2 ? std::max(s->Mcap_ctd, s->ax[1].n) : s->Mcap_ctd;
  s->Mkp_max = std::max(kTile, round_up(s->Mcap, kTile));
  const int nbmax = s->Mkp_max / kTile;
  s->ntri_max = tri_count(nbmax);
  {
    // split-K partial tiles of g: at most ~1024 workgroups, and no more
    // splits than 64-point chunks on the shortest axis
    int nqmin = 1 << 30;
    for (int d = 0; d < s->dim; ++d) nqmin = std::min(nqmin, s->ax[d].nq);
    s->nsplit_g_cap = std::min(1024 + s->ntri_max, s->ntri_max * ((nqmin + 63) / 64));
  }
  const size_t Tsz = mixed ? sizeof(float) : sizeof(double);
  I.dim = s->dim;
  I.Mcap = s->Mcap;
  I.mixed = mixed;
  I.c = s->c; I.lam = s->lam; I.omega = s->omega; I.a0 = s->a0; I.kappa = s->kappa;
  I.rd_tol = s->P.rd_tol;
  I.fp_tol = s->P.fp_tol;
  I.enrich_tol = s->P.enrich_tol;
  I.max_modes = s->P.max_modes;
  I.seed = s->P.seed;
#define AL(ptr, bytes) HIPCHK(s, A.alloc((void**)&(ptr), (bytes)))
  AL(I.sk, sizeof(double) * s->Mcap);
  AL(I.sn, sizeof(double) * s->Mcap);
  AL(I.sc, sizeof(DevScalars));
  int nqmax = 0;
  for (int d = 0; d < s->dim; ++d) {
    const AxisTables& T = s->ax[d];
    DevAxis& X = I.ax[d];
    X.n = T.n; X.nq = T.nq; X.ng = T.ng; X.SW = T.SW; X.B = T.B; X.s = T.s;
    nqmax = std::max(nqmax, T.nq);
    const size_t n = T.n, nq = T.nq, M = s->Mcap;
    AL(X.phi, sizeof(double) * nq * T.SW);
    AL(X.phif, sizeof(float) * nq * T.SW);
    AL(X.w, sizeof(double) * nq);
    AL(X.Mb, sizeof(double) * (T.B + 1) * n);
    AL(X.Kb, sizeof(double) * (T.B + 1) * n);
    AL(X.Xk, sizeof(double) * n * M);
    AL(X.MXk, sizeof(double) * n * M);
    AL(s->KXk[d], sizeof(double) * n * M);
    // Gauss-point tables: rows padded to a multiple of 64 with zero rows
    // (the cubic g kernel loads whole 64-point chunks)
    const size_t nqp = (nq + 63) / 64 * 64;
    AL(X.Xh, sizeof(double) * nqp * s->Mkp_max);
    if (mixed) AL(X.Xhf, sizeof(float) * nqp * s->Mkp_max);
    if (mixed && s->dim == 3) AL(X.Xhg, sizeof(float) * nqp * s->Mkp_max);
    AL(X.X, sizeof(double) * n * M);
    AL(X.MX, sizeof(double) * n * M);
    AL(X.KX, sizeof(double) * n * M);
    AL(X.u, sizeof(double) * n);
    AL(X.up, sizeof(double) * n);
    AL(X.Mu, sizeof(double) * n);
    AL(X.Ku, sizeof(double) * n);
    AL(X.rhs, sizeof(double) * n);
    // RHS partials: linear column chunks, then the load chunks (2D: the
    // columns of the M_xy product, 64 per chunk)
    const size_t nload = s->dim == 2 ? (size_t)(s->ax[1 - d].n + 63) / 64
                                     : (size_t)std::max(kLoadSub, s->actd ? kFieldParts : 0);
    AL(X.rpart, sizeof(double) * n * ((size_t)(3 * s->Mcap + 63) / 64 + nload));
    AL(X.v, sizeof(double) * nqp);
    if (mixed) AL(X.vf, sizeof(float) * nqp);
    AL(X.gm, sizeof(double) * M);
    AL(X.gk, sizeof(double) * M);
    AL(X.gmk, sizeof(double) * M);
    if (s->dim == 3) AL(X.g, Tsz * (size_t)s->ntri_max * kTileSq * kTile);
    std::vector<float> pf(T.phi.begin(), T.phi.end());
    HIPCHK(s, copy_sync(s, X.phi, T.phi.data(), sizeof(double) * nq * T.SW, hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, X.phif, pf.data(), sizeof(float) * nq * T.SW, hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, X.w, T.w.data(), sizeof(double) * nq, hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, X.Mb, T.Mb.data(), sizeof(double) * (T.B + 1) * n, hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, X.Kb, T.Kb.data(), sizeof(double) * (T.B + 1) * n, hipMemcpyHostToDevice));
  }
  if (s->dim == 3) {
    std::vector<int4> tri = make_triples(nbmax);
    int4* td;
    AL(td, sizeof(int4) * tri.size());
    HIPCHK(s, copy_sync(s, td, tri.data(), sizeof(int4) * tri.size(), hipMemcpyHostToDevice));
    I.tri = td;
    std::vector<int4> trih;
    std::vector<int2> map;
    make_h_order(tri, trih, map);
    s->hcost.assign(trih.size() + 1, 0);
    for (size_t t = 0; t < trih.size(); ++t) s->hcost[t + 1] = s->hcost[t] + (trih[t].w ? 40 : 64);
    std::vector<int> inv(map.size());
    for (size_t t = 0; t < map.size(); ++t) inv[map[t].x] = (int)t;
    int4* thd;
    int2* tmd;
    int* tid;
    AL(thd, sizeof(int4) * trih.size());
    AL(tmd, sizeof(int2) * map.size());
    AL(tid, sizeof(int) * inv.size());
    HIPCHK(s, copy_sync(s, thd, trih.data(), sizeof(int4) * trih.size(), hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, tmd, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, tid, inv.data(), sizeof(int) * inv.size(), hipMemcpyHostToDevice));
    I.trih = thd;
    I.trimap = tmd;
    I.thinv = tid;
    std::vector<int> tlist;
    std::vector<int2> trank;
    make_g_classes(tri, tlist, trank);
    int* tld;
    int2* trd;
    AL(tld, sizeof(int) * tlist.size());
    AL(trd, sizeof(int2) * trank.size());
    HIPCHK(s, copy_sync(s, tld, tlist.data(), sizeof(int) * tlist.size(), hipMemcpyHostToDevice));
    HIPCHK(s, copy_sync(s, trd, trank.data(), sizeof(int2) * trank.size(), hipMemcpyHostToDevice));
    int ndmax = 0;
    for (const int2& r : trank) ndmax += r.x == 0 ? 1 : 0;
    I.tlist = tld;
    I.tlist_p = tld + ndmax;
    I.trank = trd;
    AL(I.gpart, Tsz * (size_t)s->nsplit_g_cap * kTileSq * kTile);
    AL(I.S, Tsz * (size_t)s->ntri_max * kTileSq * kTile);
    const int nqt = (nqmax + 63) / 64;
    const int nsh_cap = std::max(1, std::min(s->ntri_max, (1024 + nqt - 1) / nqt)) + 1;
    AL(I.hpart, sizeof(double) * (size_t)(s->ntri_max + nsh_cap) * nqmax);
  } else {
    const size_t n0 = s->ax[0].n, n1 = s->ax[1].n, nq1 = s->ax[1].nq;
    AL(I.T1, sizeof(double) * n0 * nq1);
    {
      // Gauss-grid strip of the M_xy integrand: whole elements of axis 0,
      // about 32 MB
      const size_t ng = s->ax[0].ng;
      const size_t rows = std::max<size_t>(1, (32u << 20) / (sizeof(double) * nq1 * ng)) * ng;
      I.gq_rows = (int)std::min<size_t>(rows, (size_t)s->ax[0].nq);
      AL(I.Gq, sizeof(double) * (size_t)I.gq_rows * nq1);
    }
    AL(I.Mxy, Tsz * n0 * n1);
    AL(I.MxyT, Tsz * n0 * n1);
    AL(I.rd_count, sizeof(unsigned long long));
    if (s->P.w_rank > 0) {
      WsepBufs& W = s->wsep;
      const size_t nq0 = s->ax[0].nq, Q = s->P.w_rank;
      W.rank = (int)Q;
      W.iters = s->P.w_iters;
      AL(W.W, sizeof(double) * nq0 * wsep_ld(nq1));
      AL(W.Wt, sizeof(double) * nq1 * wsep_ld(nq0));
      AL(W.A, sizeof(double) * wsep_ld(nq0) * Q);
      AL(W.B, sizeof(double) * wsep_ld(nq1) * Q);
      AL(W.Pa, sizeof(double) * n0 * Q);
      AL(W.Pb, sizeof(double) * n1 * Q);
      AL(W.dots, sizeof(double) * (Q + 1));
      AL(W.ones, sizeof(double) * std::max(nq0, nq1));
    }
    if (s->actd) {
      AL(s->fsQ, sizeof(double) * n0 * n1);
      AL(s->fsT, sizeof(double) * n0 * n1);
    }
  }
  // energy partials: the pair route serves states of at most Mcap_ctd modes,
  // the direct 2D route one value per 64 x 64 Gauss-point tile
  const int nbmx = std::max(kTile, round_up(s->Mcap_ctd, kTile)) / kTile;
  const int npt = nbmx * (nbmx + 1) / 2;
  s->energy_partial_cap = std::max<size_t>((size_t)npt * (npt + 1) / 2 * 16, 2 * (size_t)s->Mcap) + 16;
  if (s->dim == 2)
    s->energy_partial_cap = std::max<size_t>(s->energy_partial_cap,
                                             (size_t)gemm64_blocks(s->ax[0].nq, s->ax[1].nq) + 16);
  if (s->dim == 3 && s->actd) {
    size_t nn = 1, qq = 1;
    for (int d = 0; d < 3; ++d) {
      nn *= (size_t)s->ax[d].n;
      qq *= (size_t)s->ax[d].nq;
    }
    AL(s->U3, sizeof(double) * nn);
    AL(s->R3, sizeof(double) * nn);
    // G3a also holds two n^3 products of the right-hand side (field_rhs)
    AL(s->G3a, sizeof(double) * std::max(2 * nn, qq));
    AL(s->G3b, sizeof(double) * std::max(nn, qq));
    s->energy_partial_cap = std::max<size_t>(s->energy_partial_cap,
                                             (size_t)field_partials((int64_t)std::max(nn, qq)) + 16);
  }
  AL(s->energy_partial, sizeof(double) * s->energy_partial_cap);
  {
    // directional solve per axis: fast diagonalisation (eigenvectors shared
    // by the axes of one shape) or cyclic reduction
    bool all_small = true;
    for (int d = 0; d < s->dim; ++d) all_small = all_small && s->ax[d].n <= 1024;
    const int method = s->P.solve_method;
    for (int d = 0; d < s->dim; ++d)
      s->use_fd[d] = method == CTD_SOLVE_FD || (method == CTD_SOLVE_AUTO && s->dim == 3 && all_small);
    // the eigenbases also serve the full solve of actd
    auto eig = [&](int d) { return s->use_fd[d] || s->actd; };
    for (int d = 0; d < s->dim; ++d) {
      if (!eig(d)) continue;
      const AxisTables& T = s->ax[d];
      const size_t n = T.n;
      DevAxis& X = I.ax[d];
      if (s->use_fd[d]) {
        AL(X.fdz, sizeof(double) * kFdSplit * n);
        AL(X.fdu, sizeof(double) * kFdKb * n);
      }
      int same = -1;
      for (int e = 0; e < d; ++e) {
        const AxisTables& U = s->ax[e];
        if (eig(e) && U.n == T.n && U.lo == T.lo && U.hi == T.hi && U.s == T.s &&
            U.p == T.p && U.a == T.a && U.ng == T.ng)
          same = e;
      }
      if (same >= 0) {
        X.fdV = I.ax[same].fdV;
        X.fdmu = I.ax[same].fdmu;
        s->fd[d] = s->fd[same];
        continue;
      }
      double *V = nullptr, *mu = nullptr;
      AL(V, sizeof(double) * n * n);
      AL(mu, sizeof(double) * n);
      X.fdV = V;
      X.fdmu = mu;
      if (A.dry) continue;
      std::string ferr;
      s->fd[d] = fast_diag_cached(T, ferr);
      if (!s->fd[d]) return s->fail(CTD_EUNSUPPORTED, "fast diagonalisation: " + ferr);
      HIPCHK(s, copy_sync(s, V, s->fd[d]->V.data(), sizeof(double) * n * n, hipMemcpyHostToDevice));
      HIPCHK(s, copy_sync(s, mu, s->fd[d]->mu.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    }
    // cyclic-reduction block data of axes too large for LDS live in HBM
    size_t ws = 0;
    for (int d = 0; d < s->dim; ++d)
      if (!s->use_fd[d] && !bcr_fits(s->ax[d].n, s->ax[d].B))
        ws = std::max(ws, bcr_lds_bytes(s->ax[d].n, s->ax[d].B));
    if (ws) AL(I.bcr_ws, ws);
  }
#undef AL
  if (!A.dry) {
    HIPCHK(s, hipHostMalloc((void**)&s->sc_host, 2 * sizeof(DevScalars), hipHostMallocDefault));
    for (int k = 0; k < 2; ++k) HIPCHK(s, hipEventCreateWithFlags(&s->sc_ev[k], hipEventDisableTiming));
  }
  return CTD_OK;
}

// Gauss-point tables of u^k and, on the 2D route, M_xy (frozen for the step).
int field_rhs(ctd_solver* s, bool energy);

int precompute(ctd_solver* s) {
  update_view(s);
  if (s->field3) return field_rhs(s, true);
  for (int d = 0; d < s->dim; ++d) {
    Work w = w_quad(s, d);
    LAUNCH(s, CTD_K_QUAD, w.flops, w.bytes, launch_quad_eval(s->I, d, s->stream));
  }
  if (s->dim == 2) {
    Work w = w_mxy(s);
    if (s->P.w_rank > 0)
      LAUNCH(s, CTD_K_MXY, w.flops, w.bytes, launch_mxy_separated(s->I, s->wsep, s->stream));
    else
      LAUNCH(s, CTD_K_MXY, w.flops, w.bytes, launch_mxy_build(s->I, s->stream));
  }
  return CTD_OK;
}

int read_scalars(ctd_solver* s) {
  HIPCHK(s, hipMemcpyAsync(s->sc_host, s->I.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, sync_collect(s));
  return CTD_OK;
}

// g_d of the freshly finalised factor u_d and S for the next solve direction.
int cubic_after(ctd_solver* s, int d, int next) {
  if (s->dim != 3 || s->field3) return CTD_OK;
  int other = -1;
  if (next >= 0)
    for (int e = 0; e < 3; ++e)
      if (e != d && e != next) other = e;
  Work w = w_cubic(s, d), wr = w_gred(s, other >= 0);
  LAUNCH(s, CTD_K_CUBIC_G, w.flops, w.bytes, launch_cubic_g(s->I, d, s->stream));
  LAUNCH(s, CTD_K_CUBIC_GRED, wr.flops, wr.bytes, launch_cubic_gred(s->I, d, other, s->stream));
  return CTD_OK;
}

int energy_of_uk(ctd_solver* s, double* E) {
  if (s->field3) {
    // computed with the field state's right-hand side (field_rhs)
    *E = s->energy_field;
    HIPCHK(s, sync_collect(s));
    return CTD_OK;
  }
  // view on u^k: factor buffers X^k, M X^k, K X^k and amplitudes sk
  DevInst V = s->I;
  for (int d = 0; d < s->dim; ++d) {
    V.ax[d].X = s->I.ax[d].Xk;
    V.ax[d].MX = s->I.ax[d].MXk;
    V.ax[d].KX = s->KXk[d];
  }
  V.sn = s->I.sk;
  const int M = s->Mk;
  {
    const double n = s->I.ax[0].n;
    LAUNCH(s, CTD_K_ENERGY, 4.0 * s->dim * (double)M * M * n, 24.0 * s->dim * (double)M * n,
           launch_energy_grams(V, M, s->energy_partial, s->stream));
  }
  std::vector<double> g2((size_t)2 * M);
  HIPCHK(s, hipMemcpyAsync(g2.data(), s->energy_partial, sizeof(double) * 2 * M, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, sync_collect(s));
  double u2 = 0, gr = 0;
  for (int a = 0; a < M; ++a) { u2 += g2[2 * a]; gr += g2[2 * a + 1]; }
  int np = 0;
  const double P = (double)M * (M + 1) / 2.0;
  bool direct = false;
  if (s->dim == 2) {
    // int u^4 straight from the Gauss-point field u = Xh_0 Xh_1^T when that
    // is cheaper than the pair Grams (and always for field states)
    const double q0 = s->I.ax[0].nq, q1 = s->I.ax[1].nq;
    direct = M > s->Mcap_ctd || q0 * q1 * M < (q0 + q1) * P * P;
  }
  if (direct) {
    const DevInst& I = s->I;
    GemmArgs g;
    g.m = I.ax[0].nq; g.n = I.ax[1].nq; g.K = M; g.epi = kEpiU4;
    g.A = I.ax[0].Xh; g.a_i = I.Mkp; g.a_k = 1;
    g.B = I.ax[1].Xh; g.b_k = 1; g.b_j = I.Mkp;
    g.w0 = I.ax[0].w; g.w1 = I.ax[1].w;
    g.part = s->energy_partial;
    np = gemm64_blocks(g.m, g.n);
    LAUNCH(s, CTD_K_ENERGY, 2.0 * g.m * g.n * (double)M, 8.0 * (g.m + g.n) * (double)M,
           launch_gemm64(g, s->stream));
  } else {
    double fl = 0.0, by = 0.0;
    for (int d = 0; d < s->dim; ++d) { fl += 2.0 * s->I.ax[d].nq * P * P; by += 8.0 * s->I.ax[d].nq * M; }
    LAUNCH(s, CTD_K_ENERGY, fl, by, launch_energy(V, s->energy_partial, &np, s->stream));
  }
  std::vector<double> part(np);
  if (np) {
    HIPCHK(s, hipMemcpyAsync(part.data(), s->energy_partial, sizeof(double) * np, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, sync_collect(s));
  }
  double u4 = 0;
  for (int i = 0; i < np; ++i) u4 += part[i];
  double vol = 1.0;
  for (int d = 0; d < s->dim; ++d) vol *= s->ax[d].hi - s->ax[d].lo;
  *E = s->a0 * (u4 - 2.0 * u2 + vol) + 0.5 * s->kappa * gr;
  return CTD_OK;
}

// End of step: the new modes become u^k.
int finish_step(ctd_solver* s, int M) {
  DevInst& I = s->I;
  for (int d = 0; d < s->dim; ++d) {
    std::swap(I.ax[d].Xk, I.ax[d].X);
    std::swap(I.ax[d].MXk, I.ax[d].MX);
    std::swap(s->KXk[d], I.ax[d].KX);
  }
  std::swap(I.sk, I.sn);
  s->Mk = M;
  return precompute(s);
}

// Right-hand-side tensor of a 3D field state U3 (Sec. 3.3 adaptive
// algorithm; the 3D counterpart of c M_0 U M_1 - M_xy):
//   R3 = c (M_0 (x) M_1 (x) M_2) U3 - int N~ (x) N~ (x) N~ omega (u^3 - u),
// the integral on the tensor Gauss grid (Phi along each axis, the integrand
// at every point, Phi^T along each axis).  With energy, also the field's
// energy (Sec. 2.1): a0 sum_q W (u^2 - 1)^2 + kappa/2 sum_d U3 . (K_d (x)
// M (x) M) U3.
int field_rhs(ctd_solver* s, bool energy) {
  const DevInst& I = s->I;
  int dims[3] = {I.ax[0].n, I.ax[1].n, I.ax[2].n};
  const int64_t nn = (int64_t)dims[0] * dims[1] * dims[2];
  double* a = s->G3a;
  double* b = s->G3b;
  // Gauss-grid values: axis 2, 1, 0 in turn
  int cur[3] = {dims[0], dims[1], dims[2]};
  const double* src = s->U3;
  for (int ax = 2; ax >= 0; --ax) {
    double* dst = (ax % 2 == 0) ? a : b;
    HIPCHK(s, launch_field_phi(src, dst, cur, ax, I.ax[ax], s->stream));
    cur[ax] = I.ax[ax].nq;
    src = dst;
  }
  // src == a: the Gauss-point values; integrand (and quartic energy) in place
  const int64_t nqq = (int64_t)cur[0] * cur[1] * cur[2];
  const int64_t npart = field_partials(nqq);
  HIPCHK(s, launch_field_integrand(a, cur, I.ax[0].w, I.ax[1].w, I.ax[2].w, s->omega, s->a0,
                                   energy ? s->energy_partial : nullptr, s->stream));
  double quart = 0.0;
  if (energy) {
    std::vector<double> part((size_t)npart);
    HIPCHK(s, hipMemcpyAsync(part.data(), s->energy_partial, sizeof(double) * npart, hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (double v : part) quart += v;
  }
  // back to the nodes: axis 0, 1, 2 in turn (a -> b -> a -> b)
  src = a;
  for (int ax = 0; ax < 3; ++ax) {
    double* dst = (ax % 2 == 0) ? b : a;
    HIPCHK(s, launch_field_phit(src, dst, cur, ax, I.ax[ax], s->stream));
    cur[ax] = I.ax[ax].n;
    src = dst;
  }
  // src == b: the integrated w; c M3 U into a, then R3 = c M3 U - b
  // (a holds the n^3 partial products; its first nn entries are free now)
  double* t0 = a;
  double* t1 = a + nn;
  HIPCHK(s, launch_field_band(s->U3, t0, dims, 0, I.ax[0].Mb, dims[0], I.ax[0].B, s->stream));
  HIPCHK(s, launch_field_band(t0, t1, dims, 1, I.ax[1].Mb, dims[1], I.ax[1].B, s->stream));
  HIPCHK(s, launch_field_band(t1, t0, dims, 2, I.ax[2].Mb, dims[2], I.ax[2].B, s->stream));
  HIPCHK(s, launch_field_axpby(s->R3, t0, b, s->c, nn, s->stream));
  if (energy) {
    // gradient part: sum_d U . (K_d (x) M_e (x) M_f) U
    double grad = 0.0;
    const int64_t np2 = field_partials(nn);
    std::vector<double> part((size_t)np2);
    for (int d = 0; d < 3; ++d) {
      const double* in = s->U3;
      double* bufs[2] = {t0, t1};
      for (int ax = 0; ax < 3; ++ax) {
        double* out = bufs[ax % 2];
        HIPCHK(s, launch_field_band(in, out, dims, ax, ax == d ? I.ax[ax].Kb : I.ax[ax].Mb, dims[ax],
                                    I.ax[ax].B, s->stream));
        in = out;
      }
      HIPCHK(s, launch_field_dot(s->U3, in, nn, s->energy_partial, s->stream));
      HIPCHK(s, hipMemcpyAsync(part.data(), s->energy_partial, sizeof(double) * np2, hipMemcpyDeviceToHost,
                               s->stream));
      HIPCHK(s, hipStreamSynchronize(s->stream));
      double g = 0.0;
      for (double v : part) g += v;
      grad += g;
    }
    s->energy_field = quart + 0.5 * s->kappa * grad;
  }
  return CTD_OK;
}

// Full CFE step of the adaptive algorithm in 3D: u^{k+1} of the tensor-
// product system (c M3 + lam (K_0 (x) M (x) M + M (x) K_1 (x) M + M (x) M (x)
// K_2)) u = R3, exactly, in the eigenbases of (K_d, M_d):
//   U' = (V_0 (x) V_1 (x) V_2) [((V_0 (x) V_1 (x) V_2)^T R3) / (c + lam (mu_0i + mu_1j + mu_2k))].
// From a separated u^k its field is formed first (and R3 from it); a field
// state's R3 is the step's own.  The result is the new field state.
int full_step_3d(ctd_solver* s) {
  const DevInst& I = s->I;
  int dims[3] = {I.ax[0].n, I.ax[1].n, I.ax[2].n};
  if (!s->field3) {
    DevInst V = s->I;
    for (int d = 0; d < 3; ++d) V.ax[d].X = s->I.ax[d].Xk;
    V.sn = s->I.sk;
    HIPCHK(s, launch_reconstruct(V, s->Mk, s->U3, CTD_DTYPE_F64, s->stream));
    int rc = field_rhs(s, false);
    if (rc) return rc;
  }
  double* a = s->G3a;
  double* b = s->G3b;
  const double n3 = (double)dims[0] * dims[1] * dims[2];
  const double fl = 2.0 * n3 * (dims[0] + dims[1] + dims[2]);
  LAUNCH(s, CTD_K_FULL_SOLVE, fl, 8.0 * n3 * 2, launch_field_eig(s->R3, a, dims, 0, I.ax[0].fdV, 1, s->stream));
  LAUNCH(s, CTD_K_FULL_SOLVE, 0.0, 0.0, launch_field_eig(a, b, dims, 1, I.ax[1].fdV, 1, s->stream));
  LAUNCH(s, CTD_K_FULL_SOLVE, 0.0, 0.0, launch_field_eig(b, a, dims, 2, I.ax[2].fdV, 1, s->stream));
  HIPCHK(s, launch_field_fd_div(a, dims, I.ax[0].fdmu, I.ax[1].fdmu, I.ax[2].fdmu, s->c, s->lam, s->stream));
  LAUNCH(s, CTD_K_FULL_SOLVE, fl, 8.0 * n3 * 2, launch_field_eig(a, b, dims, 0, I.ax[0].fdV, 0, s->stream));
  LAUNCH(s, CTD_K_FULL_SOLVE, 0.0, 0.0, launch_field_eig(b, a, dims, 1, I.ax[1].fdV, 0, s->stream));
  LAUNCH(s, CTD_K_FULL_SOLVE, 0.0, 0.0, launch_field_eig(a, s->U3, dims, 2, I.ax[2].fdV, 0, s->stream));
  s->field3 = true;
  return CTD_OK;
}

// Full CFE step of the adaptive algorithm (2D): u^{k+1} of the tensor-product
// system from u^k, exactly, in the eigenbases of (K_d, M_d):
//   Q = c M_0 U^k M_1 - M_xy,   U' = V_0 [(V_0^T Q V_1) / (c + lam (mu_0i + mu_1j))] V_1^T,
// written as the new modes: X_0 = U' (column j = mode j), X_1 = identity,
// amplitudes 1.  u^k (X^k, M X^k, sigma^k, M_xy) is read, not modified.
int full_step_2d(ctd_solver* s) {
  DevInst& I = s->I;
  const int n0 = I.ax[0].n, n1 = I.ax[1].n, M = s->Mk;
  double* Q = s->fsQ;
  double* T = s->fsT;
  const double bytes_nn = 8.0 * n0 * n1;
  auto run = [&](const GemmArgs& g) -> int {
    LAUNCH(s, CTD_K_FULL_SOLVE, 2.0 * g.m * g.n * (double)g.K,
           8.0 * ((double)g.m * g.K + (double)g.K * g.n) + bytes_nn, launch_gemm64(g, s->stream));
    return CTD_OK;
  };
  int rc;
  {
    // Q = c (M_0 X^k_0) diag(sigma^k) (M_1 X^k_1)^T - M_xy   (row-major n0 x n1)
    GemmArgs g;
    g.m = n0; g.n = n1; g.K = M; g.epi = kEpiAxpby;
    g.A = I.ax[0].MXk; g.a_i = 1; g.a_k = n0;
    g.B = I.ax[1].MXk; g.b_k = n1; g.b_j = 1;
    g.ks = I.sk;
    g.C = Q; g.c_i = n1; g.c_j = 1;
    g.alpha = s->c; g.D = I.Mxy; g.d_f32 = I.mixed; g.d_i = n1; g.d_j = 1;
    if ((rc = run(g))) return rc;
  }
  {
    // T = V_0^T Q
    GemmArgs g;
    g.m = n0; g.n = n1; g.K = n0;
    g.A = I.ax[0].fdV; g.a_i = 1; g.a_k = n0;
    g.B = Q; g.b_k = n1; g.b_j = 1;
    g.C = T; g.c_i = n1; g.c_j = 1;
    if ((rc = run(g))) return rc;
  }
  {
    // Q = (T V_1) / (c + lam (mu_0i + mu_1j))
    GemmArgs g;
    g.m = n0; g.n = n1; g.K = n1; g.epi = kEpiFdDiv;
    g.A = T; g.a_i = n1; g.a_k = 1;
    g.B = I.ax[1].fdV; g.b_k = n1; g.b_j = 1;
    g.C = Q; g.c_i = n1; g.c_j = 1;
    g.mu0 = I.ax[0].fdmu; g.mu1 = I.ax[1].fdmu; g.c = s->c; g.lam = s->lam;
    if ((rc = run(g))) return rc;
  }
  {
    // T = V_0 Q
    GemmArgs g;
    g.m = n0; g.n = n1; g.K = n0;
    g.A = I.ax[0].fdV; g.a_i = n0; g.a_k = 1;
    g.B = Q; g.b_k = n1; g.b_j = 1;
    g.C = T; g.c_i = n1; g.c_j = 1;
    if ((rc = run(g))) return rc;
  }
  {
    // X_0 = T V_1^T, column-major n0 x n1: column j is mode j
    GemmArgs g;
    g.m = n0; g.n = n1; g.K = n1;
    g.A = T; g.a_i = n1; g.a_k = 1;
    g.B = I.ax[1].fdV; g.b_k = 1; g.b_j = n1;
    g.C = I.ax[0].X; g.c_i = 1; g.c_j = n0;
    if ((rc = run(g))) return rc;
  }
  HIPCHK(s, launch_unit_columns(I.ax[1].X, n1, n1, s->stream));
  HIPCHK(s, launch_fill(I.sn, n1, 1.0, s->stream));
  for (int d = 0; d < 2; ++d) {
    HIPCHK(s, launch_band_mv(I.ax[d], I.ax[d].Mb, I.ax[d].X, I.ax[d].MX, n1, s->stream));
    HIPCHK(s, launch_band_mv(I.ax[d], I.ax[d].Kb, I.ax[d].X, I.ax[d].KX, n1, s->stream));
  }
  return CTD_OK;
}

int one_step(ctd_solver* s, const int32_t* replay, int replay_len, ctd_step_info* info,
             std::vector<int32_t>& log, bool full_replay = false) {
  auto t0 = std::chrono::steady_clock::now();
  const int D = s->dim;
  const bool adaptive = replay == nullptr && !full_replay;
  const int max_modes = adaptive ? s->P.max_modes : replay_len;
  if (!adaptive && replay_len > s->Mcap) return s->fail(CTD_EINVAL, "replay needs more modes than allocated");
  const int warm = s->P.init_mode == CTD_INIT_WARM;
  int M = 0, sweeps = 0, unconv = 0, zero = 0, capped = 0;
  double last_term = 0.0;
  std::vector<int32_t> iters;
  for (int mode = 0; mode < (full_replay ? 0 : max_modes); ++mode) {
    HIPCHK(s, launch_reset_scalars(s->I, s->stream));
    HIPCHK(s, launch_init_mode(s->I, s->step_index, mode, warm, s->stream));
    HIPCHK(s, launch_finalize_init(s->I, s->stream));
    {
      // the initial guesses' Grams and Gauss-point values, every direction in one launch
      Work w{0.0, 0.0};
      for (int d = 0; d < D; ++d) {
        const Work wd = w_sig(s, d, M);
        w.flops += wd.flops;
        w.bytes += wd.bytes;
      }
      LAUNCH(s, CTD_K_SIGNATURE, w.flops, w.bytes, launch_signature_all(s->I, M, s->stream));
    }
    if (D == 3) {
      int rc = cubic_after(s, 1, -1);
      if (rc) return rc;
      rc = cubic_after(s, 2, 0);
      if (rc) return rc;
    }
    const int nsw = adaptive ? std::max(1, s->P.fp_max_iter) : replay[mode];
    if (nsw < 1) return s->fail(CTD_EINVAL, "replayed sweep count must be >= 1");
    // one sweep: every direction's load, right-hand side and solve, and the
    // Grams of every direction but the last
    auto sweep = [&](int it) -> int {
      for (int d = 0; d < D; ++d) {
        if (D == 3 && !s->field3) {
          Work w = w_cubic(s, d);
          LAUNCH(s, CTD_K_CUBIC_H, w.flops, w.bytes, launch_cubic_h(s->I, d, s->stream));
        }
        {
          // 2D: the M_xy product is part of the RHS launch
          Work w = w_rhs(s, d, M);
          if (D == 2) {
            const Work wg = w_load2d(s, d);
            w.flops += wg.flops;
            w.bytes += wg.bytes;
          }
          LAUNCH(s, CTD_K_RHS, w.flops, w.bytes, launch_rhs(s->I, d, M, s->stream));
          Work ws = w_solve(s, d);
          if (s->use_fd[d]) {
            // the normalisation and the fresh factor's Grams in one launch
            LAUNCH(s, CTD_K_SOLVE, ws.flops, ws.bytes, launch_solve_fd(s->I, d, M, s->stream));
            Work wg = w_sig(s, d, M);
            LAUNCH(s, CTD_K_FINALIZE, wg.flops, wg.bytes, launch_finalize_sig(s->I, d, it, M, s->stream, kFdKb));
          } else {
            LAUNCH(s, CTD_K_SOLVE, ws.flops, ws.bytes, launch_solve_bcr(s->I, d, it, M, s->stream));
          }
        }
        if (d < D - 1) {
          if (!s->use_fd[d]) {
            Work w = w_sig(s, d, M);
            LAUNCH(s, CTD_K_SIGNATURE, w.flops, w.bytes, launch_signature(s->I, d, M, s->stream));
          }
          int rc = cubic_after(s, d, d + 1);
          if (rc) return rc;
        }
      }
      return CTD_OK;
    };
    // the start of a further sweep: the last direction's Grams (unless its
    // normalisation launch made them) and the cubic Grams
    auto carry = [&]() -> int {
      if (!s->use_fd[D - 1]) {
        Work w = w_sig(s, D - 1, M);
        LAUNCH(s, CTD_K_SIGNATURE, w.flops, w.bytes, launch_signature(s->I, D - 1, M, s->stream));
      }
      return cubic_after(s, D - 1, 0);
    };
    // Adaptive: sweep it + 1 is enqueued before the host waits for the
    // scalars of sweep it, its launches marked to return at once on the
    // device if sweep it ended the mode (the finalisation of the last
    // direction records that, with the host's own test), so the device keeps
    // working while the host reads and decides.  The decisions and the
    // arithmetic of every sweep that runs are those of the plain sequence.
    s->I.spec_nsw = adaptive ? nsw : 0;
    int it = 0;
    bool conv = false;
    bool queued = false;   // sweep it was enqueued speculatively
    int rc = CTD_OK;
    for (it = 1; it <= nsw; ++it) {
      if (!queued && (rc = sweep(it))) break;
      queued = false;
      bool last = it == nsw;
      if (adaptive) {
        DevScalars* slot = s->sc_host + (it & 1);
        HIPCHK(s, hipMemcpyAsync(slot, s->I.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipEventRecord(s->sc_ev[it & 1], s->stream));
        if (it < nsw) {
          s->I.spec_check = 1;
          s->prof.tag = ++s->spec_serial;
          rc = carry();
          if (rc == CTD_OK) rc = sweep(it + 1);
          s->I.spec_check = 0;
          s->prof.tag = 0;
          if (rc) break;
          queued = true;
        }
        HIPCHK(s, hipEventSynchronize(s->sc_ev[it & 1]));
        if (slot != s->sc_host) s->sc_host[0] = *slot;
        // a zero amplitude ends the mode (Sec. 3.3 stopping) before the
        // non-finite test: the directions solved after it in the same sweep
        // see zero fixed factors and produce NaN for a mode that is dropped
        if (s->sc_host->zero) {
          zero = 1;
          if (queued) s->prof.skipped(s->spec_serial);
          break;
        }
        if (s->sc_host->nonfinite) { rc = s->fail(CTD_ENONFINITE, "non-finite mode amplitude"); break; }
        conv = s->sc_host->converged != 0 && it >= 2;
        if (conv) last = true;
      }
      if (last) {
        if (queued) s->prof.skipped(s->spec_serial);
        break;
      }
      if (!queued && (rc = carry())) break;
    }
    s->I.spec_nsw = 0;
    s->I.spec_check = 0;
    s->prof.tag = 0;
    if (rc) return rc;
    if (zero) break;
    if (it > nsw) it = nsw;
    sweeps += it;
    if (adaptive && !conv) ++unconv;
    HIPCHK(s, launch_append(s->I, M, s->stream));
    ++M;
    iters.push_back(it);
    if (adaptive) {
      // enrichment decision from the scalars of the last sweep
      double pu = 1.0;
      for (int d = 0; d < D; ++d) pu *= s->sc_host->umax[d];
      last_term = s->sc_host->sigma[D - 1] * pu;
      if (last_term <= s->P.enrich_tol) break;
      if (M >= s->P.max_modes) { capped = 1; break; }
    }
  }
  if (!adaptive && !full_replay) {
    int rc = read_scalars(s);
    if (rc) return rc;
    if (s->sc_host->nonfinite) return s->fail(CTD_ENONFINITE, "non-finite mode amplitude");
    last_term = M > 0 ? s->sc_host->term_max : 0.0;
  }
  // adaptive algorithm: a step that needs more than M_c modes is the full solve
  const bool full = full_replay || (s->actd && capped);
  if (full && D == 3) {
    int rc = full_step_3d(s);
    if (rc) return rc;
    M = 0;
  } else if (full) {
    int rc = full_step_2d(s);
    if (rc) return rc;
    M = s->ax[1].n;
  } else {
    s->field3 = false;   // a CTD step's u^{k+1} is separated
  }
  int rc = finish_step(s, M);   // M == 0: the zero field
  if (rc) return rc;
  ++s->step_index;
  if (full) {
    log.push_back(-1);
  } else {
    log.push_back(M);
    for (int v : iters) log.push_back(v);
  }
  if (info) {
    info->full_solve = full ? 1 : 0;
    info->modes = M;
    info->sweeps = sweeps;
    info->capped = capped;
    info->fp_unconverged = unconv;
    info->zero_mode = zero;
    info->last_term_max = last_term;
    info->energy = std::numeric_limits<double>::quiet_NaN();
    info->energy_increase = 0;
    // energy stability of the scheme needs alpha >= max(w')/2 = 4 a0 on
    // |u| <= 1 (Sec. 2.5); below it the step still runs, flagged
    info->stability_warning = s->alpha < 4.0 * s->a0 ? 1 : 0;
  }
  if (s->P.energy_each_step) {
    double E;
    rc = energy_of_uk(s, &E);
    if (rc) return rc;
    if (info) {
      info->energy = E;
      info->energy_increase = std::isfinite(s->energy_prev) && E > s->energy_prev * (1.0 + 1e-12) + 1e-300;
    }
    s->energy_prev = E;
  } else {
    HIPCHK(s, sync_collect(s));
  }
  if (info) {
    auto t1 = std::chrono::steady_clock::now();
    info->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  return CTD_OK;
}

// ---------------------------------------------------------------- lockstep
// Many 2D instances advanced together: every round, the instances that start
// a mode run its initialisation launches together (multi-instance launches),
// then every instance in a mode runs one sweep together, and one read-back
// of all instances' scalars feeds each instance's own decisions (the same
// decisions, in the same order, as one_step's adaptive schedule).  Steps end
// per instance (finish_step, energy) with that instance's own launches.  The
// arithmetic of every instance is that of its standalone launches: results
// are identical to ctd_step on the instance alone.
struct LockstepInst {
  ctd_solver* s = nullptr;
  int M = 0, mode = 0, it = 1, sweeps = 0, unconv = 0, zero = 0, capped = 0;
  int steps_done = 0;
  bool pending_append = false;   // appended mode's kernel goes with the next launch group
  bool start = true;             // the next round initialises a mode
  bool done = false;
  double last_term = 0.0;
  std::vector<int32_t> iters;
  std::chrono::steady_clock::time_point t0;
};

// sync = false (no energy to read back): the step-end launches stay in flight
// on the instance's stream; the caller waits for them by an event.
int lockstep_finish(LockstepInst& L, ctd_step_info* info, std::vector<int32_t>& log, bool sync = true) {
  ctd_solver* s = L.s;
  if (L.pending_append) {
    HIPCHK(s, launch_append(s->I, L.M - 1, s->stream));
    L.pending_append = false;
  }
  int rc = finish_step(s, L.M);
  if (rc) return rc;
  ++s->step_index;
  log.push_back(L.M);
  for (int v : L.iters) log.push_back(v);
  if (info) {
    info->full_solve = 0;
    info->modes = L.M;
    info->sweeps = L.sweeps;
    info->capped = L.capped;
    info->fp_unconverged = L.unconv;
    info->zero_mode = L.zero;
    info->last_term_max = L.last_term;
    info->energy = std::numeric_limits<double>::quiet_NaN();
    info->energy_increase = 0;
    info->stability_warning = s->alpha < 4.0 * s->a0 ? 1 : 0;
  }
  if (s->P.energy_each_step) {
    double E;
    rc = energy_of_uk(s, &E);
    if (rc) return rc;
    if (info) {
      info->energy = E;
      info->energy_increase = std::isfinite(s->energy_prev) && E > s->energy_prev * (1.0 + 1e-12) + 1e-300;
    }
    s->energy_prev = E;
  } else if (sync) {
    HIPCHK(s, sync_collect(s));
  }
  if (info) {
    auto t1 = std::chrono::steady_clock::now();
    info->ms = std::chrono::duration<double, std::milli>(t1 - L.t0).count();
  }
  // next step from mode 0
  L.M = 0; L.mode = 0; L.it = 1; L.sweeps = 0; L.unconv = 0; L.zero = 0; L.capped = 0;
  L.last_term = 0.0;
  L.iters.clear();
  L.start = true;
  ++L.steps_done;
  L.t0 = std::chrono::steady_clock::now();
  return CTD_OK;
}

}  // namespace

namespace ctd {

bool lockstep_eligible(const ctd_solver* s) {
  return s->dim == 2 && s->P.schedule == CTD_SCHED_ADAPTIVE && !s->actd && !s->use_fd[0] &&
         !s->use_fd[1] && s->ax[0].B == s->ax[1].B;
}

int band_halfwidth(const ctd_solver* s) { return s->ax[0].B; }

// ------------------------------------------------------------ engine
struct Lockstep::Impl {
  hipStream_t st = nullptr;
  int B = 0;                         // band half-width shared by the instances
  int cap = 0;                       // slots of the device and pinned arrays
  DevInst* dI = nullptr;
  LsArg* dA = nullptr;
  DevScalars* dS = nullptr;
  DevInst* hI = nullptr;
  LsArg* hA = nullptr;
  DevScalars* hS = nullptr;
  std::vector<ctd_solver*> S;        // per slot (nullptr: free)
  std::vector<LockstepInst> L;
  std::vector<int> remaining;        // steps still to run per slot
  std::vector<std::vector<int32_t>> logs;
  int live = 0;
  // step-end work (append, swap, the next step's tables and M_xy) runs on
  // side streams while the other instances go on; an instance rejoins the
  // rounds once its event has completed
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  int next_side = 0;
  std::vector<hipEvent_t> ev;        // per slot
  std::vector<char> pending;         // per slot: step-end work in flight

  hipError_t sync() { return hipStreamSynchronize(st); }
  void release() {
    (void)sync();
    for (hipStream_t h : side)
      if (h) (void)hipStreamSynchronize(h);
    if (dI) (void)hipFree(dI);
    if (dA) (void)hipFree(dA);
    if (dS) (void)hipFree(dS);
    if (hI) (void)hipHostFree(hI);
    if (hA) (void)hipHostFree(hA);
    if (hS) (void)hipHostFree(hS);
    dI = nullptr; dA = nullptr; dS = nullptr; hI = nullptr; hA = nullptr; hS = nullptr;
  }
  // grow the arrays to `want` slots (the instances in use are re-uploaded)
  hipError_t grow(int want) {
    hipError_t e = sync();
    if (e != hipSuccess) return e;
    DevInst *nI = nullptr, *nhI = nullptr;
    LsArg *nA = nullptr, *nhA = nullptr;
    DevScalars *nS = nullptr, *nhS = nullptr;
    if ((e = hipMalloc(&nI, sizeof(DevInst) * want)) != hipSuccess ||
        (e = hipMalloc(&nA, sizeof(LsArg) * 4 * want)) != hipSuccess ||
        (e = hipMalloc(&nS, sizeof(DevScalars) * want)) != hipSuccess ||
        (e = hipHostMalloc(&nhI, sizeof(DevInst) * want, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc(&nhA, sizeof(LsArg) * 4 * want, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc(&nhS, sizeof(DevScalars) * want, hipHostMallocDefault)) != hipSuccess) {
      if (nI) (void)hipFree(nI);
      if (nA) (void)hipFree(nA);
      if (nS) (void)hipFree(nS);
      if (nhI) (void)hipHostFree(nhI);
      if (nhA) (void)hipHostFree(nhA);
      if (nhS) (void)hipHostFree(nhS);
      return e;
    }
    if (cap) std::memcpy(nhI, hI, sizeof(DevInst) * cap);
    release();
    dI = nI; dA = nA; dS = nS; hI = nhI; hA = nhA; hS = nhS;
    S.resize(want, nullptr);
    L.resize(want);
    remaining.resize(want, 0);
    logs.resize(want);
    ev.resize(want, nullptr);
    pending.resize(want, 0);
    cap = want;
    for (int i = 0; i < cap; ++i)
      if (S[i] && (e = hipMemcpyAsync(dI + i, hI + i, sizeof(DevInst), hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    return hipSuccess;
  }
  hipError_t upload(int i) {
    update_view(S[i]);
    hI[i] = S[i]->I;
    return hipMemcpyAsync(dI + i, hI + i, sizeof(DevInst), hipMemcpyHostToDevice, st);
  }
};

Lockstep::Lockstep(hipStream_t st) : p(new Impl) { p->st = st; }

Lockstep::~Lockstep() {
  p->release();
  // instances still in their step-end work go back to the engine's stream
  // (the side streams end here)
  for (int i = 0; i < p->cap; ++i)
    if (p->S[i] && p->pending[i]) solver_bind_stream(p->S[i], p->st);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t h : p->side)
    if (h) (void)hipStreamDestroy(h);
  delete p;
}

bool Lockstep::empty() const { return p->live == 0; }

int Lockstep::band() const { return p->B; }

int Lockstep::add(ctd_solver* s, int nsteps, int* slot, std::string& err) {
  if (!lockstep_eligible(s)) {
    err = "lockstep needs a 2D adaptive instance with cyclic-reduction solves";
    return CTD_EUNSUPPORTED;
  }
  if (p->live > 0 && s->ax[0].B != p->B) {
    err = "lockstep instances must share one band width";
    return CTD_EUNSUPPORTED;
  }
  if (nsteps < 1) {
    err = "lockstep needs at least one step";
    return CTD_EINVAL;
  }
  int i = 0;
  while (i < p->cap && p->S[i]) ++i;
  if (i == p->cap) {
    hipError_t e = p->grow(std::max(16, 2 * p->cap));
    if (e != hipSuccess) {
      err = std::string("HIP error in lockstep arrays: ") + hipGetErrorString(e);
      return e == hipErrorOutOfMemory ? CTD_ENOMEM : CTD_EDEVICE;
    }
  }
  p->B = s->ax[0].B;
  solver_bind_stream(s, p->st);
  p->S[i] = s;
  p->L[i] = LockstepInst{};
  p->L[i].s = s;
  p->L[i].t0 = std::chrono::steady_clock::now();
  p->remaining[i] = nsteps;
  p->logs[i].clear();
  ++p->live;
  hipError_t e = p->upload(i);
  if (e != hipSuccess) {
    err = std::string("HIP error in lockstep upload: ") + hipGetErrorString(e);
    return CTD_EDEVICE;
  }
  *slot = i;
  return CTD_OK;
}

int Lockstep::round(std::vector<std::pair<int, ctd_step_info>>& steps, std::vector<int>& finished,
                    std::string& err, std::vector<std::pair<int, int>>* failed) {
  Impl& E = *p;
  if (E.live == 0) return CTD_OK;
  hipStream_t st = E.st;
  const int B = E.B;
  const int N = E.cap;
  // instances whose step-end work has completed rejoin (or leave, when all
  // their steps are done); with every instance still busy, wait for one
  {
    int active = 0, first_busy = -1;
    for (int i = 0; i < N; ++i) {
      if (!E.S[i]) continue;
      if (E.pending[i]) {
        hipError_t q = hipEventQuery(E.ev[i]);
        if (q == hipErrorNotReady) {
          if (first_busy < 0) first_busy = i;
          continue;
        }
        if (q != hipSuccess) {
          err = std::string("HIP error in lockstep step end: ") + hipGetErrorString(q);
          return CTD_EDEVICE;
        }
        E.pending[i] = 0;
        solver_bind_stream(E.S[i], st);
        if (E.remaining[i] == 0) {
          E.S[i]->decisions_last.swap(E.logs[i]);
          E.logs[i].clear();
          E.S[i] = nullptr;
          --E.live;
          finished.push_back(i);
          continue;
        }
      }
      ++active;
    }
    if (active == 0) {
      if (first_busy >= 0) {
        hipError_t e = hipEventSynchronize(E.ev[first_busy]);
        if (e != hipSuccess) {
          err = std::string("HIP error in lockstep step end: ") + hipGetErrorString(e);
          return CTD_EDEVICE;
        }
      }
      return CTD_OK;
    }
  }
  auto hip = [&](hipError_t e, const char* where) {
    if (e == hipSuccess) return CTD_OK;
    err = std::string("HIP error in ") + where + ": " + hipGetErrorString(e);
    return CTD_EDEVICE;
  };
  auto fill = [&](LsArg& a, int i) {
    const ctd_solver* s = E.S[i];
    a.inst = i;
    a.M = E.L[i].M;
    a.sweep = E.L[i].it;
    a.mode = E.L[i].mode;
    a.warm = s->P.init_mode == CTD_INIT_WARM;
    a.nlin = (s->Mk + 2 * E.L[i].M + 63) / 64;
    for (int d = 0; d < 2; ++d) a.nld[d] = (s->ax[1 - d].n + 63) / 64;
    a.step = s->step_index;
  };
  // workgroup size of an instance's own initial-guess finalisation
  auto finalize_threads = [&](int i) {
    const int n = std::max(E.S[i]->ax[0].n, E.S[i]->ax[1].n);
    return n >= 1024 ? 1024 : (n + 63) / 64 * 64;
  };
  // groups of this round; the initialisation group ordered by its
  // finalisation workgroup size (one launch per size)
  std::vector<int> gi, gs;
  for (int i = 0; i < N; ++i) {
    if (!E.S[i] || E.pending[i]) continue;
    if (E.L[i].start) gi.push_back(i);
    gs.push_back(i);
  }
  std::stable_sort(gi.begin(), gi.end(),
                   [&](int a, int b) { return finalize_threads(a) < finalize_threads(b); });
  const int ni = (int)gi.size(), ns = (int)gs.size();
  LsArg* hAi = E.hA;
  LsArg* hAs = E.hA + N;
  for (int k = 0; k < ni; ++k) { fill(hAi[k], gi[k]); hAi[k].flag = E.L[gi[k]].pending_append ? 1 : 0; }
  for (int k = 0; k < ns; ++k) { fill(hAs[k], gs[k]); hAs[k].flag = E.L[gs[k]].it > 1 ? 1 : 0; }
  // the RHS launches' workgroups, packed entry after entry per direction
  int nblk[2] = {0, 0};
  for (int k = 0; k < ns; ++k)
    for (int d = 0; d < 2; ++d) {
      hAs[k].boff[d] = nblk[d];
      nblk[d] += ((E.S[gs[k]]->ax[d].n + 63) / 64) * (hAs[k].nlin + hAs[k].nld[d]);
    }
  // the solve launches: sweep entries regrouped per direction by BCR
  // storage class and thread count (blocks [2N, 3N) and [3N, 4N))
  struct SolveClass { int mode, threads, first, count; size_t shm; };
  std::vector<SolveClass> scls[2];
  for (int d = 0; d < 2; ++d) {
    std::map<std::pair<int, int>, std::vector<int>> cls;
    std::map<std::pair<int, int>, size_t> shm;
    for (int k = 0; k < ns; ++k) {
      int mode, threads;
      size_t sh;
      bcr_launch_class(E.S[gs[k]]->ax[d].n, B, mode, threads, sh);
      cls[{mode, threads}].push_back(k);
      shm[{mode, threads}] = std::max(shm[{mode, threads}], sh);
    }
    LsArg* dst = E.hA + (2 + d) * N;
    int at = 0;
    for (auto& kv : cls) {
      scls[d].push_back({kv.first.first, kv.first.second, at, (int)kv.second.size(), shm[kv.first]});
      for (int k : kv.second) dst[at++] = hAs[k];
    }
  }
  DevInst* dI = E.dI;
  LsArg* dA = E.dA;
  int rc = CTD_OK;
  if ((rc = hip(hipMemcpyAsync(dA, E.hA, sizeof(LsArg) * 4 * N, hipMemcpyHostToDevice, st), "lockstep args")))
    return rc;
  LsArg* dAi = dA;
  LsArg* dAs = dA + N;
  auto grid_of = [&](const std::vector<int>& g, const LsArg* a, int d) {
    LsGrid G;
    G.B = B;
    for (size_t k = 0; k < g.size(); ++k) {
      const ctd_solver* s = E.S[g[k]];
      const int n = d < 0 ? std::max(s->ax[0].n, s->ax[1].n) : s->ax[d].n;
      G.nmax = std::max(G.nmax, n);
      G.ndot = std::max(G.ndot, (2 * a[k].M + s->Mk + 3) / 4);
      if (d >= 0) G.nchunk = std::max(G.nchunk, a[k].nlin + a[k].nld[d]);
    }
    G.ndot = std::max(G.ndot, 1);
    return G;
  };
  // mode initialisation (after the append of the previous mode)
  if (ni > 0) {
    const LsGrid G = grid_of(gi, hAi, -1);
    if ((rc = hip(launch_multi(kLsAppend, dI, dAi, ni, G, st), "append")) ||
        (rc = hip(launch_multi(kLsReset, dI, dAi, ni, G, st), "reset")) ||
        (rc = hip(launch_multi(kLsInit, dI, dAi, ni, G, st), "init")))
      return rc;
    for (int k0 = 0; k0 < ni;) {
      int k1 = k0;
      LsGrid Gf;
      Gf.B = B;
      Gf.threads = finalize_threads(gi[k0]);
      while (k1 < ni && finalize_threads(gi[k1]) == Gf.threads) {
        Gf.nmax = std::max(Gf.nmax, std::max(E.S[gi[k1]]->ax[0].n, E.S[gi[k1]]->ax[1].n));
        ++k1;
      }
      if ((rc = hip(launch_multi(kLsFinalizeInit, dI, dAi + k0, k1 - k0, Gf, st), "finalize"))) return rc;
      k0 = k1;
    }
    if ((rc = hip(launch_multi(kLsSignatureAll, dI, dAi, ni, G, st), "signature"))) return rc;
    for (int i : gi) { E.L[i].pending_append = false; E.L[i].start = false; }
  }
  // one sweep of every instance in a mode: the signature of the last
  // direction (continued sweeps only), then per direction RHS and solve,
  // and the signature of every direction but the last
  {
    LsGrid G1 = grid_of(gs, hAs, 1);
    if ((rc = hip(launch_multi(kLsSignatureFlag, dI, dAs, ns, G1, st, 1), "signature"))) return rc;
    for (int d = 0; d < 2; ++d) {
      LsGrid G = grid_of(gs, hAs, d);
      G.nblk = nblk[d];
      if ((rc = hip(launch_multi(kLsRhs, dI, dAs, ns, G, st, d), "rhs"))) return rc;
      // the solve: one launch per BCR storage class and thread count
      for (const SolveClass& c : scls[d]) {
        LsGrid G2;
        G2.B = B;
        G2.mode = c.mode;
        G2.threads = c.threads;
        G2.shm = c.shm;
        if ((rc = hip(launch_multi(kLsSolve, dI, dA + (2 + d) * N + c.first, c.count, G2, st, d), "solve")))
          return rc;
      }
      if (d == 0) {
        const LsGrid G0 = grid_of(gs, hAs, 0);
        if ((rc = hip(launch_multi(kLsSignature, dI, dAs, ns, G0, st, 0), "signature"))) return rc;
      }
    }
  }
  // one read-back of every instance's scalars
  if ((rc = hip(launch_multi(kLsGather, dI, dAs, ns, LsGrid{}, st, 0, E.dS), "gather")) ||
      (rc = hip(hipMemcpyAsync(E.hS, E.dS, sizeof(DevScalars) * ns, hipMemcpyDeviceToHost, st), "gather")) ||
      (rc = hip(hipStreamSynchronize(st), "gather")))
    return rc;
  // decisions, as one_step takes them
  for (int k = 0; k < ns; ++k) {
    const int i = gs[k];
    LockstepInst& Li = E.L[i];
    ctd_solver* s = E.S[i];
    const DevScalars& sc = E.hS[k];
    const int nsw = std::max(1, s->P.fp_max_iter);
    bool end_step = false;
    // an instance that fails leaves the engine (failed != nullptr) or ends
    // the round with its error
    auto fail_inst = [&](int code, const std::string& msg) -> int {
      err = msg;
      if (!failed) return code;
      failed->push_back({i, code});
      E.logs[i].clear();
      E.S[i] = nullptr;
      --E.live;
      return CTD_OK;
    };
    if (sc.zero) {
      Li.zero = 1;
      end_step = true;
    } else {
      if (sc.nonfinite) {
        s->err = "non-finite mode amplitude";
        if ((rc = fail_inst(CTD_ENONFINITE, s->err))) return rc;
        continue;
      }
      const bool conv = sc.converged != 0 && Li.it >= 2;
      const bool last = Li.it == nsw || conv;
      if (!last) {
        ++Li.it;
        continue;
      }
      Li.sweeps += Li.it;
      if (!conv) ++Li.unconv;
      ++Li.M;
      Li.iters.push_back(Li.it);
      Li.pending_append = true;
      double pu = 1.0;
      for (int d = 0; d < 2; ++d) pu *= sc.umax[d];
      Li.last_term = sc.sigma[1] * pu;
      if (Li.last_term <= s->P.enrich_tol) {
        end_step = true;
      } else if (Li.M >= s->P.max_modes) {
        Li.capped = 1;
        end_step = true;
      } else {
        ++Li.mode;
        Li.it = 1;
        Li.start = true;
      }
    }
    if (end_step) {
      ctd_step_info inf{};
      // without an energy to read back, the step-end launches go to a side
      // stream and the instance sits out until they have completed
      const bool async = !s->P.energy_each_step;
      if (async) {
        hipStream_t& h = E.side[E.next_side];
        E.next_side = (E.next_side + 1) % Impl::kSide;
        if (!h && (rc = hip(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), "lockstep stream"))) return rc;
        if (!E.ev[i] && (rc = hip(hipEventCreateWithFlags(&E.ev[i], hipEventDisableTiming), "lockstep event")))
          return rc;
        solver_bind_stream(s, h);
      }
      rc = lockstep_finish(Li, &inf, E.logs[i], !async);
      if (rc == CTD_OK && async) rc = hip(hipEventRecord(E.ev[i], s->stream), "lockstep event");
      if (rc) {
        if (async) solver_bind_stream(s, st);
        if ((rc = fail_inst(rc, s->err))) return rc;
        continue;
      }
      steps.push_back({i, inf});
      --E.remaining[i];
      if (async) {
        E.pending[i] = 1;
        if (E.remaining[i] > 0 && (rc = hip(E.upload(i), "lockstep upload"))) return rc;
      } else if (E.remaining[i] == 0) {
        s->decisions_last.swap(E.logs[i]);
        E.logs[i].clear();
        E.S[i] = nullptr;
        --E.live;
        finished.push_back(i);
      } else if ((rc = hip(E.upload(i), "lockstep upload"))) {
        return rc;
      }
    }
  }
  return CTD_OK;
}

int lockstep_steps(std::vector<ctd_solver*>& S, int nsteps, ctd_step_info* info, hipStream_t st,
                   std::string& err) {
  const int N = (int)S.size();
  if (N == 0 || nsteps <= 0) return CTD_OK;
  Lockstep E(st);
  std::vector<int> slot_of(N), inst_of;
  int rc = CTD_OK;
  for (int i = 0; i < N && rc == CTD_OK; ++i) {
    int slot = -1;
    rc = E.add(S[i], nsteps, &slot, err);
    if (rc == CTD_OK) {
      slot_of[i] = slot;
      if ((int)inst_of.size() <= slot) inst_of.resize(slot + 1, -1);
      inst_of[slot] = i;
    }
  }
  std::vector<int> done_steps(N, 0);
  std::vector<std::pair<int, ctd_step_info>> steps;
  std::vector<int> finished;
  while (rc == CTD_OK && !E.empty()) {
    steps.clear();
    finished.clear();
    rc = E.round(steps, finished, err);
    for (auto& st_info : steps) {
      const int i = inst_of[st_info.first];
      if (info) info[(size_t)i * nsteps + done_steps[i]] = st_info.second;
      ++done_steps[i];
    }
  }
  return rc;
}

}  // namespace ctd

namespace {
}  // namespace

extern "C" {

int ctd_problem_default(ctd_problem* p) {
  if (!p) return CTD_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->abi_version = CTD_ABI_VERSION;
  p->dim = 2;
  for (int d = 0; d < 3; ++d) { p->nodes[d] = 64; p->lo[d] = 0.0; p->hi[d] = 1.0; }
  p->eps = 0.02; p->S = 2.0; p->dt = 1e-3;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  p->L = nan; p->kappa = nan; p->a0 = nan; p->alpha = nan;
  p->patch_s = 2; p->poly_p = 2; p->dilation_a = 12.0; p->gauss_points = 5;
  p->fp_max_iter = 20; p->fp_tol = 1e-2; p->enrich_tol = 1e-8; p->max_modes = 64;
  p->precision = CTD_PREC_FP64; p->schedule = CTD_SCHED_ADAPTIVE; p->init_mode = CTD_INIT_WARM;
  p->energy_each_step = 0; p->seed = 0;
  p->w_rank = 0; p->w_iters = 30;
  return CTD_OK;
}

int ctd_init(const ctd_problem* p, int32_t m0, const double* const* init,
             const double* amp, void* hip_stream, ctd_solver** out) {
  if (!out) { g_init_error = "out is NULL"; return CTD_EINVAL; }
  *out = nullptr;
  std::string err;
  int rc = validate(p, err);
  if (rc) { g_init_error = err; return rc; }
  if (m0 < 1 || !init) { g_init_error = "need m0 >= 1 initial modes"; return CTD_EINVAL; }
  {
    hipError_t ce = configure_kernels();
    if (ce != hipSuccess) { g_init_error = hipGetErrorString(ce); return CTD_EDEVICE; }
    if (p->dim == 3) {
      DevInst probe{};
      probe.mixed = p->precision == CTD_PREC_MIXED;
      probe.Mkp = std::max(kTile, round_up(std::max(p->max_modes, m0), kTile));
      if (cubic_h_lds_total(probe) > (size_t)max_lds_bytes()) {
        g_init_error = "max_modes exceeds the LDS-resident cubic evaluation of this precision";
        return CTD_EUNSUPPORTED;
      }
    }
  }
  for (int d = 0; d < p->dim; ++d)
    if (!init[d]) { g_init_error = "init factor pointer is NULL"; return CTD_EINVAL; }
  ctd_solver* s = new (std::nothrow) ctd_solver();
  if (!s) { g_init_error = "out of host memory"; return CTD_ENOMEM; }
  rc = setup_host(s, p, hip_stream, err);
  if (rc) { g_init_error = err; delete s; return rc; }
  rc = alloc_instance(s, m0);
  if (rc) {
    g_init_error = s->err;
    s->arena.release();
    if (s->sc_host) (void)hipHostFree(s->sc_host);
    for (hipEvent_t e : s->sc_ev)
      if (e) (void)hipEventDestroy(e);
    delete s;
    return rc;
  }
  // initial modes: fold amplitude signs into axis 0, |amp| into sk
  std::vector<double> sk(m0);
  std::vector<double> col;
  for (int d = 0; d < s->dim; ++d) {
    const size_t n = s->ax[d].n;
    std::vector<double> buf(init[d], init[d] + n * (size_t)m0);
    if (d == 0)
      for (int m = 0; m < m0; ++m) {
        double a = amp ? amp[m] : 1.0;
        if (a < 0) for (size_t i = 0; i < n; ++i) buf[(size_t)m * n + i] = -buf[(size_t)m * n + i];
      }
    hipError_t e = copy_sync(s, s->I.ax[d].Xk, buf.data(), sizeof(double) * n * m0, hipMemcpyHostToDevice);
    if (e != hipSuccess) { g_init_error = hipGetErrorString(e); ctd_destroy(s); return CTD_EDEVICE; }
  }
  for (int m = 0; m < m0; ++m) {
    double a = amp ? amp[m] : 1.0;
    if (!std::isfinite(a)) { g_init_error = "non-finite amplitude"; ctd_destroy(s); return CTD_EINVAL; }
    sk[m] = std::fabs(a);
  }
  hipError_t e = copy_sync(s, s->I.sk, sk.data(), sizeof(double) * m0, hipMemcpyHostToDevice);
  if (e != hipSuccess) { g_init_error = hipGetErrorString(e); ctd_destroy(s); return CTD_EDEVICE; }
  s->Mk = m0;
  for (int d = 0; d < s->dim; ++d) {
    e = launch_band_mv(s->I.ax[d], s->I.ax[d].Mb, s->I.ax[d].Xk, s->I.ax[d].MXk, m0, s->stream);
    if (e == hipSuccess) e = launch_band_mv(s->I.ax[d], s->I.ax[d].Kb, s->I.ax[d].Xk, s->KXk[d], m0, s->stream);
    if (e != hipSuccess) { g_init_error = hipGetErrorString(e); ctd_destroy(s); return CTD_EDEVICE; }
  }
  rc = precompute(s);
  if (rc == CTD_OK) {
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { s->err = hipGetErrorString(e); rc = CTD_EDEVICE; }
  }
  if (rc) { g_init_error = s->err; ctd_destroy(s); return rc; }
  *out = s;
  return CTD_OK;
}

int ctd_step(ctd_solver* s, int32_t nsteps, ctd_step_info* info) {
  if (!s) return CTD_EINVAL;
  if (nsteps < 0) return s->fail(CTD_EINVAL, "nsteps < 0");
  std::vector<int32_t> log;
  size_t pos = 0;
  const bool replay = s->P.schedule == CTD_SCHED_REPLAY;
  for (int k = 0; k < nsteps; ++k) {
    const int32_t* rp = nullptr;
    int rl = 0;
    bool full = false;
    if (replay) {
      if (pos >= s->decisions_next.size()) return s->fail(CTD_ESTATE, "replay log exhausted");
      rl = s->decisions_next[pos];
      if (rl == -1) {
        if (!s->actd) return s->fail(CTD_EINVAL, "replayed full solve needs actd");
        full = true;
        rl = 0;
        pos += 1;
      } else {
        // rl == 0: a step whose first mode had zero amplitude (u^{k+1} = 0)
        if (rl < 0 || pos + 1 + rl > s->decisions_next.size()) return s->fail(CTD_EINVAL, "malformed replay log");
        rp = s->decisions_next.data() + pos + 1;
        pos += 1 + rl;
      }
    }
    int rc = one_step(s, rp, rl, info ? info + k : nullptr, log, full);
    if (rc) return rc;
  }
  if (replay) s->decisions_next.erase(s->decisions_next.begin(), s->decisions_next.begin() + pos);
  s->decisions_last.swap(log);
  return CTD_OK;
}

int ctd_energy(ctd_solver* s, double* E) {
  if (!s || !E) return CTD_EINVAL;
  return energy_of_uk(s, E);
}

int ctd_reconstruct(ctd_solver* s, void* out, int32_t dtype, int32_t on_device,
                    const int64_t* strides) {
  if (!s || !out) return CTD_EINVAL;
  if (dtype != CTD_DTYPE_F64 && dtype != CTD_DTYPE_F32) return s->fail(CTD_EINVAL, "bad dtype");
  DevInst V = s->I;
  for (int d = 0; d < s->dim; ++d) V.ax[d].X = s->I.ax[d].Xk;
  V.sn = s->I.sk;
  int64_t n[3] = {1, 1, 1}, cst[3] = {0, 0, 0};
  for (int d = 0; d < s->dim; ++d) n[d] = s->ax[d].n;
  // C-order strides; a caller layout equal to them takes the direct path
  cst[s->dim - 1] = 1;
  for (int d = s->dim - 2; d >= 0; --d) cst[d] = cst[d + 1] * n[d + 1];
  bool contiguous = true;
  if (strides) {
    for (int d = 0; d < s->dim; ++d) {
      if (strides[d] < 1) return s->fail(CTD_EINVAL, "strides must be positive");
      contiguous = contiguous && strides[d] == cst[d];
    }
  }
  size_t total = 1;
  for (int d = 0; d < s->dim; ++d) total *= (size_t)n[d];
  const size_t esz = dtype == CTD_DTYPE_F32 ? 4 : 8;
  const size_t bytes = total * esz;
  void* dst = out;
  void* tmp = nullptr;
  if (!on_device || !contiguous) {
    HIPCHK(s, s->arena.raw_alloc(&tmp, bytes));
    dst = tmp;
  }
  hipError_t e;
  if (s->field3) {
    // a 3D field state is the nodal tensor itself
    e = dtype == CTD_DTYPE_F64 ? hipMemcpyAsync(dst, s->U3, bytes, hipMemcpyDeviceToDevice, s->stream)
                               : launch_field_to_f32(s->U3, (float*)dst, (int64_t)total, s->stream);
  } else {
    e = launch_reconstruct(V, s->Mk, dst, dtype, s->stream);
  }
  std::vector<unsigned char> host;
  if (e == hipSuccess && !contiguous && on_device)
    e = launch_scatter_strided(tmp, out, (int)esz, s->dim, n, strides, s->stream);
  if (e == hipSuccess && !on_device) {
    if (contiguous) {
      e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s->stream);
    } else {
      host.resize(bytes);
      e = hipMemcpyAsync(host.data(), tmp, bytes, hipMemcpyDeviceToHost, s->stream);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (tmp) s->arena.raw_free(tmp, bytes);
  if (e != hipSuccess) return s->hip_fail(e, "reconstruct");
  if (!host.empty()) {
    // host layout other than C order: place each element (marshalling only)
    unsigned char* o = (unsigned char*)out;
    size_t k = 0;
    for (int64_t i0 = 0; i0 < n[0]; ++i0)
      for (int64_t i1 = 0; i1 < n[1]; ++i1)
        for (int64_t i2 = 0; i2 < n[2]; ++i2, ++k) {
          int64_t off = i0 * strides[0];
          if (s->dim > 1) off += i1 * strides[1];
          if (s->dim > 2) off += i2 * strides[2];
          std::memcpy(o + (size_t)off * esz, host.data() + k * esz, esz);
        }
  }
  return CTD_OK;
}

int ctd_get_modes(ctd_solver* s, int32_t* m, double* amp, double* const* out, int32_t cap) {
  if (!s || !m) return CTD_EINVAL;
  if (s->field3) {
    // a 3D field state in separated form: mode j n2 + k = U[:, j, k] (x) e_j (x) e_k
    const int n0 = s->ax[0].n, n1 = s->ax[1].n, n2 = s->ax[2].n;
    const int64_t mf = (int64_t)n1 * n2;
    if (mf > INT32_MAX) return s->fail(CTD_EUNSUPPORTED, "field state too large for separated form");
    *m = (int32_t)mf;
    if (cap < mf) return (amp || out) ? s->fail(CTD_EINVAL, "cap smaller than mode count") : CTD_OK;
    HIPCHK(s, sync_collect(s));
    if (amp) std::fill(amp, amp + mf, 1.0);
    if (out && out[0]) {
      std::vector<double> U((size_t)n0 * mf);
      HIPCHK(s, copy_sync(s, U.data(), s->U3, sizeof(double) * U.size(), hipMemcpyDeviceToHost));
      for (int i = 0; i < n0; ++i)
        for (int64_t jk = 0; jk < mf; ++jk) out[0][(size_t)jk * n0 + i] = U[(size_t)i * mf + jk];
    }
    if (out && out[1]) {
      std::fill(out[1], out[1] + (size_t)n1 * mf, 0.0);
      for (int64_t jk = 0; jk < mf; ++jk) out[1][(size_t)jk * n1 + jk / n2] = 1.0;
    }
    if (out && out[2]) {
      std::fill(out[2], out[2] + (size_t)n2 * mf, 0.0);
      for (int64_t jk = 0; jk < mf; ++jk) out[2][(size_t)jk * n2 + jk % n2] = 1.0;
    }
    return CTD_OK;
  }
  *m = s->Mk;
  if (cap < s->Mk) return (amp || out) ? s->fail(CTD_EINVAL, "cap smaller than mode count") : CTD_OK;
  HIPCHK(s, sync_collect(s));
  if (amp) HIPCHK(s, copy_sync(s, amp, s->I.sk, sizeof(double) * s->Mk, hipMemcpyDeviceToHost));
  if (out)
    for (int d = 0; d < s->dim; ++d)
      if (out[d])
        HIPCHK(s, copy_sync(s, out[d], s->I.ax[d].Xk, sizeof(double) * s->ax[d].n * s->Mk, hipMemcpyDeviceToHost));
  return CTD_OK;
}

int ctd_get_step_index(ctd_solver* s, int64_t* k) {
  if (!s || !k) return CTD_EINVAL;
  *k = s->step_index;
  return CTD_OK;
}

int ctd_set_step_index(ctd_solver* s, int64_t k) {
  if (!s || k < 0) return CTD_EINVAL;
  s->step_index = k;
  return CTD_OK;
}

int ctd_get_decisions(ctd_solver* s, int32_t* buf, int64_t cap, int64_t* len) {
  if (!s || !len) return CTD_EINVAL;
  *len = (int64_t)s->decisions_last.size();
  if (!buf) return CTD_OK;
  if (cap < *len) return s->fail(CTD_EINVAL, "decision buffer too small");
  std::copy(s->decisions_last.begin(), s->decisions_last.end(), buf);
  return CTD_OK;
}

int ctd_set_decisions(ctd_solver* s, const int32_t* buf, int64_t len) {
  if (!s || (len > 0 && !buf) || len < 0) return CTD_EINVAL;
  s->decisions_next.assign(buf, buf + len);
  return CTD_OK;
}

const char* ctd_last_error(const ctd_solver* s) {
  return s ? s->err.c_str() : g_init_error.c_str();
}

void ctd_destroy(ctd_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  s->arena.release();
  s->prof.release();
  if (s->sc_host) (void)hipHostFree(s->sc_host);
  for (hipEvent_t e : s->sc_ev)
    if (e) (void)hipEventDestroy(e);
  delete s;
}

int ctd_kernel_copy(void* dst, const void* src, uint64_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16 != 0) return CTD_EINVAL;
  if (bytes == 0) return CTD_OK;
  hipError_t e = launch_copy16(dst, src, bytes, (hipStream_t)hip_stream);
  return e == hipSuccess ? CTD_OK : CTD_EDEVICE;
}

int ctd_kernel_band_solve(int32_t n, int32_t bw, const double* Mb, const double* Kb,
                          const double* alpha, const double* beta, const double* b,
                          double* x, int32_t count, void* hip_stream) {
  if (n < bw + 1 || (bw != 3 && bw != 5 && bw != 7) || count < 0) return CTD_EINVAL;
  if (!Mb || !Kb || !alpha || !beta || !b || !x) return CTD_EINVAL;
  if (count == 0) return CTD_OK;
  if (configure_kernels() != hipSuccess) return CTD_EDEVICE;
  hipError_t e = launch_band_solve_batch(n, bw, Mb, Kb, alpha, beta, b, x, count, (hipStream_t)hip_stream);
  return e == hipSuccess ? CTD_OK : CTD_EDEVICE;
}

}  // extern "C"

extern "C" int ctd_footprint_bytes(const ctd_problem* p, int32_t m0, uint64_t* bytes) {
  if (!bytes) return CTD_EINVAL;
  *bytes = 0;
  std::string err;
  int rc = validate(p, err);
  if (rc) return rc;
  if (m0 < 1) return CTD_EINVAL;
  (void)configure_kernels();   // without a device the LDS limit stays conservative
  (void)hipGetLastError();
  ctd_solver tmp;
  rc = setup_host(&tmp, p, nullptr, err);
  if (rc) return rc;
  tmp.arena.dry = true;
  rc = alloc_instance(&tmp, m0);
  if (rc) return rc;
  *bytes = tmp.arena.bytes;
  return CTD_OK;
}

namespace ctd {
void solver_bind_stream(ctd_solver* s, hipStream_t st) {
  s->stream = st;
  s->arena.stream = st;
}
size_t solver_device_bytes(const ctd_solver* s) { return s->arena.bytes; }
}  // namespace ctd

extern "C" int ctd_tuning_set_prec(int32_t precision, int32_t nb, int32_t nq, int32_t nsplit_g,
                                   int32_t nsplit_h) {
  if ((precision != CTD_PREC_FP64 && precision != CTD_PREC_MIXED) || nb < 1 || nq < 1 || nsplit_g < 1 ||
      nsplit_h < 1)
    return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[{precision, nb, nq}] = {nsplit_g, nsplit_h};
  return CTD_OK;
}

extern "C" int ctd_tuning_set(int32_t nb, int32_t nq, int32_t nsplit_g, int32_t nsplit_h) {
  return ctd_tuning_set_prec(CTD_PREC_MIXED, nb, nq, nsplit_g, nsplit_h);
}

extern "C" int ctd_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return CTD_OK;
}

extern "C" int ctd_tuning_current(ctd_solver* s, int32_t* nsplit_g, int32_t* nsplit_h) {
  if (!s || !nsplit_g || !nsplit_h) return CTD_EINVAL;
  *nsplit_g = s->dim == 3 ? s->I.nsplit_g : 0;
  *nsplit_h = s->dim == 3 ? s->I.nsplit_h : 0;
  return CTD_OK;
}

extern "C" int ctd_reduced_domain_excluded(ctd_solver* s, int64_t* count) {
  if (!s || !count) return CTD_EINVAL;
  *count = 0;
  if (s->dim != 2 || !(s->P.rd_tol > 0.0)) return CTD_OK;
  unsigned long long c = 0;
  HIPCHK(s, hipMemcpyAsync(&c, s->I.rd_count, sizeof(c), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  *count = (int64_t)c;
  return CTD_OK;
}

extern "C" int ctd_nonlinear_load(ctd_solver* s, int32_t d, const double* const* u, double* out) {
  if (!s || !u || !out || d < 0 || d >= s->dim) return CTD_EINVAL;
  if (s->field3) return s->fail(CTD_EUNSUPPORTED, "the separated load needs a separated state");
  const int D = s->dim;
  update_view(s);
  for (int e = 0; e < D; ++e) {
    if (e == d) continue;
    if (!u[e]) return s->fail(CTD_EINVAL, "u[e] is NULL");
    HIPCHK(s, hipMemcpyAsync(s->I.ax[e].u, u[e], sizeof(double) * s->ax[e].n, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, launch_signature(s->I, e, 0, s->stream));
  }
  if (D == 3) {
    int e1 = -1, e2 = -1;
    for (int e = 0; e < 3; ++e)
      if (e != d) { if (e1 < 0) e1 = e; else e2 = e; }
    int rc = cubic_after(s, e1, -1);
    if (rc) return rc;
    rc = cubic_after(s, e2, d);
    if (rc) return rc;
    Work w = w_cubic(s, d);
    LAUNCH(s, CTD_K_CUBIC_H, w.flops, w.bytes, launch_cubic_h(s->I, d, s->stream));
  }
  HIPCHK(s, launch_rhs(s->I, d, 0, s->stream, 1));
  HIPCHK(s, launch_rhs_sum(s->I, d, 0, 1, s->stream));
  HIPCHK(s, hipMemcpyAsync(out, s->I.ax[d].rhs, sizeof(double) * s->ax[d].n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, sync_collect(s));
  return CTD_OK;
}

extern "C" int ctd_profile_enable(ctd_solver* s, int32_t on) {
  return ctd_profile_select(s, on ? ~0u : 0u);
}

extern "C" int ctd_profile_select(ctd_solver* s, uint32_t mask) {
  if (!s) return CTD_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->prof.reset();
  s->prof.on = mask != 0;
  s->prof.mask = mask;
  return CTD_OK;
}

extern "C" int ctd_profile_read(ctd_solver* s, int32_t kernel, int64_t* launches, double* ms,
                                double* flops, double* bytes) {
  if (!s || kernel < 0 || kernel >= CTD_K_COUNT) return CTD_EINVAL;
  if (launches) *launches = s->prof.launches[kernel];
  if (ms) *ms = s->prof.ms[kernel];
  if (flops) *flops = s->prof.flops[kernel];
  if (bytes) *bytes = s->prof.bytes[kernel];
  return CTD_OK;
}
