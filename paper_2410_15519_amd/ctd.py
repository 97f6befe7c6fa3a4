"""Python binding of libctd.so (ctypes; argument marshalling only).

Every step of the CTD solve runs in the HIP library; this module only builds
the problem struct, passes host arrays and torch device buffers/streams, and
unpacks results.  Importing it fails loudly if the library was not built.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctd.so")

CTD_OK = 0
CTD_EAGAIN = -7
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE",
          -5: "ESTATE", -6: "EUNSUPPORTED", -7: "EAGAIN"}
PREC = {"fp64": 0, "mixed": 1}
SCHED = {"adaptive": 0, "replay": 1}
INIT = {"hash": 0, "warm": 1}
DTYPE = {"f64": 0, "f32": 1}
SOLVE = {"auto": 0, "bcr": 1, "fd": 2}
BATCH_MODE = {"auto": 0, "lockstep": 1, "streams": 2}
KERNELS = ["cubic_g", "cubic_gred", "cubic_h", "rhs", "solve", "signature", "gemv",
           "mxy_build", "energy", "quad_eval", "other", "finalize", "full_solve", "skipped"]


class CtdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("dim", C.c_int32),
        ("nodes", C.c_int64 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("eps", C.c_double), ("S", C.c_double), ("dt", C.c_double),
        ("L", C.c_double), ("kappa", C.c_double), ("a0", C.c_double), ("alpha", C.c_double),
        ("patch_s", C.c_int32), ("poly_p", C.c_int32),
        ("dilation_a", C.c_double),
        ("gauss_points", C.c_int32), ("fp_max_iter", C.c_int32),
        ("fp_tol", C.c_double), ("enrich_tol", C.c_double),
        ("max_modes", C.c_int32), ("precision", C.c_int32),
        ("schedule", C.c_int32), ("init_mode", C.c_int32),
        ("energy_each_step", C.c_int32), ("solve_method", C.c_int32),
        ("actd", C.c_int32), ("seed", C.c_uint64),
        ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("alloc_ctx", C.c_void_p),
        ("rd_tol", C.c_double), ("w_rank", C.c_int32), ("w_iters", C.c_int32),
    ]


class StepInfo(C.Structure):
    _fields_ = [
        ("modes", C.c_int32), ("sweeps", C.c_int32), ("capped", C.c_int32),
        ("fp_unconverged", C.c_int32), ("zero_mode", C.c_int32),
        ("energy_increase", C.c_int32), ("full_solve", C.c_int32),
        ("stability_warning", C.c_int32), ("energy", C.c_double),
        ("last_term_max", C.c_double), ("ms", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


REQ_STATE = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class RequestStatus(C.Structure):
    _fields_ = [("state", C.c_int32), ("steps_done", C.c_int32), ("modes", C.c_int32),
                ("error", C.c_int32), ("t_submit_ms", C.c_double), ("t_start_ms", C.c_double),
                ("t_done_ms", C.c_double), ("footprint", C.c_uint64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["state"] = REQ_STATE.get(self.state, self.state)
        return d


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("running", C.c_int64), ("bytes_in_use", C.c_uint64),
                ("budget", C.c_uint64), ("steps_done", C.c_int64), ("busy_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sig = {
        "ctd_problem_default": (C.c_int, [P(Problem)]),
        "ctd_init": (C.c_int, [P(Problem), C.c_int32, P(P(C.c_double)), P(C.c_double), vp, P(vp)]),
        "ctd_step": (C.c_int, [vp, C.c_int32, P(StepInfo)]),
        "ctd_energy": (C.c_int, [vp, P(C.c_double)]),
        "ctd_reconstruct": (C.c_int, [vp, vp, C.c_int32, C.c_int32, P(C.c_int64)]),
        "ctd_get_modes": (C.c_int, [vp, P(C.c_int32), P(C.c_double), P(P(C.c_double)), C.c_int32]),
        "ctd_get_step_index": (C.c_int, [vp, P(C.c_int64)]),
        "ctd_set_step_index": (C.c_int, [vp, C.c_int64]),
        "ctd_get_decisions": (C.c_int, [vp, P(C.c_int32), C.c_int64, P(C.c_int64)]),
        "ctd_set_decisions": (C.c_int, [vp, P(C.c_int32), C.c_int64]),
        "ctd_last_error": (C.c_char_p, [vp]),
        "ctd_destroy": (None, [vp]),
        "ctd_batch_create": (C.c_int, [C.c_int32, P(Problem), P(C.c_int32), P(P(P(C.c_double))),
                                       P(P(C.c_double)), vp, P(vp)]),
        "ctd_batch_set_workers": (C.c_int, [vp, C.c_int32]),
        "ctd_batch_set_mode": (C.c_int, [vp, C.c_int32]),
        "ctd_batch_step": (C.c_int, [vp, C.c_int32, P(StepInfo)]),
        "ctd_footprint_bytes": (C.c_int, [P(Problem), C.c_int32, P(C.c_uint64)]),
        "ctd_server_create": (C.c_int, [C.c_uint64, C.c_int32, P(vp)]),
        "ctd_server_set_lockstep": (C.c_int, [vp, C.c_int32]),
        "ctd_server_submit": (C.c_int, [vp, P(Problem), C.c_int32, P(P(C.c_double)), P(C.c_double),
                                        C.c_int32, P(C.c_int64)]),
        "ctd_server_status": (C.c_int, [vp, C.c_int64, P(RequestStatus)]),
        "ctd_server_wait": (C.c_int, [vp, C.c_int64, C.c_double]),
        "ctd_server_fetch": (C.c_int, [vp, C.c_int64, P(C.c_int32), P(C.c_double), P(P(C.c_double)),
                                       C.c_int32, C.c_int32]),
        "ctd_server_get_stats": (C.c_int, [vp, P(ServerStats)]),
        "ctd_server_last_error": (C.c_char_p, [vp]),
        "ctd_server_destroy": (None, [vp]),
        "ctd_batch_get_modes": (C.c_int, [vp, C.c_int32, P(C.c_int32), P(C.c_double),
                                          P(P(C.c_double)), C.c_int32]),
        "ctd_batch_reconstruct": (C.c_int, [vp, C.c_int32, vp, C.c_int32, C.c_int32, P(C.c_int64)]),
        "ctd_batch_last_error": (C.c_char_p, [vp]),
        "ctd_batch_destroy": (None, [vp]),
        "ctd_kernel_band_solve": (C.c_int, [C.c_int32, C.c_int32, vp, vp, vp, vp, vp, vp,
                                            C.c_int32, vp]),
        "ctd_kernel_band_solve_noalloc": (C.c_int, [C.c_int32, C.c_int32, vp, vp, vp, vp, vp, vp,
                                                    C.c_int32, vp]),
        "ctd_nonlinear_load": (C.c_int, [vp, C.c_int32, P(P(C.c_double)), P(C.c_double)]),
        "ctd_kernel_copy": (C.c_int, [vp, vp, C.c_uint64, vp]),
        "ctd_axis_fast_diag": (C.c_int, [C.c_int64, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                         C.c_double, C.c_int32, P(C.c_double), P(C.c_double)]),
        "ctd_profile_enable": (C.c_int, [vp, C.c_int32]),
        "ctd_profile_select": (C.c_int, [vp, C.c_uint32]),
        "ctd_tuning_set": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "ctd_tuning_set_prec": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "ctd_tuning_clear": (C.c_int, []),
        "ctd_tuning_current": (C.c_int, [vp, P(C.c_int32), P(C.c_int32)]),
        "ctd_reduced_domain_excluded": (C.c_int, [vp, P(C.c_int64)]),
        "ctd_profile_read": (C.c_int, [vp, C.c_int32, P(C.c_int64), P(C.c_double),
                                       P(C.c_double), P(C.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()

TUNING_PATH = os.path.join(HERE, "tuning.json")


def tuning_set(nb, nq, nsplit_g, nsplit_h, precision="mixed"):
    """ctd_tuning_set_prec: split counts of the 3D cubic contraction for
    (precision, nb, nq)."""
    rc = LIB.ctd_tuning_set_prec(PREC[precision], int(nb), int(nq), int(nsplit_g), int(nsplit_h))
    if rc != CTD_OK:
        raise CtdError(rc, "ctd_tuning_set")


def tuning_clear():
    LIB.ctd_tuning_clear()


def tuning_load(path=TUNING_PATH):
    """Register the entries of a tuning table written by tune.py (no-op when
    the file is absent); returns the number of entries."""
    if not os.path.exists(path):
        return 0
    import json
    with open(path) as f:
        table = json.load(f)
    for e in table.get("entries", []):
        tuning_set(e["nb"], e["nq"], e["nsplit_g"], e["nsplit_h"], e.get("precision", "mixed"))
    return len(table.get("entries", []))


tuning_load()


def current_stream():
    """hipStream_t of torch's current stream (None when torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


# Device allocator hooks (ctd_problem.dev_alloc / dev_free): instance memory
# from torch's caching allocator on the instance's stream.  ctypes callbacks
# take the GIL, so they are safe on the library's worker threads.
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p)


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:          # out of memory: the library reports CTD_ENOMEM
        return None


def _torch_free(ptr, nbytes, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:          # interpreter shutdown: the process frees it
        pass


TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
TORCH_FREE = _FREE_FN(_torch_free)


def _torch_has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def make_problem(inst=None, *, precision="fp64", schedule="adaptive", init="warm",
                 energy=False, solve="auto", actd=False, allocator="torch", **over) -> Problem:
    """ctd_problem from a workloads.Instance (epsilon form) plus overrides.

    allocator: "torch" (device memory from torch's caching allocator, when
    torch has a GPU) or "library" (hipMallocAsync inside the library)."""
    p = Problem()
    rc = LIB.ctd_problem_default(C.byref(p))
    if rc != CTD_OK:
        raise CtdError(rc, "ctd_problem_default")
    if inst is not None:
        p.dim = inst.dim
        for d in range(inst.dim):
            p.nodes[d] = int(inst.nodes[d])
            p.lo[d] = float(inst.lo[d])
            p.hi[d] = float(inst.hi[d])
        p.eps, p.S, p.dt = float(inst.eps), float(inst.S), float(inst.dt)
        p.patch_s, p.poly_p = int(inst.patch_s), int(inst.poly_p)
        p.dilation_a = float(inst.dilation_a)
        p.gauss_points = int(inst.gauss_points)
        p.fp_tol, p.fp_max_iter = float(inst.fp_tol), int(inst.fp_max_iter)
        p.enrich_tol, p.max_modes = float(inst.enrich_tol), int(inst.max_modes)
        p.seed = int(inst.seed)
    p.precision = PREC[precision]
    p.schedule = SCHED[schedule]
    p.init_mode = INIT[init]
    p.energy_each_step = 1 if energy else 0
    p.solve_method = SOLVE[solve]
    p.actd = 1 if actd else 0
    if allocator == "torch" and _torch_has_gpu():
        p.dev_alloc = C.cast(TORCH_ALLOC, C.c_void_p).value
        p.dev_free = C.cast(TORCH_FREE, C.c_void_p).value
    elif allocator not in ("torch", "library"):
        raise ValueError("allocator is 'torch' or 'library'")
    for k, v in over.items():
        if k in ("nodes", "lo", "hi"):
            for d, x in enumerate(v):
                getattr(p, k)[d] = x
        else:
            setattr(p, k, v)
    return p


def _factor_ptrs(factors):
    arrs = [np.asfortranarray(np.asarray(f, dtype=np.float64)) for f in factors]
    ptrs = (C.POINTER(C.c_double) * 3)()
    for d, a in enumerate(arrs):
        ptrs[d] = a.ctypes.data_as(C.POINTER(C.c_double))
    return arrs, ptrs


class Solver:
    """One CTD instance on the GPU (handle around ctd_init / ctd_step ...)."""

    def __init__(self, inst, stream=None, **kw):
        self.inst = inst
        self.problem = make_problem(inst, **kw)
        self.dim = inst.dim
        self.nodes = tuple(int(n) for n in inst.nodes[: inst.dim])
        arrs, ptrs = _factor_ptrs(inst.factors)
        amp = np.ascontiguousarray(inst.amp, dtype=np.float64)
        self._stream = stream if stream is not None else current_stream()
        h = C.c_void_p()
        rc = LIB.ctd_init(C.byref(self.problem), len(amp), ptrs,
                          amp.ctypes.data_as(C.POINTER(C.c_double)), self._stream, C.byref(h))
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_last_error(self.h).decode())

    def step(self, nsteps=1):
        info = (StepInfo * max(nsteps, 1))()
        self._check(LIB.ctd_step(self.h, nsteps, info))
        return [info[i].as_dict() for i in range(nsteps)]

    def energy(self):
        e = C.c_double()
        self._check(LIB.ctd_energy(self.h, C.byref(e)))
        return e.value

    def reconstruct(self, dtype="f64", out=None):
        """Dense nodal field.  out: optional torch device tensor or numpy array
        of the grid's shape, any positive strides (filled in place)."""
        if out is not None:
            if hasattr(out, "data_ptr"):
                # a flat buffer (or any contiguous tensor) is taken in C order
                strides = None if out.dim() != self.dim else (C.c_int64 * 3)(*out.stride())
                self._check(LIB.ctd_reconstruct(self.h, C.c_void_p(out.data_ptr()), DTYPE[dtype], 1,
                                                strides))
            else:
                strides = (None if out.ndim != self.dim else
                           (C.c_int64 * 3)(*[st // out.itemsize for st in out.strides]))
                self._check(LIB.ctd_reconstruct(self.h, out.ctypes.data_as(C.c_void_p), DTYPE[dtype],
                                                0, strides))
            return out
        arr = np.empty(self.nodes, dtype=np.float64 if dtype == "f64" else np.float32)
        self._check(LIB.ctd_reconstruct(self.h, arr.ctypes.data_as(C.c_void_p), DTYPE[dtype], 0, None))
        return arr

    def modes(self):
        m = C.c_int32()
        self._check(LIB.ctd_get_modes(self.h, C.byref(m), None, None, 0))
        M = m.value
        amp = np.empty(M)
        outs = [np.empty((n, M), order="F") for n in self.nodes]
        ptrs = (C.POINTER(C.c_double) * 3)()
        for d, a in enumerate(outs):
            ptrs[d] = a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(LIB.ctd_get_modes(self.h, C.byref(m), amp.ctypes.data_as(C.POINTER(C.c_double)),
                                      ptrs, M))
        return amp, outs

    def nonlinear_load(self, d, u):
        """F_d[i] = int N~_i prod_{e!=d} u_e L w(u^k) on the current u^k (GPU kernels)."""
        arrs = [np.ascontiguousarray(np.asarray(v if v is not None else np.zeros(n)), dtype=np.float64)
                for v, n in zip(u, self.nodes)]
        ptrs = (C.POINTER(C.c_double) * 3)()
        for e, a in enumerate(arrs):
            ptrs[e] = a.ctypes.data_as(C.POINTER(C.c_double))
        out = np.empty(self.nodes[d])
        self._check(LIB.ctd_nonlinear_load(self.h, d, ptrs, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def tuning_current(self):
        """(nsplit_g, nsplit_h) the handle uses for its current M_k (3D)."""
        g, h = C.c_int32(), C.c_int32()
        self._check(LIB.ctd_tuning_current(self.h, C.byref(g), C.byref(h)))
        return g.value, h.value

    def reduced_domain_excluded(self):
        """Elements the reduced domain (rd_tol > 0, 2D) leaves out of the M_xy
        of the next step (built from the current state)."""
        c = C.c_int64()
        self._check(LIB.ctd_reduced_domain_excluded(self.h, C.byref(c)))
        return c.value
    def profile(self, on=True, classes=None):
        """Enable (and reset) or disable per-kernel HIP-event timing; classes:
        names from KERNELS to time (default all)."""
        if not on:
            self._check(LIB.ctd_profile_select(self.h, 0))
        elif classes is None:
            self._check(LIB.ctd_profile_enable(self.h, 1))
        else:
            mask = 0
            for c in classes:
                mask |= 1 << KERNELS.index(c)
            self._check(LIB.ctd_profile_select(self.h, mask))

    def profile_read(self):
        out = {}
        for k, name in enumerate(KERNELS):
            n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            self._check(LIB.ctd_profile_read(self.h, k, C.byref(n), C.byref(ms), C.byref(fl),
                                             C.byref(by)))
            if n.value:
                out[name] = {"launches": n.value, "ms": ms.value, "flops": fl.value,
                             "bytes": by.value}
        return out

    def decisions(self):
        n = C.c_int64()
        self._check(LIB.ctd_get_decisions(self.h, None, 0, C.byref(n)))
        buf = (C.c_int32 * max(n.value, 1))()
        self._check(LIB.ctd_get_decisions(self.h, buf, n.value, C.byref(n)))
        flat = list(buf[: n.value])
        steps, i = [], 0
        while i < len(flat):
            m = flat[i]
            if m == -1:
                steps.append("full")
                i += 1
                continue
            steps.append(flat[i + 1: i + 1 + m])
            i += 1 + m
        return steps

    def set_decisions(self, steps):
        """Per step a list of sweep counts, or "full" for the full CFE solve."""
        flat = []
        for it in steps:
            if isinstance(it, str):
                if it != "full":
                    raise ValueError("a step's decisions are sweep counts or 'full'")
                flat.append(-1)
                continue
            flat.append(len(it))
            flat.extend(int(x) for x in it)
        buf = (C.c_int32 * max(len(flat), 1))(*flat)
        self._check(LIB.ctd_set_decisions(self.h, buf, len(flat)))

    @property
    def step_index(self):
        k = C.c_int64()
        self._check(LIB.ctd_get_step_index(self.h, C.byref(k)))
        return k.value

    @step_index.setter
    def step_index(self, k):
        self._check(LIB.ctd_set_step_index(self.h, int(k)))

    def close(self):
        if getattr(self, "h", None):
            LIB.ctd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Many independent instances stepped together (ctd_batch_*)."""

    def __init__(self, insts, stream=None, **kw):
        self.insts = list(insts)
        cnt = len(self.insts)
        probs = (Problem * cnt)()
        m0 = (C.c_int32 * cnt)()
        inits = (C.POINTER(C.POINTER(C.c_double)) * cnt)()
        amps = (C.POINTER(C.c_double) * cnt)()
        self._keep = []
        for i, inst in enumerate(self.insts):
            probs[i] = make_problem(inst, **kw)
            arrs, ptrs = _factor_ptrs(inst.factors)
            amp = np.ascontiguousarray(inst.amp, dtype=np.float64)
            self._keep += [arrs, ptrs, amp]
            m0[i] = len(amp)
            inits[i] = C.cast(ptrs, C.POINTER(C.POINTER(C.c_double)))
            amps[i] = amp.ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        st = stream if stream is not None else current_stream()
        rc = LIB.ctd_batch_create(cnt, probs, m0, inits, amps, st, C.byref(h))
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_batch_last_error(None).decode())
        self.h = h

    def set_workers(self, workers):
        rc = LIB.ctd_batch_set_workers(self.h, int(workers))
        if rc != CTD_OK:
            raise CtdError(rc, "ctd_batch_set_workers")

    def set_mode(self, mode):
        """"auto" | "lockstep" | "streams" (ctd_batch_set_mode)."""
        rc = LIB.ctd_batch_set_mode(self.h, BATCH_MODE[mode])
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_batch_last_error(self.h).decode())

    def modes(self, i):
        m = C.c_int32()
        rc = LIB.ctd_batch_get_modes(self.h, i, C.byref(m), None, None, 0)
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_batch_last_error(self.h).decode())
        inst = self.insts[i]
        amp, outs, ptrs = _mode_buffers(inst.nodes[: inst.dim], m.value)
        rc = LIB.ctd_batch_get_modes(self.h, i, C.byref(m), amp.ctypes.data_as(C.POINTER(C.c_double)),
                                     ptrs, m.value)
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_batch_last_error(self.h).decode())
        return amp, outs

    def step(self, nsteps=1):
        n = len(self.insts)
        info = (StepInfo * max(n * nsteps, 1))()
        rc = LIB.ctd_batch_step(self.h, nsteps, info)
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_batch_last_error(self.h).decode())
        return [[info[i * nsteps + k].as_dict() for k in range(nsteps)] for i in range(n)]

    def reconstruct(self, i, dtype="f64"):
        inst = self.insts[i]
        arr = np.empty(tuple(inst.nodes[: inst.dim]), dtype=np.float64 if dtype == "f64" else np.float32)
        rc = LIB.ctd_batch_reconstruct(self.h, i, arr.ctypes.data_as(C.c_void_p), DTYPE[dtype], 0, None)
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_batch_last_error(self.h).decode())
        return arr

    def close(self):
        if getattr(self, "h", None):
            LIB.ctd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _mode_buffers(nodes, M):
    amp = np.empty(M)
    outs = [np.empty((int(n), M), order="F") for n in nodes]
    ptrs = (C.POINTER(C.c_double) * 3)()
    for d, a in enumerate(outs):
        ptrs[d] = a.ctypes.data_as(C.POINTER(C.c_double))
    return amp, outs, ptrs


def footprint_bytes(inst, m0=None, **kw):
    """Device bytes ctd_init allocates for this instance (ctd_footprint_bytes)."""
    p = make_problem(inst, **kw)
    b = C.c_uint64()
    rc = LIB.ctd_footprint_bytes(C.byref(p), int(len(inst.amp) if m0 is None else m0), C.byref(b))
    if rc != CTD_OK:
        raise CtdError(rc, "ctd_footprint_bytes")
    return b.value


class Server:
    """Served execution with continuous batching (ctd_server_*)."""

    def __init__(self, budget_bytes=0, workers=8, lockstep=True):
        h = C.c_void_p()
        rc = LIB.ctd_server_create(int(budget_bytes), int(workers), C.byref(h))
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_server_last_error(None).decode())
        if not lockstep:
            LIB.ctd_server_set_lockstep(h, 0)
        self.h = h
        self._nodes = {}

    def _check(self, rc):
        if rc != CTD_OK:
            raise CtdError(rc, LIB.ctd_server_last_error(self.h).decode())

    def submit(self, inst, nsteps=None, **kw):
        p = make_problem(inst, **kw)
        arrs, ptrs = _factor_ptrs(inst.factors)
        amp = np.ascontiguousarray(inst.amp, dtype=np.float64)
        t = C.c_int64()
        self._check(LIB.ctd_server_submit(self.h, C.byref(p), len(amp), ptrs,
                                          amp.ctypes.data_as(C.POINTER(C.c_double)),
                                          int(inst.steps if nsteps is None else nsteps), C.byref(t)))
        self._nodes[t.value] = tuple(int(n) for n in inst.nodes[: inst.dim])
        return t.value

    def status(self, ticket):
        st = RequestStatus()
        self._check(LIB.ctd_server_status(self.h, ticket, C.byref(st)))
        return st.as_dict()

    def wait(self, ticket, timeout_ms=-1.0):
        rc = LIB.ctd_server_wait(self.h, ticket, float(timeout_ms))
        if rc == CTD_EAGAIN:
            return False
        self._check(rc)
        return True

    def fetch(self, ticket, release=True):
        """Modes of a done request; a failed request raises its error (and is
        forgotten when release is set)."""
        m = C.c_int32()
        rc = LIB.ctd_server_fetch(self.h, ticket, C.byref(m), None, None, 0, 0)
        if rc != CTD_OK:
            err = CtdError(rc, LIB.ctd_server_last_error(self.h).decode())
            if release and rc != CTD_EAGAIN and self.status(ticket)["state"] == "failed":
                LIB.ctd_server_fetch(self.h, ticket, C.byref(m), None, None, 0, 1)
                self._nodes.pop(ticket, None)
            raise err
        amp, outs, ptrs = _mode_buffers(self._nodes[ticket], m.value)
        self._check(LIB.ctd_server_fetch(self.h, ticket, C.byref(m),
                                         amp.ctypes.data_as(C.POINTER(C.c_double)), ptrs, m.value,
                                         1 if release else 0))
        if release:
            self._nodes.pop(ticket, None)
        return amp, outs

    def stats(self):
        st = ServerStats()
        self._check(LIB.ctd_server_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            LIB.ctd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def kernel_copy(dst, src, stream=None):
    """ctd_kernel_copy between torch device tensors (same byte size)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    rc = LIB.ctd_kernel_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                             stream if stream is not None else current_stream())
    if rc != CTD_OK:
        raise CtdError(rc, "ctd_kernel_copy")


def band_solve(n, bw, Mb, Kb, alpha, beta, b, x, count, stream=None):
    """ctd_kernel_band_solve on torch device tensors (float64)."""
    rc = LIB.ctd_kernel_band_solve(n, bw, C.c_void_p(Mb.data_ptr()), C.c_void_p(Kb.data_ptr()),
                                   C.c_void_p(alpha.data_ptr()), C.c_void_p(beta.data_ptr()),
                                   C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), count,
                                   stream if stream is not None else current_stream())
    if rc != CTD_OK:
        raise CtdError(rc, "ctd_kernel_band_solve")


def band_solve_noalloc(n, bw, Mb, Kb, alpha, beta, b, x, count, stream=None):
    """ctd_kernel_band_solve_noalloc on torch device tensors (float64): the
    same solve with its workspace in the library's static device array."""
    rc = LIB.ctd_kernel_band_solve_noalloc(n, bw, C.c_void_p(Mb.data_ptr()), C.c_void_p(Kb.data_ptr()),
                                           C.c_void_p(alpha.data_ptr()), C.c_void_p(beta.data_ptr()),
                                           C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), count,
                                           stream if stream is not None else current_stream())
    if rc != CTD_OK:
        raise CtdError(rc, "ctd_kernel_band_solve_noalloc")
