"""The C-ABI library loads and exports every function include/ctd.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctd.h")
LIB = os.path.join(ROOT, "paper_2410_15519_amd", "libctd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(ctd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_parses():
    names = declared_functions()
    assert "ctd_init" in names and "ctd_step" in names and "ctd_energy" in names
    assert "ctd_reconstruct" in names and "ctd_batch_step" in names


def test_library_exports_declared_symbols():
    if not os.path.exists(LIB):
        pytest.fail("libctd.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_struct_layout_and_validation():
    """ctd_problem_default and ctd_init's validation run without touching a GPU."""
    from paper_2410_15519_amd import ctd
    p = ctd.make_problem()
    assert p.abi_version == 4 and p.dim == 2 and p.max_modes == 64 and p.actd == 0
    assert p.init_mode == ctd.INIT["warm"]          # library default: warm guess
    raw = ctd.Problem()
    assert ctd.LIB.ctd_problem_default(ctypes.byref(raw)) == 0
    assert raw.init_mode == ctd.INIT["warm"] and not raw.dev_alloc and not raw.dev_free
    assert ctypes.sizeof(ctd.Problem) == 256
    assert raw.rd_tol == 0.0 and raw.w_rank == 0 and raw.w_iters == 30
    assert ctypes.sizeof(ctd.StepInfo) == 56
    # allocator hooks: both or neither
    half = ctd.make_problem(allocator="library")
    half.dev_alloc = ctypes.cast(ctd.TORCH_ALLOC, ctypes.c_void_p).value
    h = ctypes.c_void_p()
    ptrs0 = (ctypes.POINTER(ctypes.c_double) * 3)()
    assert ctd.LIB.ctd_init(ctypes.byref(half), 1, ptrs0, None, None, ctypes.byref(h)) == -1
    assert b"dev_alloc" in ctd.LIB.ctd_last_error(None)
    # invalid problems fail before any allocation or device call
    bad = ctd.make_problem(dim=4)
    h = ctypes.c_void_p()
    ptrs = (ctypes.POINTER(ctypes.c_double) * 3)()
    rc = ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert b"dim" in ctd.LIB.ctd_last_error(None)
    bad = ctd.make_problem(patch_s=1, poly_p=2)
    rc = ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h))
    assert rc == -1
    # the full-solve fallback in 3D works on the tensor Gauss grid: bounded
    bad = ctd.make_problem(dim=3, actd=True, nodes=(256, 256, 256))
    rc = ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h))
    assert rc == -6 and not h.value and b"Gauss points" in ctd.LIB.ctd_last_error(None)
    bad = ctd.make_problem(actd=True, nodes=(4096, 64, 64))
    assert ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h)) == -6
    # the reduced integration domain: finite, >= 0, and defined for the 2D M_xy
    for tol in (-1e-3, float("nan"), float("inf")):
        bad = ctd.make_problem(rd_tol=tol)
        assert ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h)) == -1
        assert b"rd_tol" in ctd.LIB.ctd_last_error(None)
    for kw in (dict(dim=3), dict(actd=True)):
        bad = ctd.make_problem(rd_tol=0.1, **kw)
        assert ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h)) == -6
        assert not h.value and b"reduced" in ctd.LIB.ctd_last_error(None)
    # the separated w: bounded rank and update count, 2D only, one alternative
    for kw in (dict(w_rank=-1), dict(w_rank=257), dict(w_rank=4, w_iters=-1)):
        bad = ctd.make_problem(**kw)
        assert ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h)) == -1
        assert b"w_rank" in ctd.LIB.ctd_last_error(None)
    for kw in (dict(dim=3), dict(actd=True), dict(rd_tol=0.1)):
        bad = ctd.make_problem(w_rank=4, **kw)
        assert ctd.LIB.ctd_init(ctypes.byref(bad), 1, ptrs, None, None, ctypes.byref(h)) == -6
        assert not h.value and b"separated" in ctd.LIB.ctd_last_error(None)
    count = ctypes.c_int64(7)
    assert ctd.LIB.ctd_reduced_domain_excluded(None, ctypes.byref(count)) == -1


def test_footprint_query_without_device():
    """ctd_footprint_bytes sizes an instance from its shape alone (no GPU needed)."""
    from paper_2410_15519_amd import ctd
    from workloads import small_instance
    f = lambda inst, **kw: ctd.footprint_bytes(inst, **kw)
    small, big = small_instance(2, 24), small_instance(2, 200)
    assert 0 < f(small) < f(big)
    assert f(small, max_modes=8) < f(small, max_modes=32)
    three = small_instance(3, 21, max_modes=16)
    # 3D adds the tile-triple Grams; FP32 tables halve those
    assert f(three, precision="mixed") < f(three, precision="fp64")
    # every buffer is rounded to 256 bytes
    assert f(small) % 256 == 0
    # actd keeps one mode per node of axis 1 for field states
    assert f(small, actd=True) > f(small)
    # the separated w holds W and W^T on the Gauss grid (5 points per element)
    nq = 5 * 23
    assert f(small, w_rank=4) - f(small) >= 16 * nq * nq
    assert f(small, rd_tol=0.1) == f(small)
    # 3D actd: the field, its right-hand-side tensor and two Gauss-grid buffers
    nq = 5 * 20
    assert f(three, actd=True) - f(three) >= 8 * (2 * 21 ** 3 + 2 * nq ** 3)
    bad = ctd.make_problem(dim=4)
    b = ctypes.c_uint64()
    assert ctd.LIB.ctd_footprint_bytes(ctypes.byref(bad), 1, ctypes.byref(b)) == -1
    assert ctd.LIB.ctd_footprint_bytes(ctypes.byref(ctd.make_problem()), 0, ctypes.byref(b)) == -1


def test_server_and_batch_argument_checks():
    from paper_2410_15519_amd import ctd
    h = ctypes.c_void_p()
    assert ctd.LIB.ctd_server_create(0, 0, ctypes.byref(h)) == -1 and not h.value
    assert ctd.LIB.ctd_server_create(0, 65, ctypes.byref(h)) == -1 and not h.value
    assert ctd.LIB.ctd_batch_set_workers(None, 4) == -1
    ctd.LIB.ctd_server_destroy(None)
    assert ctd.LIB.ctd_server_last_error(None)


def test_tuning_table_arguments_and_file():
    """The split-count table: argument checks, set/clear, and the committed
    table written by tune.py (one entry per mode-tile count, positive splits)."""
    import json
    import os
    from paper_2410_15519_amd import ctd
    assert ctd.LIB.ctd_tuning_set(0, 100, 8, 8) == -1
    assert ctd.LIB.ctd_tuning_set(1, 100, 0, 8) == -1
    assert ctd.LIB.ctd_tuning_set(1, 100, 8, -1) == -1
    assert ctd.LIB.ctd_tuning_set(1, 100, 8, 8) == 0
    assert ctd.LIB.ctd_tuning_set_prec(2, 1, 100, 8, 8) == -1
    assert ctd.LIB.ctd_tuning_set_prec(0, 1, 100, 8, 8) == 0
    assert ctd.LIB.ctd_tuning_current(None, None, None) == -1
    assert ctd.LIB.ctd_tuning_clear() == 0
    if os.path.exists(ctd.TUNING_PATH):
        with open(ctd.TUNING_PATH) as f:
            table = json.load(f)
        # one entry per (precision, mode-tile count), tile counts ascending
        keys = [(e.get("precision", "mixed"), e["nb"]) for e in table["entries"]]
        assert len(keys) == len(set(keys))
        for prec in {k[0] for k in keys}:
            assert prec in ("mixed", "fp64")
            nbs = [k[1] for k in keys if k[0] == prec]
            assert nbs == sorted(nbs)
        assert all(e["nsplit_g"] >= 1 and e["nsplit_h"] >= 1 and e["nq"] >= 1 for e in table["entries"])
        assert ctd.tuning_load() == len(keys)
        ctd.tuning_clear()
        ctd.tuning_load()


@pytest.mark.parametrize("n,s", [(7, 2), (37, 1), (64, 2), (129, 3)])
def test_axis_fast_diag_against_scipy(n, s):
    """The library's host eigen-decomposition for the fast-diagonalisation
    solve: V^T M V = I, V^T K V = diag(mu), and mu against scipy's symmetric-
    definite eigenvalues (an independent LAPACK implementation)."""
    import numpy as np
    import scipy.linalg as sla
    from paper_2410_15519_amd import ctd
    from oracle.cfe1d import Axis
    V = np.zeros((n, n))
    mu = np.zeros(n)
    rc = ctd.LIB.ctd_axis_fast_diag(n, 0.0, 1.0, s, min(s, 2), 12.0, 5,
                                    V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    ax = Axis(n, 0.0, 1.0, s=s, p=min(s, 2), a=12.0, ng=5)
    assert np.abs(V.T @ ax.M @ V - np.eye(n)).max() < 1e-12
    D = V.T @ ax.K @ V
    assert np.abs(D - np.diag(mu)).max() < 1e-12 * np.abs(mu).max()
    ref = sla.eigh(ax.K, ax.M, eigvals_only=True)
    assert np.abs(np.sort(mu) - ref).max() < 1e-12 * np.abs(ref).max()
    # the solve it enables equals a banded solve
    al, be = 5002.0, 2.5e-5
    b = np.random.default_rng(n).standard_normal(n)
    x = V @ ((V.T @ b) / (al + be * mu))
    ref = sla.solveh_banded(ax.banded(al * ax.M + be * ax.K), b, lower=True)
    assert np.linalg.norm(x - ref) < 1e-12 * np.linalg.norm(ref)
