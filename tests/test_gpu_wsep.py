"""GPU parity of the separated integration of the 2D M_xy (Sec. 3.3, eq.
MxySep): L w(u^k) on the Gauss grid replaced by w_rank greedy rank-one
terms, each from w_iters alternating least-squares updates, and M_xy formed
from products of 1D integrals.  Both sides run the same iteration from the
same counter-based start (a contraction: rounding differences do not grow),
so the results are compared at the tolerances of the full integral: 1e-12
(FP64 load), 1e-10 / 1e-6 (FP64 / mixed steps), 2e-6 (mixed load).
"""
import numpy as np
import pytest

from oracle.ctd import FullGridNonlinear, ctd_step, full_field, state_from_instance
from oracle.scheme import problem_from_instance
from workloads import make_batch, small_instance

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,rank,iters,prec", [((45, 38), 3, 40, "fp64"), ((45, 38), 3, 40, "mixed"),
                                               ((300, 260), 5, 25, "fp64"), ((70, 66), 12, 8, "fp64"),
                                               ((6, 7), 40, 6, "fp64")])
def test_separated_load_matches_oracle(ctd, n, rank, iters, prec):
    """The 2D load F_d = M_xy u_e with the separated M_xy (the last case asks
    for more terms than the 25 x 30 Gauss grid has rank)."""
    inst = small_instance(dim=2, n=n, m0=4, kmax=4)
    pr = problem_from_instance(inst, w_rank=rank, w_iters=iters)
    F = FullGridNonlinear(pr, state_from_instance(inst))
    rng = np.random.default_rng(9)
    u = [rng.uniform(-1, 1, inst.nodes[d]) for d in range(2)]
    print(f"separated load n={n} rank={rank} iters={iters} prec={prec}", flush=True)
    with ctd.Solver(inst, precision=prec, w_rank=rank, w_iters=iters) as s:
        for d in range(2):
            err = rel(s.nonlinear_load(d, u), F(d, u))
            print(f"  load d={d}: {err:.2e}", flush=True)
            assert err < (1e-12 if prec == "fp64" else 2e-6)


def test_two_terms_of_a_one_mode_state_are_the_full_integral(ctd):
    """L w of a one-mode state has rank two: the separated load with two
    terms equals the library's full-integral load."""
    inst = small_instance(dim=2, n=(40, 34), m0=1, kmax=2)
    rng = np.random.default_rng(2)
    u = [rng.uniform(-1, 1, inst.nodes[d]) for d in range(2)]
    with ctd.Solver(inst, w_rank=2, w_iters=200) as s, ctd.Solver(inst) as f:
        for d in range(2):
            assert rel(s.nonlinear_load(d, u), f.nonlinear_load(d, u)) < 1e-11


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separated_step_replay_parity(ctd, prec):
    """Time steps with the separated M_xy against the oracle's, the oracle's
    decisions replayed."""
    inst = small_instance(dim=2, n=37, m0=3, kmax=4, eps=0.05, dt=1e-3, max_modes=24)
    pr = problem_from_instance(inst, w_rank=4, w_iters=30)
    st = state_from_instance(inst)
    fields, logs = [], []
    for k in range(3):
        st, lg = ctd_step(pr, st, k)
        fields.append(full_field(st))
        logs.append(lg)
    print(f"separated replay prec={prec} modes={[len(l.iters) for l in logs]}", flush=True)
    with ctd.Solver(inst, precision=prec, schedule="replay", w_rank=4, w_iters=30) as s:
        s.set_decisions([lg.iters for lg in logs])
        for k in range(3):
            info = s.step(1)[0]
            assert info["modes"] == len(logs[k].iters)
            err = rel(s.reconstruct(), fields[k])
            print(f"  step {k}: rel l2 = {err:.3e}", flush=True)
            assert err < TOL[prec]


def test_separated_batch_equals_standalone(ctd):
    """Batched instances with the separated M_xy step exactly as standalone."""
    insts = make_batch(seed=17, count=3, nodes_range=(24, 90), max_modes=8)
    b = ctd.Batch(insts, precision="fp64", w_rank=3, w_iters=10)
    try:
        b.set_mode("lockstep")
        b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i, inst in enumerate(insts):
        with ctd.Solver(inst, precision="fp64", w_rank=3, w_iters=10) as s:
            s.step(2)
            amp, fac = s.modes()
        assert np.array_equal(got[i][0], amp) and all(np.array_equal(x, y) for x, y in zip(got[i][1], fac))


@pytest.mark.parametrize("kw", [dict(w_rank=3, w_iters=5), dict(rd_tol=0.1)])
def test_alternatives_of_the_zero_field(ctd, kw):
    """w(0) = 0: the separated terms are zero (zero denominators) and the
    reduced domain leaves out every element; steps from the zero field stay
    zero, without NaN."""
    from workloads import Instance
    base = small_instance(dim=2, n=20, m0=2, kmax=3)
    inst = Instance(**{**base.__dict__, "amp": np.zeros_like(base.amp)})
    with ctd.Solver(inst, **kw) as s:
        if "rd_tol" in kw:
            assert s.reduced_domain_excluded() == 19 * 19
        for _ in range(2):
            info = s.step(1)[0]
            assert info["modes"] == 0 and not np.any(s.reconstruct())
        if "rd_tol" in kw:
            assert s.reduced_domain_excluded() == 19 * 19


def test_alternatives_at_the_benchmarked_shape(ctd):
    """The two alternatives at the shape the bench times them on (the 2D
    workload on 1024 x 1024 nodes, its initial field, FP64): the separated
    M_xy (8 terms, 30 updates) and the reduced domain (a tolerance in the
    widest gap between element maxima near the 3 % quantile) against the
    oracle's load, every entry; the reduced domain's element count equal."""
    from oracle.ctd import element_wmax
    from workloads import make_instance
    inst = make_instance("ac2d_n128", nodes=1024)
    st = state_from_instance(inst)
    pr0 = problem_from_instance(inst)
    hats = [np.asarray(pr0.axes[d].Phi @ st.factors[d]) for d in range(2)]
    U = (hats[0] * st.sigma) @ hats[1].T
    w = np.unique(element_wmax(pr0, U).ravel())
    del U, hats
    k0, k1 = int(0.01 * (len(w) - 1)), int(0.05 * (len(w) - 1))
    gaps = (w[k0 + 1:k1 + 1] - w[k0:k1]) / w[k0 + 1:k1 + 1]
    k = k0 + int(np.argmax(gaps))
    tol = 0.5 * (w[k] + w[k + 1])
    assert gaps.max() > 2e-6
    rng = np.random.default_rng(4)
    u = [rng.uniform(-1, 1, 1024) for _ in range(2)]
    for kw in (dict(w_rank=8, w_iters=30), dict(rd_tol=tol)):
        F = FullGridNonlinear(problem_from_instance(inst, **kw), st)
        print(f"alternative {kw} at 1024^2: oracle done (excluded {F.excluded})", flush=True)
        with ctd.Solver(inst, precision="fp64", **kw) as s:
            if "rd_tol" in kw:
                assert s.reduced_domain_excluded() == F.excluded > 0
            for d in range(2):
                err = rel(s.nonlinear_load(d, u), F(d, u))
                print(f"  load d={d}: {err:.2e}", flush=True)
                assert err < 1e-12
        del F
