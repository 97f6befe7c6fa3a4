"""GPU parity of the reduced integration domain of the 2D M_xy (Sec. 3.3,
eq. MxyRD): with rd_tol > 0 the elements whose Gauss-point values of
w(u^k) all satisfy |w| <= rd_tol leave the integral.  The HIP path decides
per element from its FP64 Gauss-grid strip, the oracle from its FP64 field;
the tolerances are placed strictly between element maxima (relative gap
checked on the oracle's values) so that both take the same decisions.
Tolerances on the results as for the full integral: 1e-10 (FP64 steps),
1e-6 (mixed steps), 1e-12 / 2e-6 for the load alone.
"""
import numpy as np
import pytest

from oracle.ctd import FullGridNonlinear, ctd_step, element_wmax, full_field, state_from_instance
from oracle.scheme import problem_from_instance
from workloads import small_instance

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}
GAP = 1e-6          # smallest relative distance of an element maximum from rd_tol


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gauss_field(pr, st):
    hats = [np.asarray(pr.axes[d].Phi @ st.factors[d]) for d in range(2)]
    return (hats[0] * st.sigma) @ hats[1].T


def tol_between(wmax, q0, q1):
    """A tolerance in the middle of the widest relative gap between
    consecutive element maxima, among those from quantile q0 to q1."""
    w = np.unique(wmax.ravel())
    k0, k1 = int(q0 * (len(w) - 1)), int(q1 * (len(w) - 1))
    gaps = (w[k0 + 1:k1 + 1] - w[k0:k1]) / w[k0 + 1:k1 + 1]
    k = k0 + int(np.argmax(gaps))
    return 0.5 * (w[k] + w[k + 1])


def margin(wmax, tol):
    return float(np.min(np.abs(wmax - tol)) / tol)


@pytest.mark.parametrize("n,prec", [((45, 38), "fp64"), ((45, 38), "mixed"),
                                    ((900, 1000), "fp64")])
def test_reduced_load_matches_oracle(ctd, n, prec):
    """The 2D load F_d = M_xy u_e with the reduced domain, and the number of
    elements left out.  900 x 1000 nodes: the Gauss grid is built in six
    strips of whole elements, the last one ragged."""
    inst = small_instance(dim=2, n=n, m0=4, kmax=4)
    pr0 = problem_from_instance(inst)
    st = state_from_instance(inst)
    wmax = element_wmax(pr0, gauss_field(pr0, st))
    tol = tol_between(wmax, 0.3, 0.6)
    assert margin(wmax, tol) > GAP
    pr = problem_from_instance(inst, rd_tol=tol)
    F = FullGridNonlinear(pr, st)
    assert 0 < F.excluded < wmax.size
    rng = np.random.default_rng(5)
    u = [rng.uniform(-1, 1, inst.nodes[d]) for d in range(2)]
    print(f"reduced load n={n} prec={prec} tol={tol:.3e} excluded={F.excluded}/{wmax.size}", flush=True)
    with ctd.Solver(inst, precision=prec, rd_tol=tol) as s:
        assert s.reduced_domain_excluded() == F.excluded
        for d in range(2):
            got = s.nonlinear_load(d, u)
            err = rel(got, F(d, u))
            print(f"  load d={d}: {err:.2e}", flush=True)
            assert err < (1e-12 if prec == "fp64" else 2e-6)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_reduced_step_replay_parity(ctd, prec):
    """Time steps with the reduced domain against the oracle's, the oracle's
    decisions replayed; the element count left out agrees for every state
    (the library builds the next step's M_xy at the end of a step)."""
    inst = small_instance(dim=2, n=37, m0=3, kmax=4, eps=0.05, dt=1e-3, max_modes=24)
    pr0 = problem_from_instance(inst)
    tol = tol_between(element_wmax(pr0, gauss_field(pr0, state_from_instance(inst))), 0.2, 0.5)
    pr = problem_from_instance(inst, rd_tol=tol)
    st = state_from_instance(inst)
    steps = 3
    fields, logs, counts = [], [], []
    for k in range(steps + 1):
        wmax = element_wmax(pr, gauss_field(pr, st))
        assert margin(wmax, tol) > GAP
        counts.append(int((wmax <= tol).sum()))
        if k == steps:
            break
        st, lg = ctd_step(pr, st, k)
        fields.append(full_field(st))
        logs.append(lg)
    assert all(0 < c < wmax.size for c in counts)
    print(f"reduced replay prec={prec} tol={tol:.3e} excluded={counts}", flush=True)
    with ctd.Solver(inst, precision=prec, schedule="replay", rd_tol=tol) as s:
        s.set_decisions([lg.iters for lg in logs])
        assert s.reduced_domain_excluded() == counts[0]
        for k in range(steps):
            info = s.step(1)[0]
            assert s.reduced_domain_excluded() == counts[k + 1]
            assert info["modes"] == len(logs[k].iters)
            err = rel(s.reconstruct(), fields[k])
            print(f"  step {k}: rel l2 = {err:.3e}", flush=True)
            assert err < TOL[prec]


def test_zero_tolerance_is_the_full_integral(ctd):
    """rd_tol = 0 leaves nothing out and reports no element."""
    inst = small_instance(dim=2, n=37, m0=3, kmax=4)
    with ctd.Solver(inst, rd_tol=0.0) as a, ctd.Solver(inst) as b:
        a.step(2)
        b.step(2)
        assert a.reduced_domain_excluded() == 0
        assert np.array_equal(a.reconstruct(), b.reconstruct())


@pytest.mark.parametrize("executor", ["lockstep", "streams"])
def test_reduced_batch_equals_standalone(ctd, executor):
    """Batched instances with the reduced domain step exactly as standalone
    ones (each instance builds its own masked M_xy)."""
    from workloads import make_batch
    insts = make_batch(seed=13, count=4, nodes_range=(24, 120), max_modes=10)
    tol = 0.05
    b = ctd.Batch(insts, precision="fp64", rd_tol=tol)
    try:
        b.set_mode(executor)
        b.set_workers(3)
        b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i, inst in enumerate(insts):
        with ctd.Solver(inst, precision="fp64", rd_tol=tol) as s:
            s.step(2)
            assert s.reduced_domain_excluded() > 0
            amp, fac = s.modes()
        assert np.array_equal(got[i][0], amp) and all(np.array_equal(x, y) for x, y in zip(got[i][1], fac))
