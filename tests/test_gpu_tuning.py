"""The split-count table of the 3D cubic contraction (ctd_tuning_set): a
handle picks up an entry for its shape, and the projected load stays within
the mixed and FP64 tolerances of the oracle for any split counts (they only
change the summation order)."""
import numpy as np
import pytest

from workloads import small_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 1e-6)])
@pytest.mark.parametrize("splits", [(1, 1), (3, 2), (8, 5), (16, 40)])
def test_tuned_splits_keep_the_load(ctd, prec, tol, splits):
    from oracle.ctd import SeparatedNonlinear, state_from_instance
    from oracle.scheme import problem_from_instance
    inst = small_instance(3, (33, 41, 29), m0=40, kmax=5, max_modes=40)
    ref_of = SeparatedNonlinear(problem_from_instance(inst), state_from_instance(inst))
    rng = np.random.default_rng(5)
    u = [rng.uniform(-1, 1, n) for n in inst.nodes]
    nq = min((n - 1) * 5 for n in inst.nodes)
    nb = (40 + 15) // 16
    try:
        ctd.tuning_set(nb, nq, *splits, precision=prec)
        with ctd.Solver(inst, precision=prec) as s:
            for d in range(3):
                got = s.nonlinear_load(d, u)
                g, h = s.tuning_current()
                # clamped to the chunks of the smallest axis, the allocation and
                # the triple count
                assert 1 <= g <= splits[0] and 1 <= h <= splits[1]
                ref = ref_of(d, u)
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                print(f"splits {splits} -> ({g}, {h}) {prec} d={d}: {err:.2e}", flush=True)
                assert err < tol
    finally:
        ctd.tuning_clear()
        ctd.tuning_load()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 1e-6)])
def test_many_h_splits_keep_the_load(ctd, prec, tol):
    """More h splits than the balanced split table holds (84 triples at 112
    modes, 80 splits): the equal-count triple ranges, against the oracle."""
    from oracle.ctd import SeparatedNonlinear, state_from_instance
    from oracle.scheme import problem_from_instance
    inst = small_instance(3, (21, 19, 17), m0=112, kmax=7, max_modes=112)
    ref_of = SeparatedNonlinear(problem_from_instance(inst), state_from_instance(inst))
    rng = np.random.default_rng(11)
    u = [rng.uniform(-1, 1, n) for n in inst.nodes]
    nq = min((n - 1) * 5 for n in inst.nodes)
    nb = (112 + 15) // 16
    try:
        ctd.tuning_set(nb, nq, 2, 80, precision=prec)
        with ctd.Solver(inst, precision=prec) as s:
            for d in range(3):
                got = s.nonlinear_load(d, u)
                g, h = s.tuning_current()
                assert h == 80
                ref = ref_of(d, u)
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                print(f"80 h splits {prec} d={d}: {err:.2e}", flush=True)
                assert err < tol
    finally:
        ctd.tuning_clear()
        ctd.tuning_load()
