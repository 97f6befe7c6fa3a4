"""GPU parity of the adaptive algorithm's full-solve fallback (Sec. 3.3, 2D):
the full tensor-product CFE step in the eigenbases (FP64 MFMA products), the
switch past the mode cap, CTD steps from the resulting field state, and the
energy of field states.  Oracle: `oracle.actd` (dense full solve on tiny
grids) and the full-system residual at sizes the dense solve cannot reach.
Tolerances: 1e-10 FP64, 1e-6 mixed (relative nodal l2), as for CTD steps.
"""
import numpy as np
import pytest

from oracle.actd import actd_run, decisions
from oracle.ctd import full_field, state_from_instance
from oracle.energy import energy_fullgrid
from oracle.fullgrid import nonlinear_load
from oracle.scheme import problem_from_instance
from workloads import small_instance

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


def _inst(n=(13, 10), cap=6, kmax=4):
    return small_instance(dim=2, n=n, m0=3, kmax=kmax, eps=0.05, dt=1e-3, max_modes=cap)


@pytest.mark.parametrize("n", [(13, 10), (70, 45)])
@pytest.mark.parametrize("solve", ["auto", "fd"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_actd_replay_parity(ctd, n, solve, prec):
    """Schedule full / CTD from the field state / full / CTD: every step's
    field against the oracle's."""
    inst = _inst(n=n)
    pr = problem_from_instance(inst)
    sched = ["full", [3, 2, 2, 3], "full", [2, 2]]
    _, logs, fields = actd_run(pr, state_from_instance(inst), len(sched), replay=sched)
    print(f"actd replay n={n} solve={solve} prec={prec}", flush=True)
    with ctd.Solver(inst, precision=prec, schedule="replay", solve=solve, actd=True) as s:
        s.set_decisions(sched)
        dec = []
        for k, sc in enumerate(sched):
            info = s.step(1)[0]
            dec += s.decisions()   # the log of the last ctd_step call
            assert info["full_solve"] == (1 if sc == "full" else 0)
            assert info["modes"] == (n[1] if sc == "full" else len(sc))
            err = rel(s.reconstruct(), fields[k])
            print(f"  step {k} ({'full' if sc == 'full' else 'ctd'}): rel l2 = {err:.3e}", flush=True)
            assert err < TOL[prec]
        assert dec == sched


@pytest.mark.parametrize("cap", [6, 7])
def test_actd_adaptive_decisions(ctd, cap):
    """Adaptive run: the switch happens exactly where the oracle's does."""
    inst = _inst(n=(17, 12), cap=cap)
    pr = problem_from_instance(inst)
    _, logs, fields = actd_run(pr, state_from_instance(inst), 3)
    with ctd.Solver(inst, precision="fp64", actd=True) as s:
        infos = s.step(3)
        assert s.decisions() == decisions(logs)
        assert [i["full_solve"] for i in infos] == [int(lg.stop == "full") for lg in logs]
        assert rel(s.reconstruct(), fields[-1]) < 1e-10


def test_actd_energy_of_field_states(ctd):
    """Energy of a field state (one mode per node: the direct Gauss-grid
    route) against the full-grid energy of the oracle's field."""
    inst = _inst(n=(21, 16), cap=6)
    pr = problem_from_instance(inst)
    _, logs, fields = actd_run(pr, state_from_instance(inst), 2)
    with ctd.Solver(inst, precision="fp64", actd=True, energy=True) as s:
        infos = s.step(2)
        for k in range(2):
            assert infos[k]["full_solve"] == 1
            ref = energy_fullgrid(pr, fields[k])
            assert infos[k]["energy"] == pytest.approx(ref, rel=1e-12)
        assert infos[1]["energy"] <= infos[0]["energy"]


def test_actd_full_solve_residual_large(ctd):
    """Full step at 512 x 300 nodes (several MFMA tiles, ragged tails), where
    the dense oracle solve is out of reach: the nodal field must satisfy the
    tensor system (c M0 (x) M1 + lam (K0 (x) M1 + M0 (x) K1)) U = c M0 U^k M1 - F
    with F the oracle's full-grid nonlinear load of u^k."""
    inst = _inst(n=(512, 300), cap=2, kmax=6)
    pr = problem_from_instance(inst)
    Uk = full_field(state_from_instance(inst))
    with ctd.Solver(inst, precision="fp64", schedule="replay", actd=True) as s:
        s.set_decisions(["full"])
        s.step(1)
        U = s.reconstruct()
    ax = pr.axes
    M0, M1, K0, K1 = ax[0].M, ax[1].M, ax[0].K, ax[1].K
    lhs = pr.c * (M0 @ (M1 @ U.T).T) + pr.lam * (K0 @ (M1 @ U.T).T + M0 @ (K1 @ U.T).T)
    F = nonlinear_load(pr, Uk)
    Q = pr.c * (M0 @ (M1 @ Uk.T).T) - F
    err = rel(lhs, Q)
    print(f"  residual {err:.2e}", flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mxy_strips_nonlinear_load(ctd, prec):
    """2D nonlinear load with the Gauss-grid integrand built in several
    strips (1100 x 900 nodes: 5495 x 4495 Gauss points, a ragged last
    strip) against the oracle's full-grid integral."""
    from oracle.ctd import FullGridNonlinear
    inst = small_instance(dim=2, n=(1100, 900), m0=5, kmax=6)
    pr = problem_from_instance(inst)
    rng = np.random.default_rng(11)
    u = [rng.uniform(-1, 1, n) for n in (1100, 900)]
    F = FullGridNonlinear(pr, state_from_instance(inst))
    with ctd.Solver(inst, precision=prec) as s:
        for d in range(2):
            err = rel(s.nonlinear_load(d, u), F(d, u))
            print(f"  strips load d={d}: {err:.2e}", flush=True)
            assert err < (1e-12 if prec == "fp64" else 2e-6)


def test_actd_in_batch_equals_standalone(ctd):
    """Instances that switch to the full solve, stepped concurrently on
    worker streams, end bitwise where each alone does."""
    insts = [_inst(n=(17 + 6 * k, 12 + 3 * k), cap=6 if k % 2 == 0 else 7) for k in range(4)]
    b = ctd.Batch(insts, precision="fp64", actd=True)
    try:
        b.set_workers(4)
        b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i, inst in enumerate(insts):
        with ctd.Solver(inst, precision="fp64", actd=True) as s:
            s.step(2)
            amp, fac = s.modes()
        assert np.array_equal(got[i][0], amp), f"instance {i}"
        assert all(np.array_equal(x, y) for x, y in zip(got[i][1], fac)), f"instance {i}"


# ---------------------------------------------------------------- 3D
# The 3D fallback: the full step in the eigenbases (FP64 MFMA mode
# products), the field state held as the nodal tensor with its right-hand-
# side tensor R = c M3 U - int N w(U) (Gauss-grid passes), and CTD steps
# from it (the load of a directional solve = R contracted with the other two
# factors).  The oracle holds the field state as n1 n2 fibres and uses the
# counter-based guess for its modes (it has no modes to warm-start from).

def _inst3(n=(13, 11, 9), cap=3, kmax=3):
    return small_instance(dim=3, n=n, m0=2, kmax=kmax, eps=0.08, dt=1e-3, max_modes=cap)


@pytest.mark.parametrize("solve", ["auto", "bcr"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_actd3d_replay_parity(ctd, prec, solve):
    """Schedule full / CTD from the field state / full / CTD in 3D: every
    step's field against the oracle's (directional solves by fast
    diagonalisation or by cyclic reduction: both add the field state's load
    chunks)."""
    inst = _inst3()
    pr = problem_from_instance(inst)
    sched = ["full", [3, 2, 2], "full", [2, 3]]
    _, logs, fields = actd_run(pr, state_from_instance(inst), len(sched), replay=sched)
    print(f"actd 3D replay prec={prec} solve={solve}", flush=True)
    with ctd.Solver(inst, precision=prec, schedule="replay", actd=True, solve=solve) as s:
        s.set_decisions(sched)
        dec = []
        for k, sc in enumerate(sched):
            info = s.step(1)[0]
            dec += s.decisions()
            assert info["full_solve"] == (1 if sc == "full" else 0)
            assert info["modes"] == (0 if sc == "full" else len(sc))
            err = rel(s.reconstruct(), fields[k])
            print(f"  step {k} ({'full' if sc == 'full' else 'ctd'}): rel l2 = {err:.3e}", flush=True)
            assert err < TOL[prec]
        assert dec == sched


def test_actd3d_adaptive_decisions_and_energy(ctd):
    """Adaptive 3D run: the switches happen where the oracle's do, the fields
    agree, and the energy of every state (field states on the Gauss grid)
    equals the oracle's full-grid energy and does not increase."""
    inst = _inst3(n=(12, 10, 9), cap=3)
    pr = problem_from_instance(inst, init="warm")
    _, logs, fields = actd_run(pr, state_from_instance(inst), 3)
    print(f"actd 3D adaptive: oracle decisions {decisions(logs)}", flush=True)
    assert "full" in decisions(logs)
    with ctd.Solver(inst, precision="fp64", actd=True, energy=True) as s:
        infos = s.step(3)
        assert s.decisions() == decisions(logs)
        assert rel(s.reconstruct(), fields[-1]) < 1e-10
        for k in range(3):
            assert infos[k]["energy"] == pytest.approx(energy_fullgrid(pr, fields[k]), rel=1e-12)
        assert all(infos[k + 1]["energy"] <= infos[k]["energy"] for k in range(2))
        # the field state in separated form: n1 n2 fibres of the field
        if infos[-1]["full_solve"]:
            amp, fac = s.modes()
            U = np.einsum("m,im,jm,km->ijk", amp, *fac)
            assert np.array_equal(U, s.reconstruct())


def test_actd3d_full_solve_residual(ctd):
    """Two full steps at 40 x 33 x 27 nodes (ragged MFMA tiles; beyond the
    dense oracle solve): each field must satisfy the tensor system
    (c M3 + lam (K0 (x) M1 (x) M2 + M0 (x) K1 (x) M2 + M0 (x) M1 (x) K2)) U
      = c M3 U^k - F(U^k),
    F the oracle's tensor-Gauss-grid nonlinear load; the second step starts
    from the field state of the first (its right-hand-side tensor)."""
    inst = _inst3(n=(40, 33, 27), cap=2, kmax=5)
    pr = problem_from_instance(inst)
    ax = pr.axes

    def apply(mats, U):
        for d in range(3):
            U = np.moveaxis(np.tensordot(mats[d], U, axes=([1], [d])), 0, d)
        return U

    Ms = [a.M for a in ax]
    Uk = full_field(state_from_instance(inst))
    with ctd.Solver(inst, precision="fp64", schedule="replay", actd=True) as s:
        s.set_decisions(["full", "full"])
        for k in range(2):
            s.step(1)
            U = s.reconstruct()
            lhs = pr.c * apply(Ms, U)
            for d in range(3):
                lhs = lhs + pr.lam * apply([ax[e].K if e == d else ax[e].M for e in range(3)], U)
            Q = pr.c * apply(Ms, Uk) - nonlinear_load(pr, Uk)
            err = rel(lhs, Q)
            print(f"  full step {k}: residual {err:.2e}", flush=True)
            assert err < 1e-12
            Uk = U


def test_actd3d_in_batch_equals_standalone(ctd):
    """3D instances that switch to the full solve and step from the field
    state, on worker streams, end bitwise where each alone does (the field
    state read back as its fibres)."""
    insts = [_inst3(n=(12 + 2 * k, 10 + k, 9), cap=3) for k in range(3)]
    b = ctd.Batch(insts, precision="mixed", actd=True)
    try:
        b.set_workers(3)
        infos = b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    assert any(r["full_solve"] for inf in infos for r in inf)
    for i, inst in enumerate(insts):
        with ctd.Solver(inst, precision="mixed", actd=True) as s:
            s.step(2)
            amp, fac = s.modes()
        assert np.array_equal(got[i][0], amp), f"instance {i}"
        assert all(np.array_equal(x, y) for x, y in zip(got[i][1], fac)), f"instance {i}"
