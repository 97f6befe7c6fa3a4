"""Pins of the ACTD oracle (Sec. 3.3 adaptive algorithm, 2D and 3D): the
separated form of a nodal field, the switch to the full CFE solve past the
mode cap, and the scheme's energy law along a run that switches."""
import numpy as np
import pytest

from oracle import actd
from oracle.actd import actd_run, actd_step, field_state
from oracle.ctd import ctd_step, full_field, state_from_instance
from oracle.energy import energy_fullgrid
from oracle.fullgrid import full_step
from oracle.scheme import problem_from_instance
from workloads import small_instance


def _inst(n=(13, 10), cap=6, **kw):
    return small_instance(dim=2, n=n, m0=3, kmax=4, eps=0.05, dt=1e-3, max_modes=cap, **kw)


def test_field_state_is_the_field():
    rng = np.random.default_rng(0)
    U = rng.standard_normal((9, 14))
    st = field_state(U)
    assert st.modes == 14
    assert np.array_equal(full_field(st), U)


def test_ctd_step_from_field_state_equals_step_from_modes():
    """The CTD integrals of u^k depend on the field only: the same step from
    the 3-mode state and from its 10-mode field form agree to rounding.  The
    counter-based initial guess of a mode is used: it does not depend on the
    modes of u^k (the warm guess takes mode m of u^k, which differs between
    the two forms of the same field)."""
    inst = _inst(cap=32)
    pr = problem_from_instance(inst, init="hash")
    st = state_from_instance(inst)
    new_a, log_a = ctd_step(pr, st, 0)
    assert log_a.stop == "tol"
    fs = field_state(full_field(st))
    new_b, _ = ctd_step(pr, fs, 0, replay=log_a.iters)
    a, b = full_field(new_a), full_field(new_b)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-11


def test_switch_past_the_cap_gives_the_full_solve():
    inst = _inst(cap=6)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    _, log_ctd = ctd_step(pr, st, 0)
    assert log_ctd.stop == "cap"
    new, log = actd_step(pr, st, 0)
    assert log.stop == "full" and log.iters == []
    ref = full_step(pr, full_field(st))
    assert np.array_equal(full_field(new), ref)


def test_no_switch_within_the_cap():
    inst = _inst(cap=7)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    a, la = ctd_step(pr, st, 0)
    b, lb = actd_step(pr, st, 0)
    assert la.stop == "tol" and lb.stop == "tol" and la.iters == lb.iters
    assert np.array_equal(full_field(a), full_field(b))


def test_replay_mixes_full_and_ctd_steps():
    """Replayed schedule full / CTD from the field / full from a CTD state:
    each CTD step from a field state equals the CTD step from the same field
    held as modes (the field after a CTD step), so the run is consistent
    (counter-based initial guess: independent of how u^k is held)."""
    inst = _inst(cap=6)
    pr = problem_from_instance(inst, init="hash")
    sched = ["full", [3, 2, 2, 3], "full", [2, 2]]
    st, logs, fields = actd_run(pr, state_from_instance(inst), 4, replay=sched)
    assert actd.decisions(logs) == sched
    assert st.modes == 2
    # step 1 from the field state of step 0 == from that field's SVD modes
    U0 = fields[0]
    u, sv, vt = np.linalg.svd(U0, full_matrices=False)
    r = int(np.sum(sv > 1e-14 * sv[0]))
    from oracle.ctd import State
    st_svd = State(sv[:r].copy(), [u[:, :r].copy(), vt[:r].T.copy()])
    b, _ = ctd_step(pr, st_svd, 1, replay=sched[1])
    assert np.linalg.norm(full_field(b) - fields[1]) / np.linalg.norm(fields[1]) < 1e-10


@pytest.mark.parametrize("cap", [6, 7])
def test_actd_energy_law(cap):
    """The stabilized scheme's discrete energy does not increase along the
    run (eq. AC-discrete-semi-stable-step), with and without switches."""
    inst = _inst(n=(15, 12), cap=cap)
    pr = problem_from_instance(inst)
    st0 = state_from_instance(inst)
    _, logs, fields = actd_run(pr, st0, 4)
    E = [energy_fullgrid(pr, full_field(st0))] + [energy_fullgrid(pr, U) for U in fields]
    assert all(E[i + 1] <= E[i] * (1 + 1e-12) for i in range(len(E) - 1))
    assert {lg.stop for lg in logs} == ({"full"} if cap == 6 else {"tol"})


def test_planted_field_transpose_caught(monkeypatch):
    """A field state built from the transposed field (square grid) changes
    the next step: the comparison above must catch it."""
    inst = _inst(n=(11, 11), cap=32)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    new_a, log_a = ctd_step(pr, st, 0)
    bad = field_state(full_field(st).T)
    new_b, _ = ctd_step(pr, bad, 0, replay=log_a.iters)
    a, b = full_field(new_a), full_field(new_b)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) > 1e-6


def _inst3(n=(8, 7, 6), cap=4, **kw):
    return small_instance(dim=3, n=n, m0=2, kmax=3, eps=0.08, dt=1e-3, max_modes=cap, **kw)


def test_field_state_3d_is_the_field():
    rng = np.random.default_rng(1)
    U = rng.standard_normal((6, 5, 4))
    st = field_state(U)
    assert st.modes == 20 and st.warm_modes == 0
    assert np.array_equal(full_field(st), U)


def test_ctd_step_from_3d_field_state_equals_step_from_modes():
    """3D: the step's integrals depend on the field only, so the step from
    the 2-mode state and from its 42-fibre field form agree to rounding
    (counter-based guess on both sides)."""
    inst = _inst3(cap=24)
    pr = problem_from_instance(inst, init="hash")
    st = state_from_instance(inst)
    new_a, log_a = ctd_step(pr, st, 0)
    assert log_a.stop == "tol"
    new_b, _ = ctd_step(pr, field_state(full_field(st)), 0, replay=log_a.iters)
    a, b = full_field(new_a), full_field(new_b)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-11


def test_warm_guess_from_3d_field_state_is_the_counter_based_one():
    """A 3D field state holds no modes to start from: the warm reading gives
    the counter-based initial guess for every mode (bitwise the same step)."""
    inst = _inst3(cap=24)
    U = full_field(state_from_instance(inst))
    a, la = ctd_step(problem_from_instance(inst, init="warm"), field_state(U), 3)
    b, lb = ctd_step(problem_from_instance(inst, init="hash"), field_state(U), 3)
    assert la.iters == lb.iters
    assert np.array_equal(full_field(a), full_field(b))


def test_switch_past_the_cap_gives_the_full_solve_3d():
    inst = _inst3(cap=3)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    _, log_ctd = ctd_step(pr, st, 0)
    assert log_ctd.stop == "cap"
    new, log = actd_step(pr, st, 0)
    assert log.stop == "full"
    assert np.array_equal(full_field(new), full_step(pr, full_field(st)))
    assert new.warm_modes == 0


def test_actd_3d_replay_and_energy_law():
    """3D run replaying full / CTD from the field / full: each CTD step from
    the field state equals the same step from the field's original-mode
    form, and the discrete energy does not increase (Sec. 2.5)."""
    inst = _inst3(cap=3)
    pr = problem_from_instance(inst, init="hash")
    st0 = state_from_instance(inst)
    sched = ["full", [3, 2, 2], "full"]
    st, logs, fields = actd_run(pr, st0, 3, replay=sched)
    assert actd.decisions(logs) == sched
    E = [energy_fullgrid(pr, full_field(st0))] + [energy_fullgrid(pr, U) for U in fields]
    assert all(E[i + 1] <= E[i] * (1 + 1e-12) for i in range(len(E) - 1))
    # the full steps are the full CFE solve of the previous field
    assert np.allclose(fields[0], full_step(pr, full_field(st0)), rtol=0, atol=1e-15)
    assert np.allclose(fields[2], full_step(pr, fields[1]), rtol=0, atol=1e-15)


def test_planted_3d_fibre_order_caught():
    """A 3D field state whose fibres are taken with axes 1 and 2 swapped is a
    different field: the step-from-field comparison above must catch it."""
    inst = _inst3(n=(8, 7, 7), cap=24)
    pr = problem_from_instance(inst, init="hash")
    st = state_from_instance(inst)
    new_a, log_a = ctd_step(pr, st, 0)
    bad = field_state(full_field(st).transpose(0, 2, 1))
    new_b, _ = ctd_step(pr, bad, 0, replay=log_a.iters)
    a, b = full_field(new_a), full_field(new_b)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) > 1e-6
