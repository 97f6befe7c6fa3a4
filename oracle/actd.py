"""Adaptive CTD (ACTD) time step, 2D -- oracle, test infrastructure only.

Sec. 3.3 (adaptive algorithm): the CTD enrichment of a time step runs as
long as the mode count stays within the critical value M_c; a step that
would need more than M_c modes is computed instead by the full CFE solve of
the same scheme (the tensor-product CFE system of eq.
AC-discrete-semi-stable-K, `fullgrid.full_step`), and the time integration
goes on from that field.  Readings:
  * "needs more than M_c modes" is the cap condition of the CTD step: M_c
    modes appended and the last one still above the enrichment tolerance
    (stop == "cap"); the CTD modes of that step are discarded;
  * the field u^{k+1} of a full step enters the next step's CTD in separated
    form with one mode per node of axis 1: column j of the nodal field times
    the nodal unit vector e_j (amplitude 1).  That is the field itself, not
    an approximation of it, so the next step's integrals are unchanged;
  * M_c is the problem's max_modes.

The replayed form takes, per step, either a list of sweep counts (a CTD
step) or the string "full".
"""
from __future__ import annotations

import numpy as np

from .ctd import State, StepLog, ctd_step, full_field
from .fullgrid import full_matrices, full_step


def field_state(U: np.ndarray) -> State:
    """Separated form of a 2D nodal field: mode j = U[:, j] (x) e_j."""
    if U.ndim != 2:
        raise ValueError("field states are 2D")
    n1 = U.shape[1]
    return State(np.ones(n1), [np.array(U, dtype=np.float64), np.eye(n1)])


def actd_step(prob, state_k: State, step_index: int, replay=None, mats=None):
    """One ACTD step.  Returns (State u^{k+1}, StepLog); StepLog.stop is
    "full" when the step was the full CFE solve."""
    if prob.dim != 2:
        raise ValueError("ACTD full-solve fallback: 2D only")
    if replay is None:
        new, log = ctd_step(prob, state_k, step_index)
        if log.stop != "cap":
            return new, log
    elif not isinstance(replay, str):
        return ctd_step(prob, state_k, step_index, replay=replay)
    elif replay != "full":
        raise ValueError("replay entry must be a list of sweep counts or 'full'")
    Kf, Mf = mats if mats is not None else full_matrices(prob)
    U = full_step(prob, full_field(state_k), Kf, Mf)
    return field_state(U), StepLog(stop="full")


def actd_run(prob, state0: State, steps: int, replay=None, first_step=0):
    """Advance `steps` ACTD steps; returns (final state, logs, fields)."""
    mats = full_matrices(prob)
    st = state0
    logs, fields = [], []
    for k in range(steps):
        rp = None if replay is None else replay[k]
        st, lg = actd_step(prob, st, first_step + k, replay=rp, mats=mats)
        logs.append(lg)
        fields.append(full_field(st))
    return st, logs, fields


def decisions(logs):
    """Replay form of a run's decisions: sweep counts per mode, or "full"."""
    return ["full" if lg.stop == "full" else list(lg.iters) for lg in logs]
