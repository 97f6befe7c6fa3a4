"""Adaptive CTD (ACTD) time step, 2D and 3D -- oracle, test infrastructure only.

Sec. 3.3 (adaptive algorithm): the CTD enrichment of a time step runs as
long as the mode count stays within the critical value M_c; a step that
would need more than M_c modes is computed instead by the full CFE solve of
the same scheme (the tensor-product CFE system of eq.
AC-discrete-semi-stable-K, `fullgrid.full_step`), and the time integration
goes on from that field (Sec. 4.2 runs it in 3D with M_c = 200).  Readings:
  * "needs more than M_c modes" is the cap condition of the CTD step: M_c
    modes appended and the last one still above the enrichment tolerance
    (stop == "cap"); the CTD modes of that step are discarded;
  * the field u^{k+1} of a full step enters the next step's CTD as the field
    itself, written in separated form: 2D, one mode per node of axis 1
    (column j of the nodal field times the nodal unit vector e_j, amplitude
    1); 3D, one mode per node pair (j, k) of axes 1 and 2 (the fibre
    U[:, j, k] times e_j times e_k).  The next step's integrals are those of
    the field, not of an approximation of it;
  * the warm initial guess takes mode m of u^k as u^k is held: a 2D field
    state holds its columns as modes; a 3D field state (n_1 n_2 fibres) is
    held as a field, with no modes to start from, so every mode of the next
    step starts from the counter-based vector;
  * M_c is the problem's max_modes.

The replayed form takes, per step, either a list of sweep counts (a CTD
step) or the string "full".
"""
from __future__ import annotations

import numpy as np

from .ctd import State, StepLog, ctd_step, full_field
from .fullgrid import full_matrices, full_step


def field_state(U: np.ndarray) -> State:
    """Separated form of a nodal field.  2D: mode j = U[:, j] (x) e_j.  3D:
    mode j n_2 + k = U[:, j, k] (x) e_j (x) e_k, held with no warm modes."""
    if U.ndim == 2:
        n1 = U.shape[1]
        return State(np.ones(n1), [np.array(U, dtype=np.float64), np.eye(n1)])
    if U.ndim != 3:
        raise ValueError("field states are 2D or 3D")
    n0, n1, n2 = U.shape
    X0 = np.array(U, dtype=np.float64).reshape(n0, n1 * n2)
    X1 = np.repeat(np.eye(n1), n2, axis=1)      # column j n2 + k = e_j
    X2 = np.tile(np.eye(n2), (1, n1))           # column j n2 + k = e_k
    return State(np.ones(n1 * n2), [X0, X1, X2], warm=0)


def actd_step(prob, state_k: State, step_index: int, replay=None, mats=None):
    """One ACTD step.  Returns (State u^{k+1}, StepLog); StepLog.stop is
    "full" when the step was the full CFE solve."""
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
