"""Whole-step parity at the benchmarked 3D 256^3 shape with the mode cap reached.

The 256^3 workload (eps 0.01, dt 5e-4, 8 seeded cosine modes, cap 64, at
most 20 sweeps per mode): step 1 (M_k = 8) ends capped at 64 modes, so step
2 runs the cubic contraction at M_k = 64 (four 16-wide mode tiles, 20 tile
triples), the right-hand side with all of its column chunks up to M = 63
earlier modes, and ends capped again (Sec. 3.3 algorithm; cap = the
adaptive variant's M_c).  The oracle runs both steps adaptively on its
separated path (FP64, plain numpy) and the GPU replays its decisions, for
both readings of the initial guess of a mode.

Bars (relative nodal l2, Sec. 4.1 error metric), per step:
  * the sum of the first 16 modes (the greedy order makes this prefix a
    well-defined part of the result): FP64 1e-10, mixed 1e-6;
  * the whole field: FP64 1e-8, mixed 1e-5 against the oracle and against
    the GPU's FP64 run with the same decisions.  These are looser than the
    per-step 1e-10 / 1e-6 because a capped step of this workload amplifies
    any difference in its input: its last modes stop at the sweep limit
    before converging (18 of 64 in step 1), and the oracle itself, with its
    nonlinear load perturbed by a relative 1e-15, moves by 1.4e-11 after
    step 1 with the warm guess (1e-13: 7.8e-12; measured on the oracle
    alone), while the first 16 modes move by less than 1e-13.  The GPU's
    FP64 solves (eigenbasis products instead of a banded Cholesky) round
    differently by about 1e-14, which the step carries to the 1e-10 range;
    the mixed contraction's 2.5e-9 difference reaches 1.9e-6 there (warm
    guess, step 1; below 1e-6 with the counter-based guess).
  * the separated energy (Sec. 2.1) of the 64-mode states to 1e-12.
"""
import numpy as np
import pytest

from oracle.ctd import State, ctd_step, full_field, state_from_instance
from oracle.energy import energy_separated
from oracle.scheme import problem_from_instance
from workloads import make_instance

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}
_CACHE = {}


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle(init):
    if init not in _CACHE:
        inst = make_instance("ac3d_n256")
        pr = problem_from_instance(inst, init=init)
        states, logs = [state_from_instance(inst)], []
        for k in range(2):
            st, lg = ctd_step(pr, states[-1], k)
            states.append(st)
            logs.append(lg)
            print(f"oracle 256^3 init={init} step {k}: M_k {states[-2].modes} modes {len(lg.iters)} "
                  f"sweeps {sum(lg.iters)} stop {lg.stop}", flush=True)
        _CACHE[init] = (pr, states, logs, [full_field(st) for st in states[1:]])
    return _CACHE[init]


def prefix_field(amp, factors, m):
    return np.einsum("m,im,jm,km->ijk", amp[:m], *[f[:, :m] for f in factors], optimize=True)


@pytest.mark.parametrize("init", ["warm", "hash"])
def test_capped_steps_replay_parity_256(ctd, init):
    """Step 1 from the seeded u^0; step 2 from the oracle's own u^1 (so that
    each step is compared from the same u^k: a step's difference is not
    carried into the next)."""
    from workloads import Instance
    pr, states, logs, refs = oracle(init)
    assert [lg.stop for lg in logs] == ["cap", "cap"] and states[1].modes == 64
    inst = make_instance("ac3d_n256")
    starts = [inst, Instance(**{**inst.__dict__, "amp": states[1].sigma.copy(),
                                "factors": [f.copy() for f in states[1].factors]})]
    whole = {"fp64": 1e-8, "mixed": 1e-5}
    fields = {}
    for k in range(2):
        for prec in ("fp64", "mixed"):
            print(f"GPU 256^3 replay step {k} prec={prec} init={init}", flush=True)
            with ctd.Solver(starts[k], precision=prec, schedule="replay", init=init) as s:
                s.step_index = k
                s.set_decisions([logs[k].iters])
                info = s.step(1)[0]
                assert info["modes"] == 64
                U = s.reconstruct()
                amp, fac = s.modes()
            ref16 = prefix_field(states[k + 1].sigma, states[k + 1].factors, 16)
            e16 = rel(prefix_field(amp, fac, 16), ref16)
            err = rel(U, refs[k])
            print(f"  step {k} {prec} vs oracle: first 16 modes {e16:.3e}, whole field {err:.3e}",
                  flush=True)
            assert e16 < TOL[prec]
            assert err < whole[prec]
            fields[(k, prec)] = U
        d = rel(fields[(k, "mixed")], fields[(k, "fp64")])
        print(f"  step {k} mixed vs fp64 (same decisions, same u^k): {d:.3e}", flush=True)
        assert d < whole["mixed"]


def test_capped_energy_parity_256(ctd):
    """Energy of 64-mode states: the pair-tile Grams at M = 64 (all four tiles)."""
    pr, states, logs, refs = oracle("warm")
    inst = make_instance("ac3d_n256")
    with ctd.Solver(inst, precision="fp64", schedule="replay", init="warm", energy=True) as s:
        s.set_decisions([lg.iters for lg in logs])
        infos = s.step(2)
        amp, fac = s.modes()
    for k in range(2):
        e = energy_separated(pr, states[k + 1])
        print(f"energy after step {k}: {infos[k]['energy']:.15e} vs oracle {e:.15e}", flush=True)
        assert infos[k]["energy"] == pytest.approx(e, rel=1e-12)
    assert infos[1]["energy"] == pytest.approx(energy_separated(pr, State(amp, fac)), rel=1e-12)
    assert infos[1]["energy"] <= infos[0]["energy"]
