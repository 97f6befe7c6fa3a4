"""Whole-step parity at a benchmarked 3D shape with the mode cap reached.

256^3 mesh (the 3D 256^3 workload's parameters: eps 0.01, dt 5e-4), a u^k of
64 seeded cosine modes, cap 64: the step runs the cubic contraction at
M_k = 64 (four 16-wide mode tiles, 20 tile triples), the right-hand side
with all of its column chunks up to M = 63 earlier modes, and ends capped
(Sec. 3.3 algorithm; cap = the adaptive variant's M_c).  The oracle runs the
step adaptively on its separated path (FP64, plain numpy) with at most 3
sweeps per mode, so that it finishes in about half a minute, and the GPU
replays its decisions (sweeps per mode) for both readings of the initial
guess of a mode.  Bars: FP64 1e-10 and mixed 1e-6 relative nodal l2 against
the oracle (the per-step bound; Sec. 4.1 error metric), mixed against FP64
on the GPU to the same 1e-6, and the separated energy (Sec. 2.1) of the
64-mode states to 1e-12.
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


def workload():
    return make_instance("ac3d_n256", m0=64, max_modes=64, fp_max_iter=3)


def oracle(init):
    if init not in _CACHE:
        inst = workload()
        pr = problem_from_instance(inst, init=init)
        st0 = state_from_instance(inst)
        st1, lg = ctd_step(pr, st0, 0)
        _CACHE[init] = (pr, st0, st1, lg, full_field(st1))
        print(f"oracle 256^3 init={init}: modes {len(lg.iters)} sweeps {sum(lg.iters)} "
              f"stop {lg.stop}", flush=True)
    return _CACHE[init]


@pytest.mark.parametrize("init", ["warm", "hash"])
def test_capped_step_replay_parity_256(ctd, init):
    pr, st0, st1, lg, ref = oracle(init)
    assert lg.stop == "cap" and len(lg.iters) == 64
    inst = workload()
    fields = {}
    for prec in ("fp64", "mixed"):
        print(f"GPU 256^3 replay prec={prec} init={init}", flush=True)
        with ctd.Solver(inst, precision=prec, schedule="replay", init=init) as s:
            s.set_decisions([lg.iters])
            info = s.step(1)[0]
            assert info["modes"] == 64
            fields[prec] = s.reconstruct()
        err = rel(fields[prec], ref)
        print(f"  {prec} vs oracle: {err:.3e}", flush=True)
        assert err < TOL[prec]
    d = rel(fields["mixed"], fields["fp64"])
    print(f"  mixed vs fp64 (same decisions): {d:.3e}", flush=True)
    assert d < TOL["mixed"]


def test_capped_energy_parity_256(ctd):
    """Energy of 64-mode states: the pair-tile Grams at M = 64 (all four tiles)."""
    pr, st0, st1, lg, ref = oracle("warm")
    inst = workload()
    with ctd.Solver(inst, precision="fp64", schedule="replay", init="warm", energy=True) as s:
        E0 = s.energy()
        s.set_decisions([lg.iters])
        info = s.step(1)[0]
        amp, fac = s.modes()
    e0 = energy_separated(pr, st0)
    e1 = energy_separated(pr, st1)
    print(f"energy u^k {E0:.15e} vs {e0:.15e}; u^k+1 {info['energy']:.15e} vs {e1:.15e}", flush=True)
    assert E0 == pytest.approx(e0, rel=1e-12)
    assert info["energy"] == pytest.approx(e1, rel=1e-12)
    assert info["energy"] == pytest.approx(energy_separated(pr, State(amp, fac)), rel=1e-12)
