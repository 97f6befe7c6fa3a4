"""GPU parity across the CFE space parameters (p, s) the paper studies in
Sec. 4 (reproduction order p, patch size s at dilation a = 12): (1, 1),
(1, 2), (2, 2), (3, 3), i.e. band half-widths 3, 5, 7 of M_d and K_d.

The 3D grid has 21 nodes per axis (element size 0.05, the mesh of that
study).  Replay parity against the oracle for both directional solvers and
both precisions, adaptive decisions in FP64, and the nonlinear load alone.
Tolerances as in the other step tests: 1e-10 FP64, 1e-6 mixed (relative
nodal l2).
"""
import numpy as np
import pytest

from oracle.ctd import ctd_step, full_field, state_from_instance, FullGridNonlinear
from oracle.scheme import problem_from_instance
from workloads import small_instance

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}
PS = [(1, 1), (1, 2), (2, 2), (3, 3)]
_cache = {}


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def instance(dim, n, p, s):
    return small_instance(dim=dim, n=n, m0=3, kmax=4, eps=0.05, dt=1e-3, max_modes=24,
                          patch_s=s, poly_p=p)


def oracle_run(dim, n, p, s, steps=2):
    key = (dim, n, p, s, steps)
    if key not in _cache:
        inst = instance(dim, n, p, s)
        pr = problem_from_instance(inst)
        st = state_from_instance(inst)
        fields, logs = [], []
        for k in range(steps):
            st, lg = ctd_step(pr, st, k)
            fields.append(full_field(st))
            logs.append(lg)
        _cache[key] = (inst, fields, logs)
    return _cache[key]


@pytest.mark.parametrize("p,s", PS)
@pytest.mark.parametrize("dim,n,solve", [(2, 37, "auto"), (3, 21, "bcr"), (3, 21, "fd")])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ps_step_replay_parity(ctd, p, s, dim, n, solve, prec):
    inst, fields, logs = oracle_run(dim, n, p, s)
    print(f"(p,s)=({p},{s}) dim={dim} n={n} solve={solve} prec={prec}", flush=True)
    with ctd.Solver(inst, precision=prec, schedule="replay", solve=solve) as sv:
        sv.set_decisions([lg.iters for lg in logs])
        for k in range(len(logs)):
            info = sv.step(1)[0]
            assert info["modes"] == len(logs[k].iters)
            err = rel(sv.reconstruct(), fields[k])
            print(f"  step {k}: rel l2 = {err:.3e}", flush=True)
            assert err < TOL[prec]


@pytest.mark.parametrize("p,s", PS)
def test_ps_adaptive_decisions(ctd, p, s):
    inst, fields, logs = oracle_run(3, 21, p, s)
    with ctd.Solver(inst, precision="fp64", solve="fd") as sv:
        sv.step(len(logs))
        assert sv.decisions() == [lg.iters for lg in logs]
        assert rel(sv.reconstruct(), fields[-1]) < 1e-10


@pytest.mark.parametrize("p,s", [(1, 1), (3, 3)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ps_nonlinear_load(ctd, p, s, prec):
    inst = small_instance(dim=3, n=23, m0=5, kmax=5, patch_s=s, poly_p=p)
    pr = problem_from_instance(inst)
    rng = np.random.default_rng(5)
    u = [rng.uniform(-1, 1, 23) for _ in range(3)]
    F = FullGridNonlinear(pr, state_from_instance(inst))
    with ctd.Solver(inst, precision=prec) as sv:
        for d in range(3):
            err = rel(sv.nonlinear_load(d, u), F(d, u))
            print(f"  (p,s)=({p},{s}) load d={d}: {err:.2e}", flush=True)
            assert err < (1e-12 if prec == "fp64" else 2e-6)
