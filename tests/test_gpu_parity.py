"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Decisions: the oracle runs adaptively and its decision log (sweeps per mode,
modes per step) is handed to the GPU in replay mode, so the comparison
isolates arithmetic; the GPU's own adaptive decisions are compared with the
oracle's separately.  Tolerances (relative nodal l2, the paper's error metric
of Sec. 4.1): 1e-10 for the FP64 path, 1e-6 for the mixed path.
"""
import numpy as np
import pytest

from oracle.ctd import ctd_step, full_field, state_from_instance, State
from oracle.energy import energy_separated
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


def oracle_run(inst, steps, **kw):
    pr = problem_from_instance(inst, **kw)
    st = state_from_instance(inst)
    fields, logs = [], []
    for k in range(steps):
        st, lg = ctd_step(pr, st, k)
        fields.append(full_field(st))
        logs.append(lg)
    return pr, st, fields, logs


def test_band_solve_kernel(ctd):
    import torch
    import scipy.linalg as sla
    from oracle.cfe1d import Axis
    # block data in LDS up to (3, 515); (2, 2048) and (3, 1300): odd blocks in
    # LDS, even blocks in a device workspace; the last two: all blocks in the
    # workspace
    for s, n in ((1, 37), (2, 100), (2, 1031), (3, 515), (2, 2048), (3, 1300), (2, 2600), (3, 2000)):
        ax = Axis(n, 0.0, 1.0, s=s, p=min(s, 2), a=12.0, ng=5)
        bw = 2 * s + 1
        Mb, Kb = ax.banded(ax.M), ax.banded(ax.K)
        rng = np.random.default_rng(n)
        count = 5
        al = rng.uniform(10.0, 3000.0, count)
        be = rng.uniform(1e-6, 1e-2, count)
        b = rng.standard_normal((count, n))
        dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
        x = torch.zeros((count, n), dtype=torch.float64, device="cuda")
        print(f"band solve s={s} n={n}", flush=True)
        ctd.band_solve(n, bw, dev(Mb), dev(Kb), dev(al), dev(be), dev(b), x, count)
        torch.cuda.synchronize()
        xh = x.cpu().numpy()
        for k in range(count):
            ref = sla.solveh_banded(al[k] * Mb + be[k] * Kb, b[k], lower=True)
            assert rel(xh[k], ref) < 1e-12


@pytest.mark.parametrize("dim,n,m0,steps,solve", [(2, 37, 3, 3, "auto"), (3, 21, 3, 2, "bcr"),
                                                  (3, 21, 3, 2, "fd"), (2, (1500, 24), 3, 2, "auto"),
                                                  (3, (40, 17, 23), 3, 2, "fd")])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("init", ["warm", "hash"])
def test_step_replay_parity(ctd, dim, n, m0, steps, solve, prec, init):
    inst = small_instance(dim=dim, n=n, m0=m0, kmax=4, eps=0.05, dt=1e-3, max_modes=24)
    pr, st, fields, logs = oracle_run(inst, steps, init=init)
    print(f"replay dim={dim} n={n} solve={solve} prec={prec} init={init} "
          f"modes={[len(l.iters) for l in logs]}", flush=True)
    with ctd.Solver(inst, precision=prec, schedule="replay", solve=solve, init=init) as s:
        s.set_decisions([lg.iters for lg in logs])
        for k in range(steps):
            info = s.step(1)[0]
            assert info["modes"] == len(logs[k].iters)
            U = s.reconstruct()
            err = rel(U, fields[k])
            print(f"  step {k}: rel l2 = {err:.3e}", flush=True)
            assert err < TOL[prec]


@pytest.mark.parametrize("dim,n,m0,steps,solve", [(2, 37, 3, 3, "auto"), (3, 21, 3, 2, "bcr"),
                                                  (3, 21, 3, 2, "fd")])
def test_adaptive_decisions_match_oracle(ctd, dim, n, m0, steps, solve):
    inst = small_instance(dim=dim, n=n, m0=m0, kmax=4, eps=0.05, dt=1e-3, max_modes=24)
    pr, st, fields, logs = oracle_run(inst, steps)
    with ctd.Solver(inst, precision="fp64", solve=solve) as s:
        s.step(steps)
        dec = s.decisions()
        U = s.reconstruct()
    assert dec == [lg.iters for lg in logs]
    assert rel(U, fields[-1]) < 1e-10


@pytest.mark.parametrize("dim,n", [(2, 37), (3, 21)])
def test_energy_matches_oracle(ctd, dim, n):
    inst = small_instance(dim=dim, n=n, m0=4, kmax=4)
    pr = problem_from_instance(inst)
    with ctd.Solver(inst) as s:
        E0 = s.energy()
        assert E0 == pytest.approx(energy_separated(pr, state_from_instance(inst)), rel=1e-12)
        s.step(1)
        amp, fac = s.modes()
        E1 = s.energy()
        assert E1 == pytest.approx(energy_separated(pr, State(amp, fac)), rel=1e-12)
        assert E1 <= E0


@pytest.mark.parametrize("dim,n,prec", [(2, 45, "fp64"), (3, 23, "fp64"), (3, 23, "mixed")])
def test_nonlinear_load_matches_oracle(ctd, dim, n, prec):
    """The dominant contraction alone: F_d for random fixed factors."""
    from oracle.ctd import FullGridNonlinear
    inst = small_instance(dim=dim, n=n, m0=5, kmax=5)
    pr = problem_from_instance(inst)
    rng = np.random.default_rng(3)
    u = [rng.uniform(-1, 1, n) for _ in range(dim)]
    F = FullGridNonlinear(pr, state_from_instance(inst))
    with ctd.Solver(inst, precision=prec) as s:
        for d in range(dim):
            got = s.nonlinear_load(d, u)
            ref = F(d, u)
            err = rel(got, ref)
            print(f"  load d={d}: {err:.2e}", flush=True)
            assert err < (1e-12 if prec == "fp64" else 2e-6)


def test_00_device_limits(ctd):
    import torch
    p = torch.cuda.get_device_properties(0)
    print("device:", p.name, "LDS/block:", getattr(p, "shared_memory_per_block", None),
          "LDS/block optin:", getattr(p, "shared_memory_per_block_optin", None),
          "CUs:", p.multi_processor_count, flush=True)


@pytest.mark.parametrize("dim,n,m0", [(3, (37, 45, 70), 60), (3, (20, 33, 66), 170),
                                      (2, (100, 130), 12)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_reconstruct_matches_definition(ctd, dim, n, m0, dtype):
    """Nodal field sum_m amp_m prod_d X_d[:, m] (Kronecker property: nodal
    values are the coefficients), ragged 64 x 64 tiles.  FP64 output: FP64
    MFMA (60 modes) or, past its LDS, the FP64 tiled / node-parallel forms
    (170 modes).  FP32 output: FP32 MFMA with FP32 accumulation, bounded by
    its rounding: inputs, weights and products rounded to 2^-24 and M - 1
    FP32 additions give |error| <= (M + 5) 2^-24 sum_m |term_m| per node."""
    inst = small_instance(dim=dim, n=n, m0=m0, kmax=6, max_modes=m0)
    with ctd.Solver(inst) as s:
        U = s.reconstruct(dtype)
    sub = "m,im,jm,lm->ijl" if dim == 3 else "m,im,jm->ij"
    ref = np.einsum(sub, inst.amp, *inst.factors)
    assert U.shape == ref.shape
    if dtype == "f64":
        assert rel(U, ref) < 1e-14
    else:
        absref = np.einsum(sub, np.abs(inst.amp), *[np.abs(f) for f in inst.factors])
        bound = (m0 + 5) * 2.0 ** -24 * np.linalg.norm(absref) / np.linalg.norm(ref)
        err = rel(U, ref)
        print(f"FP32 reconstruction rel l2 {err:.2e}, first-order bound {bound:.2e}", flush=True)
        assert err < bound
