"""Batched and served execution on the GPU: concurrency must not change results.

Each instance's arithmetic is that of one ctd_solver on one stream, so a
result is compared bitwise: standalone vs inside a concurrent batch, and a
served request alone vs in a mix of other requests.  One standalone result
is also pinned to the oracle by the replay parity tests; here the
standalone solver is the reference.
"""
import numpy as np
import pytest

from workloads import Instance, small_instance, make_batch, make_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


def standalone(ctd, inst, steps, **kw):
    with ctd.Solver(inst, **kw) as s:
        s.step(steps)
        return s.modes()


def same_modes(a, b):
    (amp_a, fa), (amp_b, fb) = a, b
    return (amp_a.shape == amp_b.shape and np.array_equal(amp_a, amp_b)
            and all(np.array_equal(x, y) for x, y in zip(fa, fb)))


def uneven_2d(count, seed=11):
    # the batched workload's generator, sizes capped so the test stays short
    return make_batch(seed=seed, count=count, nodes_range=(24, 160), max_modes=12)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("init", ["hash", "warm"])
@pytest.mark.parametrize("executor", ["lockstep", "streams"])
def test_batch_concurrent_equals_standalone(ctd, prec, init, executor):
    insts = uneven_2d(6)
    print(f"batch sizes {[i.nodes[0] for i in insts]} prec={prec} init={init} "
          f"executor={executor}", flush=True)
    b = ctd.Batch(insts, precision=prec, init=init)
    try:
        b.set_mode(executor)
        b.set_workers(4)
        b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i, inst in enumerate(insts):
        assert same_modes(got[i], standalone(ctd, inst, 2, precision=prec, init=init)), f"instance {i}"


def _with_n(inst, n, **kw):
    """The instance's parameters on an n x n grid (its modes resampled)."""
    t = np.arange(n, dtype=np.float64) / (n - 1)
    src = np.arange(inst.nodes[0], dtype=np.float64) / (inst.nodes[0] - 1)
    f = [np.ascontiguousarray(np.stack([np.interp(t, src, x[:, m]) for m in range(x.shape[1])], 1))
         for x in inst.factors]
    p = inst.params()
    p.update(nodes=(n, n), **kw)
    return Instance(amp=inst.amp.copy(), factors=f, **p)


def test_lockstep_storage_classes_zero_and_energy(ctd):
    """Lockstep over every storage class of the banded solve (LDS, split,
    workspace) and both finalisation widths, with a zero initial field (its
    first mode has zero amplitude: u^{k+1} = 0) and the energy of every step:
    modes, step records and energies identical to the standalone solver."""
    base = uneven_2d(4, seed=31)
    insts = [_with_n(base[0], 40), _with_n(base[1], 700), _with_n(base[2], 2048),
             _with_n(base[3], 2600)]
    z = _with_n(base[1], 64)
    z.amp = np.zeros_like(z.amp)
    insts.append(z)
    kw = dict(precision="fp64", energy=True)
    print(f"lockstep classes sizes {[i.nodes[0] for i in insts]}", flush=True)
    b = ctd.Batch(insts, **kw)
    try:
        b.set_mode("lockstep")
        infos = b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i, inst in enumerate(insts):
        with ctd.Solver(inst, **kw) as s:
            ref_info = s.step(2)
            ref = s.modes()
        assert same_modes(got[i], ref), f"instance {i}"
        for a, r in zip(infos[i], ref_info):
            for key in ("modes", "sweeps", "capped", "fp_unconverged", "zero_mode", "last_term_max"):
                assert a[key] == r[key], (i, key)
            assert a["energy"] == r["energy"] or (np.isnan(a["energy"]) and np.isnan(r["energy"]))
    assert infos[-1][0]["zero_mode"] == 1 and infos[-1][0]["modes"] == 0


def test_lockstep_needs_one_band_width(ctd):
    """Instances of two patch sizes (two band widths): lockstep is refused,
    the default executor falls back to worker streams, results unchanged."""
    insts = uneven_2d(3, seed=41)
    insts[1] = _with_n(insts[1], insts[1].nodes[0], patch_s=1, poly_p=1)
    b = ctd.Batch(insts, precision="fp64")
    try:
        with pytest.raises(ctd.CtdError):
            b.set_mode("lockstep")
        b.set_mode("auto")
        b.step(1)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i, inst in enumerate(insts):
        assert same_modes(got[i], standalone(ctd, inst, 1, precision="fp64")), f"instance {i}"


@pytest.mark.parametrize("lockstep", [True, False])
def test_served_alone_equals_mix(ctd, lockstep):
    target = small_instance(dim=2, n=40, m0=3, kmax=4, seed=5, max_modes=12)
    target3 = small_instance(dim=3, n=17, m0=3, kmax=4, seed=6, max_modes=8)
    others = [inst for _, inst in make_requests(seed=3, count=8, nodes2d_range=(24, 96),
                                                nodes3d_range=(12, 20), steps_range=(1, 3),
                                                max_modes=10)]
    ref = standalone(ctd, target, 3, precision="mixed")
    ref3 = standalone(ctd, target3, 2, precision="mixed")
    print(f"served mix, lockstep route {lockstep}", flush=True)
    with ctd.Server(workers=1, lockstep=lockstep) as srv:
        t = srv.submit(target, nsteps=3, precision="mixed")
        assert srv.wait(t, 60000)
        alone = srv.fetch(t)
    assert same_modes(alone, ref)
    with ctd.Server(workers=4, lockstep=lockstep) as srv:
        tickets = [srv.submit(o, precision="mixed") for o in others[:4]]
        t = srv.submit(target, nsteps=3, precision="mixed")
        t3 = srv.submit(target3, nsteps=2, precision="mixed")
        tickets += [srv.submit(o, precision="mixed") for o in others[4:]]
        for k in tickets + [t, t3]:
            assert srv.wait(k, 120000)
        mixed = srv.fetch(t)
        mixed3 = srv.fetch(t3)
        st = [srv.status(k) for k in tickets]
        assert all(s["state"] == "done" for s in st)
        assert all(s["t_done_ms"] >= s["t_start_ms"] >= s["t_submit_ms"] for s in st)
        for k in tickets:
            srv.fetch(k)
        stats = srv.stats()
        assert stats["completed"] == len(tickets) + 2 and stats["failed"] == 0
        assert stats["bytes_in_use"] == 0
    assert same_modes(mixed, ref)
    assert same_modes(mixed3, ref3)


def test_served_join_while_running(ctd):
    """Lockstep route: requests that arrive while others are mid-step join the
    running set at their own first step; each equals its standalone run."""
    import time
    reqs = [small_instance(dim=2, n=n, m0=3, kmax=4, seed=20 + k, max_modes=10)
            for k, n in enumerate((36, 90, 50, 130))]
    refs = [standalone(ctd, r, 3, precision="fp64") for r in reqs]
    with ctd.Server(workers=2) as srv:
        first = srv.submit(reqs[0], nsteps=3, precision="fp64")
        tickets = [first]
        for r in reqs[1:]:
            # wait until the running set has made progress, then join it
            t0 = time.time()
            while srv.status(tickets[-1])["state"] == "queued" and time.time() - t0 < 30:
                time.sleep(0.001)
            tickets.append(srv.submit(r, nsteps=3, precision="fp64"))
        for t in tickets:
            assert srv.wait(t, 120000)
        st = [srv.status(t) for t in tickets]
        got = [srv.fetch(t) for t in tickets]
    # later requests started before earlier ones finished (they overlapped)
    assert any(st[k + 1]["t_start_ms"] < st[k]["t_done_ms"] for k in range(len(st) - 1))
    for k in range(len(reqs)):
        assert same_modes(got[k], refs[k]), f"request {k}"


def test_server_admits_by_footprint(ctd):
    a = small_instance(dim=2, n=48, m0=3, kmax=4, seed=8, max_modes=8)
    b = small_instance(dim=2, n=48, m0=3, kmax=4, seed=9, max_modes=8)
    fa = ctd.footprint_bytes(a)
    fb = ctd.footprint_bytes(b)
    assert fa == fb > 0
    with ctd.Server(budget_bytes=fa + fb // 2, workers=2) as srv:
        ta = srv.submit(a, nsteps=1)
        tb = srv.submit(b, nsteps=1)
        assert srv.wait(ta, 60000)
        # a is done but holds its memory until fetched: b cannot be admitted
        assert not srv.wait(tb, 300)
        assert srv.status(tb)["state"] == "queued"
        assert srv.stats()["bytes_in_use"] == fa
        srv.fetch(ta)
        assert srv.wait(tb, 60000)
        assert srv.status(tb)["footprint"] == fb
        srv.fetch(tb)
    with ctd.Server(budget_bytes=fa // 2, workers=1) as srv:
        with pytest.raises(ctd.CtdError):
            srv.submit(a, nsteps=1)


@pytest.mark.parametrize("lockstep", [True, False])
def test_nonfinite_input_fails_alone(ctd, lockstep):
    """A request whose initial factors hold a NaN ends with ENONFINITE (the
    kernels run normally on it); the requests served beside it complete and
    equal their standalone runs (on the lockstep route the failing request
    leaves the running set and the others go on)."""
    good = small_instance(dim=2, n=40, m0=3, kmax=4, seed=5, max_modes=12)
    bad_f = [f.copy() for f in good.factors]
    bad_f[1][7, 0] = float("nan")
    bad = Instance(**{**good.__dict__, "factors": bad_f})
    with ctd.Solver(bad, precision="fp64") as s:
        with pytest.raises(ctd.CtdError) as ei:
            s.step(1)
        assert "NONFINITE" in str(ei.value)
    ref = standalone(ctd, good, 2, precision="fp64")
    with ctd.Server(workers=2, lockstep=lockstep) as srv:
        tb = srv.submit(bad, nsteps=2, precision="fp64")
        tg = srv.submit(good, nsteps=2, precision="fp64")
        # waiting on a failed request returns its error
        with pytest.raises(ctd.CtdError) as ei:
            srv.wait(tb, 60000)
        assert "NONFINITE" in str(ei.value)
        assert srv.wait(tg, 60000)
        assert srv.status(tb)["state"] == "failed"
        assert srv.status(tg)["state"] == "done"
        got = srv.fetch(tg)
        stats = srv.stats()
        assert stats["failed"] == 1 and stats["completed"] == 1
    assert same_modes(got, ref)


def _oracle_steps(inst, steps):
    from oracle.ctd import ctd_step, full_field, state_from_instance
    from oracle.scheme import problem_from_instance
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    logs = []
    for k in range(steps):
        st, lg = ctd_step(pr, st, k)
        logs.append(lg.iters)
    return full_field(st), logs


def _field(amp, factors):
    sub = "m,im,jm->ij" if len(factors) == 2 else "m,im,jm,km->ijk"
    return np.einsum(sub, amp, *factors)


@pytest.mark.parametrize("executor", ["lockstep", "streams"])
def test_batched_instances_match_oracle(ctd, executor):
    """Instances stepped inside a concurrent batch against the CPU oracle
    (FP64, adaptive on both sides: same decisions, fields to 1e-10)."""
    insts = uneven_2d(5, seed=21)
    b = ctd.Batch(insts, precision="fp64")
    try:
        b.set_mode(executor)
        b.set_workers(3)
        b.step(2)
        got = [b.modes(i) for i in range(len(insts))]
    finally:
        b.close()
    for i in (0, 2, 4):
        ref, logs = _oracle_steps(insts[i], 2)
        U = _field(*got[i])
        err = float(np.linalg.norm(U - ref) / np.linalg.norm(ref))
        print(f"batched instance {i} n={insts[i].nodes[0]}: rel l2 {err:.2e}", flush=True)
        assert err < 1e-10


def test_served_request_matches_oracle(ctd):
    """A 2D and a 3D request served in a mix of others against the oracle."""
    t2 = small_instance(dim=2, n=36, m0=3, kmax=4, seed=15, max_modes=10)
    t3 = small_instance(dim=3, n=15, m0=3, kmax=4, seed=16, max_modes=8)
    others = [inst for _, inst in make_requests(seed=4, count=5, nodes2d_range=(24, 80),
                                                nodes3d_range=(12, 18), steps_range=(1, 3),
                                                max_modes=10)]
    with ctd.Server(workers=3) as srv:
        tk = [srv.submit(o, precision="fp64") for o in others[:2]]
        a = srv.submit(t2, nsteps=2, precision="fp64")
        c = srv.submit(t3, nsteps=2, precision="fp64")
        tk += [srv.submit(o, precision="fp64") for o in others[2:]]
        for k in tk + [a, c]:
            assert srv.wait(k, 120000)
        got2, got3 = srv.fetch(a), srv.fetch(c)
        for k in tk:
            srv.fetch(k)
    for inst, got in ((t2, got2), (t3, got3)):
        ref, _ = _oracle_steps(inst, 2)
        err = float(np.linalg.norm(_field(*got) - ref) / np.linalg.norm(ref))
        print(f"served dim={inst.dim}: rel l2 {err:.2e}", flush=True)
        assert err < 1e-10
