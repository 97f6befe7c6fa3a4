"""Pins of the oracle's scheme, CTD algorithm and energy (CPU only).

Each pin is fixed by the paper or by mathematics outside the oracle: closed
forms, reductions to a lower-dimensional or library computation, the full
tensor solve the method converges to, theorem-level invariants, and values the
paper prints.  A few tests plant a plausible mistake in the oracle and check
that a pin catches it.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ctd as ctdmod
from oracle.cfe1d import Axis
from oracle.ctd import State, ctd_step, full_field, state_from_instance
from oracle.energy import energy_fullgrid, energy_separated
from oracle.fullgrid import full_matrices, full_step, functional_J
from oracle.hashinit import init_vector, splitmix64
from oracle.scheme import Problem, paper_dofs, problem_from_eps, problem_from_instance
from workloads import small_instance

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _prob(dim, n, **kw):
    base = dict(eps=0.1, S=2.0, dt=1e-2, s=2, p=2)
    base.update(kw)
    return problem_from_eps(dim, n, **base)


# ---------------------------------------------------------------------------
# values the paper prints
# ---------------------------------------------------------------------------

def test_paper_mesh_dof_counts():
    """(5/h + 1)^d reproduces the DoF counts printed for the 2D and 3D meshes."""
    with open(os.path.join(GOLD, "paper_mesh_dofs.json")) as f:
        g = json.load(f)
    for h, dofs in g["2d"]:
        assert paper_dofs(h, 2, g["side"]) == dofs
    for h, dofs in g["3d"]:
        assert paper_dofs(h, 3, g["side"]) == dofs


def test_paper_stabilizer_satisfies_bound():
    """alpha = 50 >= max(w')/2 = 40 for a0 = 10 on [-1, 1] (eq. AC-discrete-semi-stable-step)."""
    with open(os.path.join(GOLD, "paper_parameters.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        ax = [Axis(8)] * 2
        pr = Problem(dim=2, axes=ax, L=case["L"], kappa=case["kappa"],
                     a0=case["a0"], alpha=g["alpha"], dt=g["dt"])
        assert pr.max_w_prime() / 2 == pytest.approx(40.0)
        assert pr.energy_stable()
    # the epsilon-form mapping needs S >= 1
    assert _prob(2, 8, S=2.0).energy_stable()
    assert not _prob(2, 8, S=0.5).energy_stable()


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLD, "splitmix64.json")) as f:
        outs = [int(h, 16) for h in json.load(f)["outputs_hex"]]
    state = 0
    for o in outs:
        assert splitmix64(state) == o
        state = (state + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
    v = init_vector(3, 1, 2, 0, 1000)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 0.1


# ---------------------------------------------------------------------------
# closed forms and reductions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_constant_state_closed_form(dim):
    """K 1 = 0 and sum N~ = 1 give u' = u - L w(u) / (1/dt + alpha L) for constant u."""
    n = 9
    pr = _prob(dim, n, eps=0.05, dt=5e-2)
    u0 = 0.37
    st = State(np.array([u0]), [np.ones((n, 1)) for _ in range(dim)])
    new, log = ctd_step(pr, st, 0)
    U = full_field(new)
    w = 4 * pr.a0 * (u0 ** 3 - u0)
    expect = u0 - pr.L * w / pr.c
    assert np.abs(U - expect).max() < 1e-12
    assert log.iters[0] == 2          # exact after one sweep, confirmed by the second


def test_y_constant_data_reduces_to_1d():
    """u^k = f(x) 1(y): the 2D step equals the 1D CFE step of the same scheme."""
    n = 15
    pr = _prob(2, n, eps=0.08, dt=2e-2)
    ax = pr.axes[0]
    f = 0.8 * np.cos(np.pi * ax.x) + 0.1
    st = State(np.array([1.0]), [f[:, None], np.ones((n, 1))])
    new, log = ctd_step(pr, st, 0)
    # independent 1D computation with the 1D matrices and the 1D Gauss rule
    fq = ax.Phi @ f
    F1 = ax.Phi.T @ (ax.W * pr.omega * (fq ** 3 - fq))
    g = np.linalg.solve(pr.c * ax.M + pr.lam * ax.K, pr.c * ax.M @ f - F1)
    U = full_field(new)
    assert np.abs(U - g[:, None]).max() < 1e-12


def _eig_pairs(ax):
    mu, V = sla.eigh(ax.K, ax.M)       # K v = mu M v, V^T M V = I
    return mu, V


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_case_eigen_product(dim):
    """a0 = 0: u^k = prod v_i with K v = mu M v gives u' = c/(c + lam sum mu) u^k in one mode."""
    n = 11
    pr = _prob(dim, n, eps=0.2, dt=1e-2)
    pr.a0 = 0.0
    mu, V = _eig_pairs(pr.axes[0])
    idx = [2, 5, 3][:dim]
    st = State(np.array([0.6]), [V[:, [i]] for i in idx])
    new, log = ctd_step(pr, st, 0)
    factor = pr.c / (pr.c + pr.lam * sum(mu[i] for i in idx))
    U = full_field(new)
    assert np.abs(U - factor * full_field(st)).max() < 1e-10 * np.abs(full_field(st)).max()
    assert log.iters[0] == 2


def test_linear_case_two_eigen_products():
    """Sum of two M-orthogonal eigen-products: two modes, each damped by its own factor."""
    n = 12
    pr = _prob(2, n, eps=0.2, dt=1e-2, fp_tol=1e-12, fp_max_iter=400)
    pr.a0 = 0.0
    mu, V = _eig_pairs(pr.axes[0])
    (i1, j1), (i2, j2) = (1, 4), (3, 2)
    st = State(np.array([0.5, 0.3]),
               [V[:, [i1, i2]], V[:, [j1, j2]]])
    new, log = ctd_step(pr, st, 0)
    f1 = pr.c / (pr.c + pr.lam * (mu[i1] + mu[j1]))
    f2 = pr.c / (pr.c + pr.lam * (mu[i2] + mu[j2]))
    expect = 0.5 * f1 * np.outer(V[:, i1], V[:, j1]) + 0.3 * f2 * np.outer(V[:, i2], V[:, j2])
    assert np.abs(full_field(new) - expect).max() < 1e-10
    assert len(log.iters) <= 3 and log.term_max[-1] < 1e-9 * 0.5 or len(log.iters) == 2


@pytest.mark.parametrize("dim,n", [(2, 12), (3, 8)])
def test_ctd_converges_to_full_tensor_solve(dim, n):
    """Sec. 3.2 / 4.1: CTD tends to the full CFE solution as modes are added."""
    inst = small_instance(dim=dim, n=n, m0=3, kmax=3, eps=0.1, dt=1e-2)
    pr = problem_from_instance(inst, fp_tol=1e-9, fp_max_iter=300,
                               enrich_tol=1e-13, max_modes=n ** (dim - 1) + 8)
    st = state_from_instance(inst)
    Kf, Mf = full_matrices(pr)
    ref = full_step(pr, full_field(st), Kf, Mf)
    errs = []

    def capped(mc):
        pr2 = problem_from_instance(inst, fp_tol=1e-9, fp_max_iter=300,
                                    enrich_tol=1e-13, max_modes=mc)
        new, _ = ctd_step(pr2, st, 0)
        return np.linalg.norm(full_field(new) - ref) / np.linalg.norm(ref)

    for mc in (1, 3, 6):
        errs.append(capped(mc))
    new, log = ctd_step(pr, st, 0)
    final = np.linalg.norm(full_field(new) - ref) / np.linalg.norm(ref)
    assert errs[0] > errs[1] > errs[2] > final
    assert final < 1e-8


def test_full_solve_matches_1d_fast_diagonalisation():
    """Linear full solve (a0 = 0) via the generalized eigenbasis of (K, M) in every direction."""
    n = 9
    pr = _prob(2, n, eps=0.15, dt=1e-2)
    pr.a0 = 0.0
    rng = np.random.default_rng(4)
    U0 = rng.uniform(-0.5, 0.5, (n, n))
    U1 = full_step(pr, U0)
    mu, V = _eig_pairs(pr.axes[0])
    # coefficients in the eigenbasis: U0 = V C V^T with V^T M V = I
    M = pr.axes[0].M
    C = V.T @ M @ U0 @ M @ V
    D = pr.c / (pr.c + pr.lam * (mu[:, None] + mu[None, :]))
    assert np.abs(V @ (C * D) @ V.T - U1).max() < 1e-11


# ---------------------------------------------------------------------------
# nonlinear term and energy: two evaluations, invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n", [(2, 10), (3, 7)])
def test_separated_nonlinear_equals_full_grid(dim, n):
    inst = small_instance(dim=dim, n=n, m0=3, kmax=3)
    pr = problem_from_instance(inst)
    rng0 = np.random.default_rng(9)
    st = State(rng0.uniform(0.2, 0.5, 4), [rng0.uniform(-1, 1, (n, 4)) for _ in range(dim)])
    full = ctdmod.FullGridNonlinear(pr, st)
    sep = ctdmod.SeparatedNonlinear(pr, st)
    rng = np.random.default_rng(1)
    u = [rng.uniform(-1, 1, n) for _ in range(dim)]
    for d in range(dim):
        a, b = full(d, u), sep(d, u)
        assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("dim,n", [(2, 10), (3, 7)])
def test_energy_separated_equals_full_grid(dim, n):
    inst = small_instance(dim=dim, n=n, m0=3, kmax=3)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    a = energy_fullgrid(pr, full_field(st))
    b = energy_separated(pr, st)
    assert a == pytest.approx(b, rel=1e-13)


def test_energy_of_constant_states():
    """E(+-1) = 0, E(0) = a0 |Omega| (double well, no gradient)."""
    n = 8
    pr = _prob(2, n)
    for u0, e in ((1.0, 0.0), (-1.0, 0.0), (0.0, pr.a0)):
        st = State(np.array([1.0]), [np.full((n, 1), u0), np.ones((n, 1))])
        assert energy_separated(pr, st) == pytest.approx(e, abs=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 10), (3, 6)])
def test_energy_law_full_solve(dim, n):
    """App. A: alpha >= max(w')/2 makes E non-increasing for any dt (full CFE solve)."""
    inst = small_instance(dim=dim, n=n, m0=3, kmax=3, eps=0.08)
    for dt in (1e-3, 1e-1, 10.0):
        pr = problem_from_instance(inst)
        pr.dt = dt
        Kf, Mf = full_matrices(pr)
        U = full_field(state_from_instance(inst))
        E = energy_fullgrid(pr, U)
        for _ in range(4):
            U = full_step(pr, U, Kf, Mf)
            E1 = energy_fullgrid(pr, U)
            assert E1 <= E * (1 + 1e-12)
            E = E1


def test_energy_law_can_fail_without_stabilizer():
    """alpha = 0 with dt above 2/(L max w') (eq. AC-discrete-semi-step): the
    explicit w-term overshoots around u = 1 and the energy rises by a finite,
    measured amount (no overflow); the same data with alpha = max(w')/2 on the
    range the field visits (eq. AC-discrete-semi-stable-step) decreases."""
    n = 10
    inst = small_instance(dim=2, n=n, m0=3, kmax=2, eps=0.02)
    U0 = full_field(state_from_instance(inst))
    U0 = 1.0 + 0.05 * U0 / np.abs(U0).max()          # near the well u = 1
    for alpha, expect_rise in ((0.0, True), (None, False)):
        pr = problem_from_instance(inst)
        pr.dt = 1.5
        # stabilised case: alpha >= max w'/2 over |u| <= 1.06 (the field stays there)
        pr.alpha = 0.5 * pr.max_w_prime(1.06) if alpha is None else alpha
        Kf, Mf = full_matrices(pr)
        U = U0.copy()
        E = energy_fullgrid(pr, U)
        rises = []
        for _ in range(5):
            U = full_step(pr, U, Kf, Mf)
            E1 = energy_fullgrid(pr, U)
            assert np.isfinite(E1) and np.abs(U).max() < 2.0
            rises.append(E1 - E)
            E = E1
        if expect_rise:
            assert max(rises) > 1e-3          # a rise of about 10x the initial energy
        else:
            assert max(rises) <= 1e-12 * abs(E)
            assert np.abs(U).max() <= 1.06


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_closed_forms(dim):
    """Sec. 2.1 energy of fields whose integrals are known exactly (the rule is
    exact: u^4 of a degree-1 factor is degree 4 per axis, 5 Gauss points):
      u = x (x) 1 (x) ...:  a0 int (x^2-1)^2 + kappa/2 int 1 = a0 8/15 + kappa/2,
      u = x (x) y (x) ...:  a0 (5^-D - 2 3^-D + 1) + kappa/2 D 3^-(D-1).
    Pins the gradient coefficient (kappa/2) and the quartic and quadratic
    terms of both oracle evaluations independently of each other."""
    n = 9
    inst = small_instance(dim=dim, n=n, m0=1, kmax=1, eps=0.3)
    pr = problem_from_instance(inst)
    x = np.linspace(0.0, 1.0, n)[:, None]
    one = np.ones((n, 1))
    cases = [
        (State(np.array([1.0]), [x] + [one] * (dim - 1)), pr.a0 * 8.0 / 15.0 + 0.5 * pr.kappa),
        (State(np.array([1.0]), [x] * dim),
         pr.a0 * (5.0 ** -dim - 2.0 * 3.0 ** -dim + 1.0) + 0.5 * pr.kappa * dim * 3.0 ** -(dim - 1)),
    ]
    for st, ref in cases:
        assert energy_separated(pr, st) == pytest.approx(ref, rel=1e-13, abs=1e-14)
        assert energy_fullgrid(pr, full_field(st)) == pytest.approx(ref, rel=1e-13, abs=1e-14)


def test_ctd_energy_decreases_and_bounded():
    """CTD steps of a cosine state: energy non-increasing and |u| <= 1 at the nodes."""
    inst = small_instance(dim=2, n=20, m0=4, kmax=4, eps=0.05, dt=1e-3)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    E = energy_separated(pr, st)
    for k in range(4):
        st, _ = ctd_step(pr, st, k)
        E1 = energy_separated(pr, st)
        assert E1 <= E * (1 + 1e-9)
        assert np.abs(full_field(st)).max() <= 1.0 + 1e-6
        E = E1


def test_directional_solves_decrease_J():
    """Each directional solve minimises J(u) = u^T K u / 2 - u^T Q over its factor."""
    n = 9
    inst = small_instance(dim=2, n=n, m0=3, kmax=3, eps=0.1, dt=1e-2)
    pr = problem_from_instance(inst, fp_tol=1e-6, fp_max_iter=30, max_modes=6)
    st = state_from_instance(inst)
    U0 = full_field(st)
    Kf, Mf = full_matrices(pr)
    seen = []

    def on_solve(mode, it, d, sigma, u, new):
        field = full_field(new) if new.modes else np.zeros((n, n))
        field = field + sigma * np.outer(u[0], u[1])
        seen.append(functional_J(pr, field, U0, Kf, Mf))

    ctd_step(pr, st, 0, on_solve=on_solve)
    J = np.array(seen)
    assert len(J) > 10
    assert np.all(np.diff(J) <= 1e-12 * np.abs(J).max())


def test_replay_reproduces_adaptive_run():
    inst = small_instance(dim=2, n=16, m0=3, kmax=3)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    a, log = ctd_step(pr, st, 0)
    b, log2 = ctd_step(pr, st, 0, replay=log.iters)
    assert log2.iters == log.iters
    assert np.abs(full_field(a) - full_field(b)).max() == 0.0


# ---------------------------------------------------------------------------
# planted mistakes (in the oracle, on the CPU): the pins above must catch them
# ---------------------------------------------------------------------------

def test_planted_sign_error_caught(monkeypatch):
    """Flipping the sign of the stiffness term in K_d breaks the linear closed form."""
    n = 11
    pr = _prob(2, n, eps=0.2, dt=1e-2)
    pr.a0 = 0.0
    mu, V = _eig_pairs(pr.axes[0])
    st = State(np.array([0.6]), [V[:, [2]], V[:, [5]]])
    factor = pr.c / (pr.c + pr.lam * (mu[2] + mu[5]))
    orig = ctdmod.solve_direction

    class Neg:
        def __init__(self, p):
            self.p = p

        def __getattr__(self, k):
            if k == "lam":
                return -self.p.lam
            return getattr(self.p, k)

    def bad(prob, *a, **k):
        return orig(Neg(prob), *a, **k)

    monkeypatch.setattr(ctdmod, "solve_direction", bad)
    new, _ = ctd_step(pr, st, 0)
    err = np.abs(full_field(new) - factor * full_field(st)).max()
    assert err > 1e-6


def test_planted_transpose_caught(monkeypatch):
    """Using M_xy instead of M_xy^T in the y-solve breaks full-solve convergence."""
    inst = small_instance(dim=2, n=10, m0=3, kmax=3, eps=0.1, dt=1e-2)
    pr = problem_from_instance(inst, fp_tol=1e-9, fp_max_iter=300,
                               enrich_tol=1e-13, max_modes=20)
    st = state_from_instance(inst)
    ref = full_step(pr, full_field(st))
    orig = ctdmod.FullGridNonlinear.__call__

    def bad(self, d, u):
        if d == 1:
            return self.Mxy @ u[0]
        return orig(self, d, u)

    monkeypatch.setattr(ctdmod.FullGridNonlinear, "__call__", bad)
    new, _ = ctd_step(pr, st, 0, nonlinear="full")
    assert np.linalg.norm(full_field(new) - ref) / np.linalg.norm(ref) > 1e-8


# ---------------------------------------------------------------------------
# reduced integration domain Omega_r (Sec. 3.3, eq. MxyRD), 2D
# ---------------------------------------------------------------------------

def _gauss_field(pr, st):
    hats = [np.asarray(pr.axes[d].Phi @ st.factors[d]) for d in range(2)]
    return (hats[0] * st.sigma) @ hats[1].T


def test_reduced_domain_tiny_tolerance_is_the_full_integral():
    """A tolerance below every element's max |w| leaves nothing out: the
    masked M_xy is the full one, bitwise."""
    inst = small_instance(2, (30, 26), m0=4, kmax=3)
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    full = ctdmod.FullGridNonlinear(pr, st)
    pr_r = problem_from_instance(inst, rd_tol=1e-300)
    red = ctdmod.FullGridNonlinear(pr_r, st)
    assert red.excluded == 0
    assert np.array_equal(red.Mxy, full.Mxy)


def test_reduced_domain_drops_only_vanishing_elements():
    """u = 1 on a band (the CFE basis reproduces constants): those elements
    have |w| at rounding level and are left out; the integral changes by no
    more than rounding, while the elements across the band's edge stay."""
    inst = small_instance(2, (24, 30), m0=1, kmax=1)
    pr = problem_from_instance(inst)
    n0, n1 = inst.nodes
    fy = np.where(np.arange(n1) < n1 // 2, 1.0, 0.3)
    st = State(np.ones(1), [np.ones((n0, 1)), fy.reshape(n1, 1)])
    full = ctdmod.FullGridNonlinear(pr, st)
    red = ctdmod.FullGridNonlinear(problem_from_instance(inst, rd_tol=1e-12), st)
    wmax = ctdmod.element_wmax(pr, _gauss_field(pr, st))
    assert red.excluded == int((wmax <= 1e-12).sum()) > 0
    assert (wmax > 1e-3).sum() > 0                     # the rest is kept
    assert np.abs(red.Mxy - full.Mxy).max() < 1e-12 * np.abs(full.Mxy).max()


def test_reduced_domain_against_element_loop():
    """The masked M_xy against a plain loop over the kept elements and their
    Gauss points (eq. MxyRD written out), with a tolerance that leaves out a
    share of the elements and no element near the threshold."""
    inst = small_instance(2, (12, 10), m0=3, kmax=3)
    st = state_from_instance(inst)
    pr0 = problem_from_instance(inst)
    U = _gauss_field(pr0, st)
    wmax = ctdmod.element_wmax(pr0, U)
    tol = float(np.median(wmax))
    gap = np.abs(wmax - tol) / tol
    tol *= 1.0 + 0.5 * gap[gap > 0].min()              # strictly between two element maxima
    pr = problem_from_instance(inst, rd_tol=tol)
    red = ctdmod.FullGridNonlinear(pr, st)
    ax0, ax1 = pr.axes
    P0, P1 = ax0.Phi.toarray(), ax1.Phi.toarray()
    ref = np.zeros((inst.nodes[0], inst.nodes[1]))
    dropped = 0
    for e0 in range(ax0.nq // ax0.ng):
        for e1 in range(ax1.nq // ax1.ng):
            pts = [(e0 * ax0.ng + g0, e1 * ax1.ng + g1) for g0 in range(ax0.ng) for g1 in range(ax1.ng)]
            w = [4.0 * pr.a0 * (U[q0, q1] ** 3 - U[q0, q1]) for q0, q1 in pts]
            if max(abs(x) for x in w) <= tol:
                dropped += 1
                continue
            for (q0, q1), wq in zip(pts, w):
                ref += np.outer(P0[q0], P1[q1]) * (pr.L * wq * ax0.W[q0] * ax1.W[q1])
    assert dropped == red.excluded and 0 < dropped < wmax.size
    assert np.abs(red.Mxy - ref).max() < 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# separated integration of the 2D M_xy (Sec. 3.3, eq. MxySep)
# ---------------------------------------------------------------------------

def test_separated_w_of_a_one_mode_state_is_exact():
    """u^k = sigma x^ y^T gives L w = omega (sigma^3 x^3 (y^3)^T - sigma x y^T),
    of rank two: two terms reproduce the full integral."""
    inst = small_instance(2, (26, 22), m0=1, kmax=2)
    st = state_from_instance(inst)
    full = ctdmod.FullGridNonlinear(problem_from_instance(inst), st)
    sep = ctdmod.FullGridNonlinear(problem_from_instance(inst, w_rank=2, w_iters=300), st)
    assert np.abs(sep.Mxy - full.Mxy).max() < 1e-11 * np.abs(full.Mxy).max()
    one = ctdmod.FullGridNonlinear(problem_from_instance(inst, w_rank=1, w_iters=300), st)
    assert np.abs(one.Mxy - full.Mxy).max() > 1e-3 * np.abs(full.Mxy).max()


def test_separated_w_equals_truncated_svd():
    """With singular values apart, the greedy terms converge to the leading
    singular triplets (Eckart-Young): the rank-Q approximant equals LAPACK's
    truncated SVD of the Gauss-grid values of L w."""
    inst = small_instance(2, (30, 25), m0=3, kmax=3)
    st = state_from_instance(inst)
    pr0 = problem_from_instance(inst)
    Wg = pr0.omega * (_gauss_field(pr0, st) ** 3 - _gauss_field(pr0, st))
    U_, S_, Vt = np.linalg.svd(Wg)
    # the first Q whose next singular value is at most half of it
    Q = next(q for q in range(1, 8) if S_[q] < 0.5 * S_[q - 1] and all(S_[p + 1] < 0.8 * S_[p] for p in range(q)))
    pr = problem_from_instance(inst, w_rank=Q, w_iters=400)
    A, B = ctdmod.pgd_separate(pr, Wg)
    ref = (U_[:, :Q] * S_[:Q]) @ Vt[:Q]
    assert np.linalg.norm(A @ B.T - ref) < 1e-9 * np.linalg.norm(ref)
    # and the residual is the SVD tail (Frobenius)
    tail = np.sqrt((S_[Q:] ** 2).sum())
    assert np.linalg.norm(Wg - A @ B.T) == pytest.approx(tail, rel=1e-8)


def test_separated_integral_is_the_sum_of_1d_integrals():
    """eq. MxySep: M_xy = sum_q (int N~_x^T w_x^q)(int N~_y w_y^q), each a 1D
    Gauss sum, against the oracle's 2D Gauss sum of the approximant."""
    inst = small_instance(2, (18, 21), m0=3, kmax=3)
    pr = problem_from_instance(inst, w_rank=3, w_iters=20)
    sep = ctdmod.FullGridNonlinear(pr, state_from_instance(inst))
    A, B = sep.wsep
    ax0, ax1 = pr.axes
    ref = np.zeros((inst.nodes[0], inst.nodes[1]))
    for q in range(A.shape[1]):
        ix = np.array([sum(ax0.Phi[g, i] * ax0.W[g] * A[g, q] for g in range(ax0.nq)) for i in range(inst.nodes[0])])
        iy = np.array([sum(ax1.Phi[g, j] * ax1.W[g] * B[g, q] for g in range(ax1.nq)) for j in range(inst.nodes[1])])
        ref += np.outer(ix, iy)
    assert np.abs(sep.Mxy - ref).max() < 1e-13 * np.abs(ref).max()


def test_separated_w_of_the_zero_field():
    """w(0) = 0: every factor is zero (zero denominators), M_xy = 0."""
    inst = small_instance(2, 16, m0=2, kmax=2)
    st = state_from_instance(inst)
    st = State(np.zeros_like(st.sigma), st.factors)
    sep = ctdmod.FullGridNonlinear(problem_from_instance(inst, w_rank=2, w_iters=5), st)
    assert not np.any(sep.wsep[0]) and not np.any(sep.wsep[1]) and not np.any(sep.Mxy)


def test_alternative_integrals_need_2d_and_one_at_a_time():
    inst = small_instance(2, 16, m0=2, kmax=2)
    st = state_from_instance(inst)
    with pytest.raises(ValueError):
        ctdmod.FullGridNonlinear(problem_from_instance(inst, w_rank=2, rd_tol=0.1), st)
    inst3 = small_instance(3, 9, m0=2, kmax=2)
    with pytest.raises(ValueError):
        ctdmod.FullGridNonlinear(problem_from_instance(inst3, w_rank=2), state_from_instance(inst3))
