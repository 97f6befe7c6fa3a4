"""CTD time step -- oracle, test infrastructure only.

Implements the solution algorithm of Sec. 3.3 for one time step of the
stabilized semi-implicit scheme (Sec. 2.5): the new field u^{k+1} is built
from scratch as a sum of rank-one products of 1D CFE functions (eq. CTD,
eq. u-increment), one mode at a time (greedy enrichment, steps 1-7), each
mode by alternating fixed-point sweeps over the directions x, y(, z).  The
directional problem is eq. (ux)/(KxQx) for 2D and its 3D analogue obtained by
the derivation of App. D with the test function du_x u_y u_z:

  K_d = (c prod_e m_e) M_d + lam (prod_e m_e) K_d + lam (sum_e k_e prod_{f!=e} m_f) M_d
  Q_d = c sum_j sig^k_j a^k_j M_d X^k_dj
        - sum_m sig_m [c a_m M_d + lam a_m K_d + lam b_m M_d] X_dm  - F_d
  m_e = u_e^T M_e u_e, k_e = u_e^T K_e u_e, a^k_j = prod_e u_e^T M_e X^k_ej,
  a_m = prod_e u_e^T M_e X_em, b_m = sum_e (u_e^T K_e X_em) prod_{f!=e} u_f^T M_f X_fm,
  F_d = int N~_d prod_e u_e L w(u^k)      (the M_xy u_y term of eq. KxQx)

(c = 1/dt + alpha L, lam = L kappa; e, f range over the fixed directions.)

Readings where the paper is silent or loose (each is mirrored by the HIP
library, which shares no code with this module):
  * initial guess of a mode: counter-based pseudo-random vector (hashinit),
    or optionally mode m of u^k ("warm");
  * each solved factor is rescaled to unit M-norm and its norm carried as the
    mode amplitude sigma (the product is invariant under such scalings);
  * fixed-point test (eps1): relative Frobenius change of the nodal rank-one
    tensor between consecutive sweeps, from the second sweep on, through the
    Gram identity ||P - P'||^2 = ||P||^2 + ||P'||^2 - 2 <P, P'>; at most
    fp_max_iter sweeps;
  * enrichment stop (eps2): nodal max of the appended rank-one term,
    sigma * prod_d max|u_d| <= enrich_tol (the triggering mode is kept), or
    the mode cap max_modes (the adaptive variant's M_c, capped rather than
    switched to a full solve); a mode with zero amplitude is dropped and ends
    the step;
  * the mode count restarts from zero every time step;
  * the alternatives to the full 2D M_xy integral (Sec. 3.3): the reduced
    domain drops an element when |w| <= rd_tol at all its Gauss points; the
    separated w is a greedy rank-one (PGD) decomposition with a fixed count
    of alternating updates per term (pgd_separate).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .hashinit import init_vector


@dataclass
class State:
    """Separated field u = sum_m sigma_m prod_d X_d[:, m] (nodal coefficients).

    warm: how many of its modes a following step may take as warm initial
    guesses (None: all of them; a 3D field state holds none, see
    oracle.actd.field_state)."""
    sigma: np.ndarray
    factors: list
    warm: int | None = None

    @property
    def modes(self):
        return len(self.sigma)

    @property
    def warm_modes(self):
        return self.modes if self.warm is None else self.warm

    def copy(self):
        return State(self.sigma.copy(), [f.copy() for f in self.factors], self.warm)


def state_from_instance(inst) -> State:
    return State(np.array(inst.amp, dtype=np.float64),
                 [np.array(f, dtype=np.float64) for f in inst.factors])


def full_field(state: State) -> np.ndarray:
    """Dense nodal tensor sum_m sigma_m X_m (x) Y_m (x) ... (tiny/medium grids)."""
    D = len(state.factors)
    if D == 2:
        X, Y = state.factors
        return (X * state.sigma) @ Y.T
    X, Y, Z = state.factors
    return np.einsum("m,im,jm,km->ijk", state.sigma, X, Y, Z, optimize=True)


# ---------------------------------------------------------------------------
# nonlinear term F_d = int N~_d prod_{e != d} u_e L w(u^k) dOmega
# ---------------------------------------------------------------------------

def element_wmax(prob, U):
    """max |w(u^k)| = 4 a0 |u^3 - u| over the Gauss points of each element
    (e_x, e_y) of the 2D tensor Gauss grid (the Gauss points of axis d are
    element-major, q = e ng + g)."""
    ng0, ng1 = prob.axes[0].ng, prob.axes[1].ng
    w = 4.0 * prob.a0 * np.abs(U ** 3 - U)
    ne0, ne1 = w.shape[0] // ng0, w.shape[1] // ng1
    return w.reshape(ne0, ng0, ne1, ng1).max(axis=(1, 3))


def element_mask(prob, U):
    """Reduced domain Omega_r (Sec. 3.3, eq. MxyRD): 0 at every Gauss point of
    an element whose values of w(u^k) all satisfy |w| <= rd_tol, else 1."""
    ng0, ng1 = prob.axes[0].ng, prob.axes[1].ng
    keep = (element_wmax(prob, U) > prob.rd_tol).astype(np.float64)
    return np.repeat(np.repeat(keep, ng0, axis=0), ng1, axis=1)


def pgd_separate(prob, Wg):
    """Separated form of the Gauss-grid values Wg[q_x, q_y] of L w(u^k), the
    decomposition before eq. MxySep (Sec. 3.3), read as the progressive
    (greedy rank-one) decomposition of the HOPGD family: w_rank terms
    a_q(x) b_q(y) are added one at a time, each from w_iters alternating
    updates of its two factors, each update the least-squares factor against
    the residual R = Wg - sum_{p<q} a_p b_p^T with the other factor fixed:
        a <- R b / (b.b),   b <- R^T a / (a.a)
    (R is applied as Wg b - A (B^T b), never formed).  b starts from the
    counter-based vector keyed (seed, step 0, term q, key 7).  A zero
    denominator gives a zero factor.  Returns A (n_qx x Q), B (n_qy x Q)."""
    Q, K = prob.w_rank, prob.w_iters
    n0, n1 = Wg.shape
    A = np.zeros((n0, Q))
    B = np.zeros((n1, Q))
    for q in range(Q):
        b = init_vector(prob.seed, 0, q, 7, n1)
        a = np.zeros(n0)
        for _ in range(K):
            bb = b @ b
            a = (Wg @ b - A[:, :q] @ (B[:, :q].T @ b)) / bb if bb != 0.0 else np.zeros(n0)
            aa = a @ a
            b = (Wg.T @ a - B[:, :q] @ (A[:, :q].T @ a)) / aa if aa != 0.0 else np.zeros(n1)
        A[:, q] = a
        B[:, q] = b
    return A, B


class FullGridNonlinear:
    """Full integration on the tensor Gauss grid (eq. KxxMxx, the M_xy entry).

    2D: M_xy = int N~_x^T N~_y L w(u^k) is formed once per step and
    F_x = M_xy u_y, F_y = M_xy^T u_x (eq. KxQx / KyQy).
    3D: the quadrature-point field of u^k is kept and contracted directly.
    """

    def __init__(self, prob, state_k: State):
        self.prob = prob
        D = prob.dim
        ax = prob.axes
        hats = [ax[d].Phi @ state_k.factors[d] for d in range(D)]
        if D == 2:
            U = (hats[0] * state_k.sigma) @ hats[1].T
        else:
            U = np.einsum("m,im,jm,km->ijk", state_k.sigma, *hats, optimize=True)
        G = prob.omega * (U ** 3 - U)
        self.excluded = 0
        self.wsep = None
        rd, wr = getattr(prob, "rd_tol", 0.0) > 0.0, getattr(prob, "w_rank", 0) > 0
        if (rd or wr) and D != 2:
            raise ValueError("the reduced domain and the separated w are defined for the 2D M_xy")
        if rd and wr:
            raise ValueError("one alternative integration at a time")
        if rd:
            mask = element_mask(prob, U)
            self.excluded = int(round((mask == 0).sum() / (ax[0].ng * ax[1].ng)))
            G = G * mask
        if wr:
            # the integral of the separated approximant on the same Gauss rule
            self.wsep = pgd_separate(prob, G)
            G = self.wsep[0] @ self.wsep[1].T
        for d in range(D):
            shp = [1] * D
            shp[d] = -1
            G = G * ax[d].W.reshape(shp)
        self.G = G
        if D == 2:
            self.Mxy = np.asarray(ax[0].Phi.T @ (ax[1].Phi.T @ G.T).T)

    def __call__(self, d, u):
        prob = self.prob
        ax = prob.axes
        if prob.dim == 2:
            return self.Mxy @ u[1] if d == 0 else self.Mxy.T @ u[0]
        v = [ax[e].Phi @ u[e] for e in range(3)]
        if d == 0:
            r = np.einsum("ijk,j,k->i", self.G, v[1], v[2])
        elif d == 1:
            r = np.einsum("ijk,i,k->j", self.G, v[0], v[2])
        else:
            r = np.einsum("ijk,i,j->k", self.G, v[0], v[1])
        return ax[d].Phi.T @ r


class SeparatedNonlinear:
    """Exact separated evaluation of the same quadrature sum.

    On the tensor Gauss grid u^k(q) = sum_a sigma_a prod_d Xh_d[q_d, a] with
    Xh_d = Phi_d X^k_d, so
      int N~_i prod_e u_e (u^k)^3 = sum_q Phi_d[q,i] W_d[q] h_d[q],
      h_d[q] = sum_{abc} sigma_a sigma_b sigma_c Xh_d[q,a] Xh_d[q,b] Xh_d[q,c]
               prod_{e != d} g_e[a,b,c],
      g_e[a,b,c] = sum_q W_e[q] (Phi_e u_e)[q] Xh_e[q,a] Xh_e[q,b] Xh_e[q,c],
    and the linear part of w integrates to M_d X^k_d (sigma * a^k).  The
    product of 1D Gauss rules is the tensor rule, so this equals the
    full-grid sum up to rounding.
    """

    CHUNK = 256

    def __init__(self, prob, state_k: State):
        self.prob = prob
        self.sk = state_k.sigma
        self.Xk = state_k.factors
        self.hats = [prob.axes[d].Phi @ state_k.factors[d] for d in range(prob.dim)]

    def _g(self, e, u_e):
        ax = self.prob.axes[e]
        Y = self.hats[e]
        wv = ax.W * (ax.Phi @ u_e)
        Mk = Y.shape[1]
        g = np.zeros((Mk, Mk * Mk))
        for q0 in range(0, Y.shape[0], self.CHUNK):
            Yc = Y[q0:q0 + self.CHUNK]
            KR = (Yc[:, :, None] * Yc[:, None, :]).reshape(len(Yc), Mk * Mk)
            g += (Yc * wv[q0:q0 + self.CHUNK, None]).T @ KR
        return g.reshape(Mk, Mk, Mk)

    def __call__(self, d, u):
        prob = self.prob
        ax = prob.axes[d]
        s = self.sk
        T = s[:, None, None] * s[None, :, None] * s[None, None, :]
        for e in range(prob.dim):
            if e != d:
                T = T * self._g(e, u[e])
        X = self.hats[d]
        Mk = X.shape[1]
        T2 = T.reshape(Mk * Mk, Mk)
        h = np.zeros(X.shape[0])
        for q0 in range(0, X.shape[0], self.CHUNK):
            Xc = X[q0:q0 + self.CHUNK]
            KR = (Xc[:, :, None] * Xc[:, None, :]).reshape(len(Xc), Mk * Mk)
            h[q0:q0 + self.CHUNK] = np.sum((KR @ T2) * Xc, axis=1)
        C = ax.Phi.T @ (ax.W * h)
        ak = self.sk.copy()
        for e in range(prob.dim):
            if e != d:
                ak = ak * (self.Xk[e].T @ (prob.axes[e].M @ u[e]))
        lin = ax.M @ (self.Xk[d] @ ak)
        return prob.omega * (C - lin)


def make_nonlinear(prob, state_k, kind="auto"):
    if prob.dim == 2 and (getattr(prob, "rd_tol", 0.0) > 0.0 or getattr(prob, "w_rank", 0) > 0):
        kind = "full"        # the alternatives change the integral of the full route
    if kind == "auto":
        nq = [ax.nq for ax in prob.axes]
        kind = "full" if np.prod(nq, dtype=float) <= 2.5e7 else "separated"
    if kind == "full":
        return FullGridNonlinear(prob, state_k)
    return SeparatedNonlinear(prob, state_k)


# ---------------------------------------------------------------------------
# the step
# ---------------------------------------------------------------------------

@dataclass
class StepLog:
    iters: list = field(default_factory=list)      # sweeps per appended mode
    converged: list = field(default_factory=list)  # eps1 met (vs sweep cap)
    change: list = field(default_factory=list)     # last relative change r
    sigma: list = field(default_factory=list)
    term_max: list = field(default_factory=list)   # sigma * prod max|u_d|
    stop: str = ""                                 # "tol" | "cap" | "zero" | "replay"


def _mnorm(ax, v):
    return float(np.sqrt(v @ (ax.M @ v)))


def solve_direction(prob, d, u, new: State, state_k: State, F):
    """Assemble K_d, Q_d (eq. KxQx, 3D analogue) and solve the banded system."""
    ax = prob.axes
    D = prob.dim
    c, lam = prob.c, prob.lam
    others = [e for e in range(D) if e != d]
    m = {e: float(u[e] @ (ax[e].M @ u[e])) for e in others}
    k = {e: float(u[e] @ (ax[e].K @ u[e])) for e in others}
    pm = np.prod([m[e] for e in others])
    grad = sum(k[e] * np.prod([m[f] for f in others if f != e]) for e in others)
    Kd = (c * pm + lam * grad) * ax[d].M + lam * pm * ax[d].K

    ak = state_k.sigma.copy()
    for e in others:
        ak = ak * (state_k.factors[e].T @ (ax[e].M @ u[e]))
    Q = c * (ax[d].M @ (state_k.factors[d] @ ak))
    if new.modes:
        mm = {e: new.factors[e].T @ (ax[e].M @ u[e]) for e in others}
        kk = {e: new.factors[e].T @ (ax[e].K @ u[e]) for e in others}
        am = np.prod([mm[e] for e in others], axis=0)
        bm = sum(kk[e] * np.prod([mm[f] for f in others if f != e], axis=0)
                 for e in others)
        Xd = new.factors[d]
        Q -= c * (ax[d].M @ (Xd @ (new.sigma * am)))
        Q -= lam * (ax[d].K @ (Xd @ (new.sigma * am)))
        Q -= lam * (ax[d].M @ (Xd @ (new.sigma * bm)))
    Q -= F(d, u)
    return sla.solveh_banded(ax[d].banded(Kd), Q, lower=True)


def ctd_step(prob, state_k: State, step_index: int, replay=None,
             nonlinear="auto", on_solve=None):
    """One time step k -> k+1.  Returns (State u^{k+1}, StepLog).

    replay: optional list of sweep counts per mode; the step then appends
    exactly len(replay) modes, mode m after replay[m] sweeps, and takes no
    decision of its own (used to compare arithmetic with a run whose
    threshold decisions are fixed).
    """
    ax = prob.axes
    D = prob.dim
    F = make_nonlinear(prob, state_k, nonlinear)
    new = State(np.zeros(0), [np.zeros((ax[d].n, 0)) for d in range(D)])
    log = StepLog()
    max_modes = prob.max_modes if replay is None else len(replay)
    for mode in range(max_modes):
        if prob.init == "warm" and mode < state_k.warm_modes:
            u = [state_k.factors[d][:, mode].copy() for d in range(D)]
        else:
            u = [init_vector(prob.seed, step_index, mode, d, ax[d].n)
                 for d in range(D)]
        u = [u[d] / _mnorm(ax[d], u[d]) for d in range(D)]
        sweeps = prob.fp_max_iter if replay is None else replay[mode]
        prev = None
        sigma = 0.0
        conv = False
        r = float("nan")
        it = 0
        zero = False
        for it in range(1, sweeps + 1):
            for d in range(D):
                ud = solve_direction(prob, d, u, new, state_k, F)
                sigma = _mnorm(ax[d], ud)
                if not np.isfinite(sigma):
                    raise FloatingPointError("non-finite mode amplitude")
                if sigma == 0.0:
                    zero = True
                    break
                u[d] = ud / sigma
                if on_solve is not None:
                    on_solve(mode, it, d, sigma, u, new)
            if zero:
                break
            if prev is not None:
                ps, pu = prev
                nn = sigma * sigma * np.prod([u[d] @ u[d] for d in range(D)])
                oo = ps * ps * np.prod([pu[d] @ pu[d] for d in range(D)])
                no = sigma * ps * np.prod([u[d] @ pu[d] for d in range(D)])
                r = float(np.sqrt(max(nn + oo - 2.0 * no, 0.0) / nn))
                if replay is None and r <= prob.fp_tol:
                    conv = True
                    break
            prev = (sigma, [v.copy() for v in u])
        if zero:
            if replay is not None:
                raise FloatingPointError("replayed mode has zero amplitude")
            log.stop = "zero"
            break
        new.sigma = np.append(new.sigma, sigma)
        for d in range(D):
            new.factors[d] = np.column_stack([new.factors[d], u[d]])
        tmax = sigma * np.prod([np.abs(u[d]).max() for d in range(D)])
        log.iters.append(it)
        log.converged.append(conv)
        log.change.append(r)
        log.sigma.append(sigma)
        log.term_max.append(float(tmax))
        if replay is None and tmax <= prob.enrich_tol:
            log.stop = "tol"
            break
    else:
        log.stop = "cap" if replay is None else "replay"
    return new, log


def run(prob, state0: State, steps: int, replay=None, nonlinear="auto",
        first_step=0):
    """Advance `steps` time steps; replay is an optional list of per-step lists."""
    st = state0
    logs = []
    for k in range(steps):
        rp = None if replay is None else replay[k]
        st, lg = ctd_step(prob, st, first_step + k, replay=rp, nonlinear=nonlinear)
        logs.append(lg)
    return st, logs
