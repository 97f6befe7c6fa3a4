"""Problem statement and scheme coefficients -- oracle, test infrastructure only.

Allen-Cahn in the paper's form (Sec. 2.1, eq. AC):
    du/dt + L (dF/du - kappa Lap u) = 0,  F(u) = a0 (u^2 - 1)^2  (eq. energyfunction)
with homogeneous Neumann data (Sec. 2.2).  The stabilized semi-implicit scheme
(Sec. 2.5, eq. AC-discrete-semi-stable-K) is
    [(1/dt + alpha L) M + L kappa K] u^{k+1} = (1/dt + alpha L) M u^k - int N^T L w(u^k),
with w = dF/du = 4 a0 (u^3 - u), energy stable for alpha >= max(w')/2
(eq. AC-discrete-semi-stable-step, App. A).

Reading of the epsilon form (u_t = eps^2 Lap u - (u^3 - u) with stabilizer
S): L = 1, kappa = eps^2, a0 = 1/4, alpha = S.

Shorthands: c = 1/dt + alpha L, lam = L kappa, omega = 4 a0 L, so that
L w(u) = omega (u^3 - u).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

from .cfe1d import Axis


@dataclass
class Problem:
    dim: int
    axes: list
    L: float
    kappa: float
    a0: float
    alpha: float
    dt: float
    fp_tol: float = 1e-2
    fp_max_iter: int = 20
    enrich_tol: float = 1e-8
    max_modes: int = 64
    seed: int = 0
    init: str = "warm"          # "warm" (mode m of u^k when m < M_k) or "hash"
    # reduced integration domain (Sec. 3.3, eq. MxyRD), 2D: an element whose
    # Gauss-point values of w(u^k) all have |w| <= rd_tol is left out of the
    # M_xy integral; 0 leaves out only elements where w vanishes exactly
    rd_tol: float = 0.0
    # separated integration of M_xy (Sec. 3.3, eq. MxySep), 2D: L w(u^k) on
    # the Gauss grid replaced by w_rank terms of a greedy rank-one (PGD)
    # decomposition, each from w_iters alternating updates; 0 = full integral
    w_rank: int = 0
    w_iters: int = 30

    @property
    def c(self):
        return 1.0 / self.dt + self.alpha * self.L

    @property
    def lam(self):
        return self.L * self.kappa

    @property
    def omega(self):
        return 4.0 * self.a0 * self.L

    def max_w_prime(self, umax=1.0):
        """max over |u| <= umax of w'(u) = 4 a0 (3u^2 - 1)."""
        return 4.0 * self.a0 * (3.0 * umax * umax - 1.0)

    def energy_stable(self):
        """alpha >= max(w')/2 (eq. AC-discrete-semi-stable-step) on [-1, 1]."""
        return self.alpha >= 0.5 * self.max_w_prime()


def problem_from_eps(dim, nodes, eps, S, dt, lo=(0.0,) * 3, hi=(1.0,) * 3,
                     s=2, p=2, a=12.0, ng=5, **kw) -> Problem:
    if isinstance(nodes, int):
        nodes = (nodes,) * dim
    axes = [Axis(nodes[d], lo[d], hi[d], s=s, p=p, a=a, ng=ng) for d in range(dim)]
    return Problem(dim=dim, axes=axes, L=1.0, kappa=eps * eps, a0=0.25,
                   alpha=S, dt=dt, **kw)


def problem_from_instance(inst, **kw) -> Problem:
    """Build from a workloads.Instance (raw parameters only)."""
    args = dict(fp_tol=inst.fp_tol, fp_max_iter=inst.fp_max_iter,
                enrich_tol=inst.enrich_tol, max_modes=inst.max_modes,
                seed=inst.seed)
    args.update(kw)
    return problem_from_eps(inst.dim, inst.nodes, inst.eps, inst.S, inst.dt,
                            lo=inst.lo, hi=inst.hi, s=inst.patch_s,
                            p=inst.poly_p, a=inst.dilation_a,
                            ng=inst.gauss_points, **args)


def paper_dofs(h, dim, length=5.0):
    """Nodes of a uniform box mesh with element size h: (length/h + 1)^dim."""
    n = int(round(length / h)) + 1
    return n ** dim
