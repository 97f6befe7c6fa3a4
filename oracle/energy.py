"""Discrete energy E(u) = int a0 (u^2 - 1)^2 + kappa/2 |grad u|^2 -- oracle.

Energy functional of Sec. 2.1 with the double-well F of eq. (energyfunction),
integrated with the same tensor Gauss rule as every other integral.  Two
evaluations: on the full tensor Gauss grid (plain definition, small grids)
and in separated form (quartic term through per-axis fourth-moment tensors,
quadratic and gradient terms through 1D Gram matrices).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def energy_fullgrid(prob, U_nodal):
    ax = prob.axes
    D = prob.dim

    def to_q(T, d, mat):
        return np.moveaxis(np.tensordot(mat, T, axes=([1], [d])), 0, d)

    Uq = U_nodal
    for d in range(D):
        Uq = to_q(Uq, d, ax[d].Phi.toarray())
    grad2 = np.zeros_like(Uq)
    for g in range(D):
        T = U_nodal
        for d in range(D):
            T = to_q(T, d, (ax[d].dPhi if d == g else ax[d].Phi).toarray())
        grad2 += T * T
    dens = prob.a0 * (Uq * Uq - 1.0) ** 2 + 0.5 * prob.kappa * grad2
    for d in range(D):
        shp = [1] * D
        shp[d] = -1
        dens = dens * ax[d].W.reshape(shp)
    return float(dens.sum())


def energy_separated(prob, state):
    """Same quadrature, separated: needs only 1D contractions of the factors."""
    ax = prob.axes
    D = prob.dim
    s = state.sigma
    Mm = [state.factors[d].T @ ax[d].M @ state.factors[d] for d in range(D)]
    Km = [state.factors[d].T @ ax[d].K @ state.factors[d] for d in range(D)]
    ss = np.outer(s, s)
    u2 = float(np.sum(ss * np.prod(Mm, axis=0)))
    g2 = 0.0
    for d in range(D):
        P = Km[d].copy()
        for e in range(D):
            if e != d:
                P = P * Mm[e]
        g2 += float(np.sum(ss * P))
    M = len(s)
    t4 = np.einsum("a,b,c,d->abcd", s, s, s, s)
    for d in range(D):
        X = ax[d].Phi @ state.factors[d]
        G4 = np.einsum("q,qa,qb,qc,qd->abcd", ax[d].W, X, X, X, X, optimize=True)
        t4 = t4 * G4
    u4 = float(t4.sum())
    vol = float(np.prod([ax[d].hi - ax[d].lo for d in range(D)]))
    return prob.a0 * (u4 - 2.0 * u2 + vol) + 0.5 * prob.kappa * g2
