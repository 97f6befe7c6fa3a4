"""Full tensor-product CFE solve of the same scheme -- oracle, tiny grids only.

The limit CTD approaches as modes are added (Sec. 3.2: same shape functions;
Sec. 4.1 uses the CFE solution as reference) and the full solve the adaptive
variant falls back to (Sec. 3.3, adaptivity).  The basis is the tensor
product of the 1D CFE functions; K and Q of eq. (AC-discrete-semi-stable-K)
are assembled as Kronecker products of the 1D matrices and the nonlinear
load is integrated on the tensor Gauss grid.

Test infrastructure only.
"""
from __future__ import annotations

from functools import reduce

import numpy as np


def _kron_all(mats):
    return reduce(np.kron, mats)


def full_matrices(prob):
    """K_full = c (x)M + lam sum_d (K at d, M elsewhere); also (x)M."""
    ax = prob.axes
    D = prob.dim
    Mfull = _kron_all([ax[d].M for d in range(D)])
    Kg = sum(_kron_all([ax[e].K if e == d else ax[e].M for e in range(D)])
             for d in range(D))
    return prob.c * Mfull + prob.lam * Kg, Mfull


def nonlinear_load(prob, U_nodal):
    """int N~_I L w(u) dOmega for every tensor basis function I (tensor Gauss)."""
    ax = prob.axes
    D = prob.dim
    Uq = U_nodal
    for d in range(D):
        Uq = np.moveaxis(np.tensordot(ax[d].Phi.toarray(), Uq, axes=([1], [d])), 0, d)
    G = prob.omega * (Uq ** 3 - Uq)
    for d in range(D):
        shp = [1] * D
        shp[d] = -1
        G = G * ax[d].W.reshape(shp)
    for d in range(D):
        G = np.moveaxis(np.tensordot(ax[d].Phi.toarray().T, G, axes=([1], [d])), 0, d)
    return G


def full_step(prob, U_nodal, Kfull=None, Mfull=None):
    """u^{k+1} of the full tensor CFE system, nodal tensor in and out."""
    if Kfull is None:
        Kfull, Mfull = full_matrices(prob)
    F = nonlinear_load(prob, U_nodal).ravel()
    Q = prob.c * (Mfull @ U_nodal.ravel()) - F
    return np.linalg.solve(Kfull, Q).reshape(U_nodal.shape)


def functional_J(prob, U_nodal, U_prev, Kfull=None, Mfull=None):
    """J(u) = 1/2 u^T K u - u^T Q(u^k): each CTD directional solve minimises it."""
    if Kfull is None:
        Kfull, Mfull = full_matrices(prob)
    F = nonlinear_load(prob, U_prev).ravel()
    Q = prob.c * (Mfull @ U_prev.ravel()) - F
    v = U_nodal.ravel()
    return 0.5 * v @ (Kfull @ v) - v @ Q
