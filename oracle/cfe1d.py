"""1D convolution finite-element (CFE) space -- oracle, test infrastructure only.

Follows App. B (radial-basis patch interpolation: cubic spline kernel, the
reproducing conditions and the printed closed forms of L and K through the
inverse of R0), App. C (1D convolution shape functions as the FE-weighted sum
of the two nodal patch functions of an element) and Sec. 3.3 eq. (KxxMxx)
(1D mass and stiffness matrices).

Readings (where the paper is silent):
  * natural element coordinates: element e spans [-1, 1] with its left node
    at -1; node j sits at 2(j - e) - 1 (the App. B example puts the patch of
    the left node at {-3, -1, 1});
  * the dilation a is measured in those natural units (App. B kernel
    argument z = |xi - xi_I| / a);
  * a nodal patch is {i-s .. i+s} truncated to the mesh (Sec. 3.2: boundary
    patches drop the part outside the domain); s >= p keeps P^T R0^-1 P
    invertible;
  * Gauss-Legendre with n_g points per element for every integral.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def psi(z):
    """Cubic spline kernel Psi_a(z), z = |xi - xi_I| / a (App. B)."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    out = np.zeros_like(z)
    m1 = z <= 0.5
    m2 = (z > 0.5) & (z <= 1.0)
    z1, z2 = z[m1], z[m2]
    out[m1] = 2.0 / 3.0 - 4.0 * z1 ** 2 + 4.0 * z1 ** 3
    out[m2] = 4.0 / 3.0 - 4.0 * z2 + 4.0 * z2 ** 2 - 4.0 / 3.0 * z2 ** 3
    return out


def dpsi_dz(z):
    """Derivative of the cubic spline kernel with respect to z >= 0."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    out = np.zeros_like(z)
    m1 = z <= 0.5
    m2 = (z > 0.5) & (z <= 1.0)
    z1, z2 = z[m1], z[m2]
    out[m1] = -8.0 * z1 + 12.0 * z1 ** 2
    out[m2] = -4.0 + 8.0 * z2 - 4.0 * z2 ** 2
    return out


def patch_matrices(xi_nodes, a, p):
    """R0, P, L, K of one nodal patch (App. B, moment matrices and closed forms).

    L = (P^T R0^-1 P)^-1 P^T R0^-1 and K = R0^-1 (I - P L), literally.
    """
    xi_nodes = np.asarray(xi_nodes, dtype=np.float64)
    R0 = psi(np.abs(xi_nodes[:, None] - xi_nodes[None, :]) / a)
    P = np.vander(xi_nodes, p + 1, increasing=True)
    R0inv = np.linalg.inv(R0)
    L = np.linalg.inv(P.T @ R0inv @ P) @ P.T @ R0inv
    K = R0inv @ (np.eye(len(xi_nodes)) - P @ L)
    return R0, P, L, K


def patch_function(xi, xi_nodes, a, p):
    """Patch function W(xi) = Psi_a(xi) K + p(xi) L and dW/dxi (App. B).

    Returns two arrays of shape (len(xi), len(xi_nodes)); column j is the
    coefficient of nodal value u_j.
    """
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    xi_nodes = np.asarray(xi_nodes, dtype=np.float64)
    _, _, L, K = patch_matrices(xi_nodes, a, p)
    t = xi[:, None] - xi_nodes[None, :]
    Psi = psi(np.abs(t) / a)
    dPsi = dpsi_dz(np.abs(t) / a) * np.sign(t) / a
    pv = np.vander(xi, p + 1, increasing=True)
    dpv = np.zeros_like(pv)
    for k in range(1, p + 1):
        dpv[:, k] = k * xi ** (k - 1)
    return Psi @ K + pv @ L, dPsi @ K + dpv @ L


def nodal_patch(i, n, s):
    """Nodal patch A_s^i of node i: {i-s .. i+s} truncated to [0, n-1]."""
    return list(range(max(0, i - s), min(n - 1, i + s) + 1))


def element_support(e, n, s):
    """Convolution support A_s^e of element e = union of the two nodal patches."""
    return list(range(max(0, e - s), min(n - 1, e + 1 + s) + 1))


def element_shape(e, n, s, p, a, xi):
    """CFE shape functions of element e and their xi-derivatives (App. C).

    N~_k(xi) = sum_{i in {e, e+1}} N_i(xi) W^{xi_i}_{a,k}(xi), with the linear
    FE functions N_e = (1 - xi)/2, N_{e+1} = (1 + xi)/2.
    Returns (support nodes, N~ (len(xi) x |support|), dN~/dxi).
    """
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    support = element_support(e, n, s)
    col = {k: c for c, k in enumerate(support)}
    N = np.zeros((len(xi), len(support)))
    dN = np.zeros((len(xi), len(support)))
    for i, Ni, dNi in ((e, (1.0 - xi) / 2.0, -0.5), (e + 1, (1.0 + xi) / 2.0, 0.5)):
        patch = nodal_patch(i, n, s)
        xi_nodes = np.array([2.0 * (j - e) - 1.0 for j in patch])
        W, dW = patch_function(xi, xi_nodes, a, p)
        for c, j in enumerate(patch):
            N[:, col[j]] += Ni * W[:, c]
            dN[:, col[j]] += dNi * W[:, c] + Ni * dW[:, c]
    return support, N, dN


class Axis:
    """CFE space on one uniform 1D mesh: quadrature tables and matrices.

    Phi  (n_q x n, sparse): N~ at the Gauss points, row q = e*n_g + g
    dPhi (n_q x n, sparse): dN~/dx = (2/h) dN~/dxi
    W    (n_q,)           : quadrature weights (h/2) w_g
    M, K (n x n, dense)   : int N~^T N~ dx and int B~^T B~ dx (eq. KxxMxx)
    """

    def __init__(self, n, lo=0.0, hi=1.0, s=2, p=2, a=12.0, ng=5):
        if s < 1 or p < 0 or s < p:
            raise ValueError("need s >= 1, 0 <= p <= s")
        if n < 2 * s + 2:
            raise ValueError("need at least 2s+2 nodes")
        self.n, self.lo, self.hi = int(n), float(lo), float(hi)
        self.s, self.p, self.a, self.ng = int(s), int(p), float(a), int(ng)
        self.h = (self.hi - self.lo) / (self.n - 1)
        self.x = self.lo + self.h * np.arange(self.n)
        xg, wg = np.polynomial.legendre.leggauss(self.ng)
        self.xi_g, self.w_g = xg, wg
        ne = self.n - 1
        self.nq = ne * self.ng
        self.xq = (self.lo + self.h * np.arange(ne)[:, None]
                   + (xg[None, :] + 1.0) * self.h / 2.0).ravel()
        self.W = np.tile(wg * self.h / 2.0, ne)
        rows, cols, vals, dvals = [], [], [], []
        for e in range(ne):
            support, N, dN = element_shape(e, self.n, self.s, self.p, self.a, xg)
            for g in range(self.ng):
                q = e * self.ng + g
                for c, k in enumerate(support):
                    rows.append(q); cols.append(k)
                    vals.append(N[g, c]); dvals.append(dN[g, c] * 2.0 / self.h)
        shape = (self.nq, self.n)
        self.Phi = sp.csr_matrix((vals, (rows, cols)), shape=shape)
        self.dPhi = sp.csr_matrix((dvals, (rows, cols)), shape=shape)
        Wd = sp.diags(self.W)
        self.M = np.asarray((self.Phi.T @ Wd @ self.Phi).todense())
        self.K = np.asarray((self.dPhi.T @ Wd @ self.dPhi).todense())
        self.bandwidth = 2 * self.s + 1

    def banded(self, A):
        """Lower banded storage ab[t, i] = A[i+t, i] for scipy.linalg.solveh_banded."""
        b = self.bandwidth
        ab = np.zeros((b + 1, self.n))
        for t in range(b + 1):
            ab[t, : self.n - t] = np.diagonal(A, -t)
        return ab

    def eval(self, coeffs):
        """Values at the Gauss points of a nodal coefficient vector / matrix."""
        return self.Phi @ coeffs

    def deval(self, coeffs):
        return self.dPhi @ coeffs
