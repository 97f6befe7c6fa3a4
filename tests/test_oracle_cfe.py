"""Pins of the oracle's 1D convolution-FE space against the paper and mathematics.

Everything here runs on the CPU; none of it touches the HIP library.
"""
import json
import os

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import cfe1d
from oracle.cfe1d import Axis, element_shape, patch_function, psi

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_kernel_values_printed():
    """App. B: the two kernel pieces at z = 0, 1/2, 1 and zero support beyond 1."""
    with open(os.path.join(GOLD, "cubic_kernel.json")) as f:
        vals = json.load(f)["values"]
    for z, v in vals:
        assert psi(z) == pytest.approx(v, abs=1e-15)


def test_kernel_is_cubic_bspline():
    """The kernel equals the centred cubic B-spline B3(2z) (library B-spline)."""
    b3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
    z = np.linspace(0.0, 1.2, 241)
    ref = np.nan_to_num(b3(2.0 * z))
    assert np.abs(psi(z) - ref).max() < 1e-14
    # C1 continuity at the piece boundary z = 1/2 from the derivative formula
    e = 1e-7
    assert abs(cfe1d.dpsi_dz(0.5 - e) - cfe1d.dpsi_dz(0.5 + e)) < 1e-5


def test_square_patch_is_lagrange():
    """p + 1 patch nodes: P is square, so L = P^-1, K = 0 and W is Lagrange interpolation."""
    xi_nodes = np.array([-3.0, -1.0, 1.0])
    xi = np.linspace(-1.0, 1.0, 17)
    W, dW = patch_function(xi, xi_nodes, 12.0, 2)
    for j in range(3):
        others = [xi_nodes[k] for k in range(3) if k != j]
        lag = np.prod([(xi - o) / (xi_nodes[j] - o) for o in others], axis=0)
        assert np.abs(W[:, j] - lag).max() < 1e-13
    _, _, L, K = cfe1d.patch_matrices(xi_nodes, 12.0, 2)
    assert np.abs(K).max() < 1e-12


@pytest.mark.parametrize("s,p", [(1, 1), (2, 1), (2, 2), (3, 2), (3, 3)])
def test_shape_function_count(s, p):
    """App. C: an interior element has 2s + 2 convolution shape functions."""
    n = 4 * s + 6
    support, N, dN = element_shape(2 * s + 1, n, s, p, 12.0, np.array([0.3]))
    assert len(support) == 2 * s + 2
    assert N.shape[1] == 2 * s + 2


@pytest.mark.parametrize("s,p", [(1, 1), (2, 1), (2, 2), (3, 3), (1, 0)])
def test_kronecker_and_partition_of_unity(s, p):
    """Sec. 3.2: Kronecker delta at the nodes and partition of unity, boundary elements included."""
    n = 3 * s + 8
    xi = np.linspace(-1.0, 1.0, 9)
    for e in range(n - 1):
        support, N, dN = element_shape(e, n, s, p, 12.0, np.array([-1.0, 1.0]))
        for r, node in enumerate((e, e + 1)):
            target = np.array([1.0 if k == node else 0.0 for k in support])
            assert np.abs(N[r] - target).max() < 1e-12
        _, N, dN = element_shape(e, n, s, p, 12.0, xi)
        assert np.abs(N.sum(axis=1) - 1.0).max() < 1e-12
        assert np.abs(dN.sum(axis=1)).max() < 1e-11


@pytest.mark.parametrize("s,p", [(1, 1), (2, 2), (3, 3), (3, 2)])
def test_polynomial_reproduction(s, p):
    """App. B reproducing conditions: polynomials of degree <= p and their derivatives are exact."""
    ax = Axis(3 * s + 9, -0.5, 2.0, s=s, p=p, a=12.0, ng=5)
    for t in range(p + 1):
        assert np.abs(ax.Phi @ ax.x ** t - ax.xq ** t).max() < 1e-11
        d = t * ax.xq ** (t - 1) if t else np.zeros(ax.nq)
        assert np.abs(ax.dPhi @ ax.x ** t - d).max() < 1e-9


def test_reproduction_fails_above_p():
    """Degree p + 1 is not reproduced (the pin above is not vacuous)."""
    ax = Axis(16, 0.0, 1.0, s=2, p=1, a=12.0, ng=5)
    assert np.abs(ax.Phi @ ax.x ** 2 - ax.xq ** 2).max() > 1e-5


@pytest.mark.parametrize("s,p,n", [(1, 1, 12), (2, 2, 20), (2, 2, 6), (3, 3, 17)])
def test_matrix_invariants(s, p, n):
    """eq. (KxxMxx): symmetric, M SPD, 1^T M 1 = |Omega|, K 1 = 0, exact quadratic energies."""
    lo, hi = 0.25, 1.75
    ax = Axis(n, lo, hi, s=s, p=p, a=12.0, ng=5)
    M, K = ax.M, ax.K
    assert np.abs(M - M.T).max() < 1e-14 * np.abs(M).max()
    assert np.abs(K - K.T).max() < 1e-14 * np.abs(K).max()
    assert np.linalg.eigvalsh(M).min() > 0
    assert np.linalg.eigvalsh(K).min() > -1e-12
    one = np.ones(n)
    assert one @ M @ one == pytest.approx(hi - lo, rel=1e-13)
    assert np.abs(K @ one).max() < 1e-11
    x = ax.x
    assert x @ K @ x == pytest.approx(hi - lo, rel=1e-11)
    assert x @ M @ x == pytest.approx((hi ** 3 - lo ** 3) / 3, rel=1e-12)
    if p >= 2:
        assert (x ** 2) @ K @ (x ** 2) == pytest.approx(4 * (hi ** 3 - lo ** 3) / 3, rel=1e-10)
    # banded with half-bandwidth 2s+1
    b = 2 * s + 1
    i, j = np.nonzero(np.abs(M) > 0)
    assert np.abs(i - j).max() <= b


def test_matrices_shift_invariant_interior():
    """Uniform mesh: interior rows of M and K are translates of each other."""
    ax = Axis(30, 0.0, 1.0, s=2, p=2, a=12.0, ng=5)
    b = 5
    r1 = ax.M[12, 12 - b:12 + b + 1]
    r2 = ax.M[17, 17 - b:17 + b + 1]
    assert np.abs(r1 - r2).max() < 1e-15 * 1e3


def test_quadrature_exact_for_mass():
    """Gauss 5 vs 8 points: mass and stiffness unchanged (N~ is a degree-4 polynomial per element at a=12)."""
    a5 = Axis(14, 0.0, 1.0, s=2, p=2, a=12.0, ng=5)
    a8 = Axis(14, 0.0, 1.0, s=2, p=2, a=12.0, ng=8)
    assert np.abs(a5.M - a8.M).max() < 1e-15 * 1e2
    assert np.abs(a5.K - a8.K).max() < 1e-12


def test_invalid_parameters():
    with pytest.raises(ValueError):
        Axis(10, s=1, p=2)
    with pytest.raises(ValueError):
        Axis(5, s=2, p=2)
