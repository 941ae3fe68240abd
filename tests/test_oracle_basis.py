"""Pins of the oracle's quadrature and basis matrices against closed forms,
numpy's Gauss-Legendre rule and exactness properties (textbook facts, not the
oracle's own formulas)."""
import math

import numpy as np
import pytest

from oracle import oracle as O

NS = list(range(0, 10))


@pytest.mark.parametrize("N", NS)
def test_gl_against_numpy_leggauss(N):
    b = O.basis(N)
    x, w = np.polynomial.legendre.leggauss(N + 1)
    # numpy's rule carries a few ulp of its own rounding
    assert np.max(np.abs(b["xi"] - (x + 1) / 2)) <= 2e-15
    assert np.max(np.abs(b["w"] - w / 2)) <= 2e-15


def test_gl_closed_forms():
    b = O.basis(1)
    assert np.allclose(b["xi"], [0.5 - 0.5 / math.sqrt(3), 0.5 + 0.5 / math.sqrt(3)], atol=4e-16, rtol=0)
    assert np.allclose(b["w"], [0.5, 0.5], atol=4e-16, rtol=0)
    b = O.basis(2)
    r = math.sqrt(3 / 5) / 2
    assert np.allclose(b["xi"], [0.5 - r, 0.5, 0.5 + r], atol=4e-16, rtol=0)
    assert np.allclose(b["w"], [5 / 18, 8 / 18, 5 / 18], atol=4e-16, rtol=0)


@pytest.mark.parametrize("N", NS)
def test_gl_exactness_and_symmetry(N):
    b = O.basis(N)
    for k in range(2 * N + 2):
        assert abs(np.sum(b["w"] * b["xi"] ** k) - 1.0 / (k + 1)) <= 4e-16 * (k + 1)
    assert np.max(np.abs(b["xi"] + b["xi"][::-1] - 1.0)) <= 4e-16
    assert np.max(np.abs(b["w"] - b["w"][::-1])) <= 4e-16


@pytest.mark.parametrize("N", range(1, 10))
def test_derivative_matrix_exact_on_polynomials(N):
    b = O.basis(N)
    xi = b["xi"]
    for k in range(N + 1):
        f = xi ** k
        df = k * xi ** (k - 1) if k else np.zeros_like(xi)
        assert np.max(np.abs(b["D"] @ f - df)) <= 2e-14 * max(1, k * N)


@pytest.mark.parametrize("N", range(1, 10))
def test_boundary_values_and_integration_by_parts(N):
    b = O.basis(N)
    xi = b["xi"]
    for k in range(N + 1):
        f = xi ** k
        assert abs(b["e0"] @ f - (1.0 if k == 0 else 0.0)) <= 5e-14
        assert abs(b["e1"] @ f - 1.0) <= 5e-14
    # integral of phi_i' over [0,1] = phi_i(1) - phi_i(0)
    assert np.max(np.abs(b["w"] @ b["D"] - (b["e1"] - b["e0"]))) <= 2e-14


@pytest.mark.parametrize("N", range(1, 10))
def test_time_matrix_integrates_polynomials(N):
    """q = Q + dt P R is the DG-in-time solution of dq/dt = R with upwind value
    Q at tau=0; it integrates exactly: (P r)_a = int_0^{tau_a} r for r of
    degree <= N-1 (the exact solution is then in the space)."""
    b = O.basis(N)
    xi = b["xi"]
    for k in range(N):
        lhs = b["P"] @ (xi ** k)
        rhs = xi ** (k + 1) / (k + 1)
        assert np.max(np.abs(lhs - rhs)) <= 2e-14


@pytest.mark.parametrize("N", [1, 3, 6])
def test_lagrange_at_points(N):
    b = O.basis(N)
    xs = [0.0, 1 / 3, 0.5, 2 / 3, 0.987]
    for x in xs:
        vals = np.array([O.lagrange(N, j, x) for j in range(N + 1)])
        # interpolate monomials: sum_j phi_j(x) xi_j^k = x^k
        for k in range(N + 1):
            assert abs(vals @ (b["xi"] ** k) - x ** k) <= 1e-13
