"""Pins of the oracle's total-variation indicator, its statistics and flags
(paper eqs. tv, refinement-criterion, chebychev): brute force with an
independent polynomial derivative, exact rational statistics, a linear field
with a closed-form TV, and Chebyshev/Cantelli bounds."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I


def periodic(nx):
    return dict(nx=nx, nz=nx, max_level=0, x0=0.0, z0=0.0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4)


def brute_tv_rho(Q, N, nx):
    """TV of rho per cell: derivative of the interpolating polynomial from
    numpy's polyfit (not the derivative matrix), Gauss quadrature with numpy's
    Gauss-Legendre rule on the reference element (weights summing to one) of
    the physical gradient (1/h derivative scaling): the mean of
    |df/dx| + |df/dz| over the cell."""
    n = N + 1
    x, w = np.polynomial.legendre.leggauss(n)
    xi, w = (x + 1) / 2, w / 2
    h = 1.0 / nx
    out = []
    for c in range(Q.shape[0]):
        f = Q[c, 0]
        dx = np.zeros((n, n))
        dz = np.zeros((n, n))
        for j in range(n):
            pc = np.polynomial.polynomial.polyfit(xi, f[j, :], N)
            dx[j, :] = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(pc))
        for i in range(n):
            pc = np.polynomial.polynomial.polyfit(xi, f[:, i], N)
            dz[:, i] = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(pc))
        integrand = (np.abs(dx) + np.abs(dz)) / h
        out.append(np.sum(np.outer(w, w) * integrand))
    return np.array(out)


def exact_flags(tv, Tr, Tc):
    """Mean and population variance in exact rationals of the float TVs;
    comparisons tv >= mu + T sigma decided exactly."""
    fr = [Fraction(float(v)) for v in tv]
    C = len(fr)
    mu = sum(fr) / C
    var = sum((v - mu) ** 2 for v in fr) / C
    def ge(v, T):   # v >= mu + T*sigma  <=>  v - mu >= T*sqrt(var)
        d = v - mu
        T = Fraction(T)
        if T >= 0:
            return d >= 0 and d * d >= T * T * var
        return d >= 0 or d * d <= T * T * var
    flags = []
    for v in fr:
        if var == 0:
            flags.append(0)
        elif ge(v, Tr):
            flags.append(1)
        elif not ge(v, Tc):
            flags.append(-1)
        else:
            flags.append(0)
    return np.array(flags, dtype=np.int8), mu, var


@pytest.mark.parametrize("N", [1, 2, 3])
def test_tv_brute_force_and_exact_flags(N):
    nx = 3
    Q = I.random_state_cfd(nx * nx, N, seed=20 + N)
    phys = dict(I.CFD, N=N, mu=0.0, mms=0)
    Tr, Tc = 0.5, -0.5
    tv, flags, st = O.tv(phys, periodic(nx), Q, O.VAR_RHO, Tr, Tc)
    bt = brute_tv_rho(Q, N, nx)
    assert np.max(np.abs(tv - bt)) <= 1e-14 * np.max(bt) * 10
    ef, mu, var = exact_flags(tv, Tr, Tc)
    assert abs(st[1] - float(mu)) <= 1e-14 * float(mu)
    assert abs(st[2] - math.sqrt(float(var))) <= 1e-13 * math.sqrt(float(var))
    sig = math.sqrt(float(var))
    near = np.minimum(np.abs(tv - (float(mu) + Tr * sig)), np.abs(tv - (float(mu) + Tc * sig)))
    ok = (flags == ef) | (near <= 1e-12 * np.abs(float(mu) + Tr * sig))
    assert ok.all()
    assert st[0] == nx * nx


def test_tv_of_linear_field():
    """f = a x + b z: TV = |a| + |b| on every cell, whatever its size."""
    N, nx = 3, 4
    n = N + 1
    b = O.basis(N)
    h = 1.0 / nx
    a, bb = -0.3, 0.7
    Q = np.zeros((nx * nx, 4, n, n))
    for c in range(nx * nx):
        i, j = c % nx, c // nx
        X = i * h + h * b["xi"]
        Z = j * h + h * b["xi"]
        Q[c, 0] = 2.0 + a * X[None, :] + bb * Z[:, None]
        Q[c, 3] = 2.5
    tv, flags, st = O.tv(dict(I.CFD, N=N, mu=0.0, mms=0), periodic(nx), Q, O.VAR_RHO, 1.0, -1.0)
    assert np.max(np.abs(tv - (abs(a) + abs(bb)))) <= 1e-14
    # identical TVs: sigma ~ 0 within rounding of the TV (|a| + |b| = 1)
    assert st[2] <= 1e-14 * (abs(a) + abs(bb))


def test_tv_of_linear_field_on_a_refined_mesh():
    """Cell-size independence of the indicator: on a mesh with coarse cells
    and 3x3 children, a linear field f = a x + b z has TV = |a| + |b| on
    every leaf, so a refined family carries its parent's TV (the indicator
    compares gradients, not cell sizes)."""
    N, nx = 2, 3
    n = N + 1
    b = O.basis(N)
    a, bb = 0.4, -1.1
    leaves = I.refined_leaves(nx, nx, [(1, 1), (0, 2)])
    mesh = dict(periodic(nx), max_level=1, leaves=leaves)
    Q = np.zeros((len(leaves), 4, n, n))
    for c, (l, i, j) in enumerate(leaves):
        h = 1.0 / (nx * 3 ** l)
        X = i * h + h * b["xi"]
        Z = j * h + h * b["xi"]
        Q[c, 0] = 2.0 + a * X[None, :] + bb * Z[:, None]
        Q[c, 3] = 2.5
    tv, _, _ = O.tv(dict(I.CFD, N=N, mu=0.0, mms=0), mesh, Q, O.VAR_RHO, 1.0, -1.0)
    assert np.max(np.abs(tv - (abs(a) + abs(bb)))) <= 1e-13


def test_constant_tv_keeps_everything():
    N, nx = 2, 3
    n = N + 1
    Q = np.zeros((nx * nx, 4, n, n))
    Q[:, 0], Q[:, 3] = 1.0, 2.5
    tv, flags, st = O.tv(dict(I.CFD, N=N, mu=0.0, mms=0), periodic(nx), Q, O.VAR_RHO, 1.0, -1.0)
    # rows of D sum to zero up to rounding; equal TVs give sigma == 0 exactly
    assert np.max(tv) <= 1e-15 and st[2] == 0 and np.all(flags == 0)


def test_theta_tv_vanishes_on_background():
    """The hydrostatic background has constant potential temperature, so the
    TV of theta is zero up to rounding."""
    w = I.bubble(9, 4, bubbles=[])
    Q = O.ic(w["phys"], w["mesh"], "bubbles", [])
    tv, _, _ = O.tv(w["phys"], w["mesh"], Q, O.VAR_THETA, 1.5, -0.5)
    # mean gradient of theta on 111 m cells: rounding of theta (300 K) / h
    assert np.max(tv) <= 1e-9 * 300.0 / (1000.0 / 9)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("Tr", [0.5, 1.5, 2.5])
def test_chebyshev_cantelli_bound_on_refinement_fraction(seed, Tr):
    """Chebyshev (paper eq. chebychev) and its one-sided form bound the
    fraction of cells flagged for refinement: #refine <= C / (1 + Tr^2)."""
    rng = np.random.default_rng(seed)
    nx, N = 5, 2
    Q = I.random_state_cfd(nx * nx, N, seed=100 + seed)
    # make the field heavy-tailed across cells
    Q[:, 0] = 1.0 + (Q[:, 0] - 1.0) * rng.pareto(1.5, nx * nx)[:, None, None] * 0.2
    Q[:, 0] = np.maximum(Q[:, 0], 0.2)
    tv, flags, st = O.tv(dict(I.CFD, N=N, mu=0.0, mms=0), periodic(nx), Q, O.VAR_RHO, Tr, -0.5)
    C = nx * nx
    assert (flags == 1).sum() <= C / (1 + Tr * Tr) + 1e-12
    # coarsen: tv < mu - 0.5 sigma  -> fraction <= 1/(1+0.25)
    assert (flags == -1).sum() <= C / 1.25 + 1e-12


def test_input_constants_follow_paper():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    cb = I.cosine_bubble()
    assert (cb[1], cb[2], cb[4], cb[5]) == tuple(g["cosine_bubble"][k] for k in ("A", "a", "xc", "zc"))
    cold = I.cold_bubble()
    assert (cold[1], cold[2], cold[3], cold[4], cold[5]) == tuple(
        g["cold_bubble"][k] for k in ("A", "a", "s", "xc", "zc"))
    c = g["cfd_constants"]
    assert I.CFD["gamma"] == c["gamma"] and I.CFD["Pr"] == c["Pr"]
    assert abs(I.CFD["cp"] - I.CFD["R"] - c["c_v"]) < 1e-15
    a = g["atmosphere_constants"]
    assert I.ATMO["gamma"] == a["gamma"] and I.ATMO["Pr"] == a["Pr"] and I.ATMO["p0"] == a["p0"]
