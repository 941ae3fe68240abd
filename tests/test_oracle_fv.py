"""Pins of the oracle's MUSCL-Hancock finite-volume scheme (van Albada
limiter, Rusanov flux, no viscosity): properties of the published limiter,
exactness of the Hancock half step for linear advection, preservation of
constant states, conservation, symmetries, the total-variation bound, the
exact solution of Sod's shock tube and second-order convergence."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I

WALL, PER = I.BC_WALL, I.BC_PERIODIC


def cfd(cfl=0.9):
    return dict(I.CFD, N=0, picard_iters=0, mu=0.0, mms=0, cfl=cfl)


def grid(nx, nz, L=1.0, bc=PER):
    return dict(nx=nx, nz=nz, x0=0.0, z0=0.0, Lx=L, Lz=L * nz / nx, bc=[bc] * 4 if np.isscalar(bc) else list(bc))


# ------------------------------------------------------------------ limiter
def test_van_albada_limiter_properties():
    """phi(r) = (r^2 + r) / (r^2 + 1): the limited slope is b phi(a/b) for
    same-signed differences, 0 otherwise; symmetric in (a, b), exact on
    equal differences, homogeneous of degree one, bounded by the larger
    difference and by twice the smaller (the TVD region), and phi(1/r) =
    phi(r) / r."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b = rng.uniform(-3, 3, 2)
        s = O.van_albada(a, b)
        if a * b <= 0:
            assert s == 0.0
            continue
        r = a / b
        assert math.isclose(s, b * (r * r + r) / (r * r + 1), rel_tol=1e-14)
        assert math.isclose(s, O.van_albada(b, a), rel_tol=1e-15)
        assert math.isclose(O.van_albada(2.5 * a, 2.5 * b), 2.5 * s, rel_tol=1e-14)
        assert abs(s) <= max(abs(a), abs(b)) * (1 + 1e-15)
        assert abs(s) <= 2 * min(abs(a), abs(b)) * (1 + 1e-15)
        phi = lambda x: (x * x + x) / (x * x + 1)
        assert math.isclose(phi(1 / r), phi(r) / r, rel_tol=1e-13)
    assert O.van_albada(0.7, 0.7) == 0.7
    assert O.van_albada(0.0, 1.0) == 0.0


# ------------------------------------------------------- state constructors
def advected(rho, u, w, p, gamma=1.4):
    """Conserved state of density rho moving with constant (u, w) at constant p."""
    rho = np.asarray(rho, dtype=np.float64)
    Q = np.empty(rho.shape + (4,))
    Q[..., 0] = rho
    Q[..., 1] = rho * u
    Q[..., 2] = rho * w
    Q[..., 3] = p / (gamma - 1) + 0.5 * rho * (u * u + w * w)
    return Q


def centres(mesh):
    h = mesh["Lx"] / mesh["nx"]
    x = mesh["x0"] + (np.arange(mesh["nx"]) + 0.5) * h
    z = mesh["z0"] + (np.arange(mesh["nz"]) + 0.5) * h
    return np.meshgrid(x, z)   # [nz][nx]


def test_hancock_half_step_exact_for_linear_advection():
    """rho linear in x, constant velocity and pressure: the van Albada slope of
    a linear profile is exact, and the evolved face values equal the exact
    solution rho(x_f - u dt/2) at the face at half the step (cells away from
    the periodic seam)."""
    m = grid(12, 3)
    h = m["Lx"] / m["nx"]
    X, Z = centres(m)
    u, w, p = 0.6, 0.0, 1.0
    rho = 1.0 + 0.3 * X
    Q = advected(rho, u, w, p).reshape(-1, 4)
    dt = 0.02
    E, inc = O.fv_predict(cfd(), m, Q, dt)
    E = E.reshape(3, 12, 4, 4)
    for i in range(2, 10):
        xw, xe = i * h, (i + 1) * h
        for f, xf in ((0, xw), (1, xe)):
            exact = 1.0 + 0.3 * (xf - u * dt / 2)
            assert np.allclose(E[:, i, f, 0], exact, rtol=0, atol=1e-14)
            assert np.allclose(E[:, i, f, 1], u * exact, rtol=0, atol=1e-14)
            assert np.allclose(E[:, i, f, 3], p / 0.4 + 0.5 * exact * u * u, rtol=0, atol=1e-13)
        # z faces: no variation along z, so the face values are the advected centre value
        exact_c = 1.0 + 0.3 * ((i + 0.5) * h - u * dt / 2)
        assert np.allclose(E[:, i, 2:, 0], exact_c, rtol=0, atol=1e-14)


def test_constant_state_preserved():
    m = grid(5, 4)
    Q = np.tile([1.2, 0.3, -0.2, 2.6], (20, 1))
    assert np.max(np.abs(O.fv_step(cfd(), m, Q, 0.01) - Q)) <= 1e-15 * 2.6


def test_conservation_on_periodic_grid():
    m = grid(8, 6)
    rng = np.random.default_rng(3)
    Q = I.random_state_cfd(48, 0, seed=3).reshape(48, 4)
    dt = O.fv_dt(cfd(), m, Q)
    out = O.fv_step(cfd(), m, Q, dt)
    assert np.all(np.abs(out.sum(axis=0) - Q.sum(axis=0)) <= 1e-13 * np.abs(Q).sum(axis=0))
    assert np.max(np.abs(out - Q)) > 1e-4


def test_mirror_and_transpose_symmetry():
    """x -> -x (x momentum negated) and x <-> z (momenta swapped) commute
    with the step on a periodic grid without gravity."""
    nx = nz = 6
    m = grid(nx, nz)
    Q = I.random_state_cfd(36, 0, seed=9).reshape(nz, nx, 4)
    dt = O.fv_dt(cfd(), m, Q.reshape(-1, 4))
    step = lambda S: O.fv_step(cfd(), m, S.reshape(-1, 4), dt).reshape(nz, nx, 4)
    mirror = lambda S: S[:, ::-1] * np.array([1, -1, 1, 1])
    a, b = mirror(step(Q)), step(mirror(Q))
    assert np.max(np.abs(a - b)) <= 1e-14 * 3
    trans = lambda S: S.transpose(1, 0, 2)[..., [0, 2, 1, 3]]
    a, b = trans(step(Q)), step(trans(Q))
    assert np.max(np.abs(a - b)) <= 1e-14 * 3


def test_total_variation_of_an_advected_step_does_not_grow():
    """A density step carried by a constant flow at constant pressure (a
    contact): the scheme keeps velocity and pressure constant and the total
    variation of the density does not grow (van Albada is a TVD limiter)."""
    m = grid(64, 1)
    X, _ = centres(m)
    rho = np.where((X > 0.25) & (X < 0.6), 2.0, 1.0)
    Q = advected(rho, 0.8, 0.0, 1.0).reshape(-1, 4)
    tv0 = np.abs(np.diff(np.r_[Q[:, 0], Q[0, 0]])).sum()
    for _ in range(60):
        Q = O.fv_step(cfd(), m, Q, O.fv_dt(cfd(), m, Q))
        tv = np.abs(np.diff(np.r_[Q[:, 0], Q[0, 0]])).sum()
        assert tv <= tv0 * (1 + 1e-12)
        tv0 = tv
    assert np.allclose(Q[:, 1] / Q[:, 0], 0.8, rtol=0, atol=1e-12)
    p = 0.4 * (Q[:, 3] - 0.5 * Q[:, 1] ** 2 / Q[:, 0])
    assert np.allclose(p, 1.0, rtol=0, atol=1e-12)


# ------------------------------------------------- exact Riemann solution
def sod_exact(x, t, x0=0.5, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), g=1.4):
    """Density of the exact solution of the Riemann problem (textbook exact
    solver: Newton on the pressure function, then sampling)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fk(p, r, pk, ck):
        if p > pk:
            A, B = 2 / ((g + 1) * r), (g - 1) / (g + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B)), math.sqrt(A / (B + p)) * (1 - (p - pk) / (2 * (B + p)))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1), (p / pk) ** (-(g + 1) / (2 * g)) / (r * ck)

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, cl)
        f2, d2 = fk(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    f1, _ = fk(p, rl, pl, cl)
    f2, _ = fk(p, rr, pr, cr)
    us = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    out = np.empty_like(x)
    for k, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:   # left of the contact
            if p > pl:
                SL = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
                out[k] = rl if s <= SL else rl * ((p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1))
            else:
                cs = cl * (p / pl) ** ((g - 1) / (2 * g))
                if s <= ul - cl:
                    out[k] = rl
                elif s >= us - cs:
                    out[k] = rl * (p / pl) ** (1 / g)
                else:
                    out[k] = rl * (2 / (g + 1) + (g - 1) / ((g + 1) * cl) * (ul - s)) ** (2 / (g - 1))
        else:
            if p > pr:
                SR = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
                out[k] = rr if s >= SR else rr * ((p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1))
            else:
                cs = cr * (p / pr) ** ((g - 1) / (2 * g))
                if s >= ur + cr:
                    out[k] = rr
                elif s <= us + cs:
                    out[k] = rr * (p / pr) ** (1 / g)
                else:
                    out[k] = rr * (2 / (g + 1) - (g - 1) / ((g + 1) * cr) * (ur - s)) ** (2 / (g - 1))
    return out


def sod_run(nx, T=0.2):
    m = grid(nx, 1, bc=[WALL, WALL, PER, PER])
    X, _ = centres(m)
    x = X[0]
    Q = np.where(x[:, None] < 0.5, [1.0, 0.0, 0.0, 1.0 / 0.4], [0.125, 0.0, 0.0, 0.1 / 0.4])
    t = 0.0
    ph = cfd(0.9)
    while t < T - 1e-15:
        dt = min(O.fv_dt(ph, m, Q), T - t)
        Q = O.fv_step(ph, m, Q, dt)
        t += dt
    return x, Q


def test_sod_shock_tube_against_exact_solution():
    """Sod's problem to t = 0.2 (walls far from the waves): the L1 density
    error against the exact solution is small and falls with the cell size
    (first order at the discontinuities)."""
    errs = []
    for nx in (100, 200, 400):
        x, Q = sod_run(nx)
        errs.append(np.mean(np.abs(Q[:, 0] - sod_exact(x, 0.2))))
    assert errs[2] < 6e-3, errs
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1], errs


def test_second_order_on_a_smooth_wave():
    """Advected density wave (periodic, constant velocity and pressure): the
    L1 error at t = 0.25 falls by about four per halving of the cell size."""
    ph = dict(cfd(0.9), mms_amp=0.1, mms_u=0.5, mms_w=0.25, mms_kx=2 * math.pi, mms_kz=2 * math.pi, mms_p=1.0)
    errs = []
    for nx in (32, 64):
        m = grid(nx, nx)
        Q = O.fv_ic(ph, m, "wave")
        t, T = 0.0, 0.25
        while t < T - 1e-15:
            dt = min(O.fv_dt(ph, m, Q), T - t)
            Q = O.fv_step(ph, m, Q, dt)
            t += dt
        ex = O.fv_ic(ph, m, "wave", t0=T)
        errs.append(np.mean(np.abs(Q[:, 0] - ex[:, 0])))
    order = math.log2(errs[0] / errs[1])
    assert order > 1.7, (errs, order)


def test_resting_atmosphere_stays_nearly_at_rest():
    """Hydrostatic background in a walled box (cells of 15.9 m): the linear
    reconstruction of the background is not exactly balanced; the spurious
    velocities stay below 1e-5 m/s over 50 steps."""
    w = I.bubble(63, 6)
    ph = dict(w["phys"], N=0, mu=0.0, cfl=0.9)
    Q = O.fv_ic(ph, w["mesh"], "bubbles", [])
    Q2, t = O.fv_run(ph, w["mesh"], Q, 0.0, 50)
    assert t > 0.5
    assert np.max(np.abs(Q2[:, 1:3] / Q2[:, :1])) < 1e-5


def test_buoyancy_of_a_bubble_at_rest():
    """A warm bubble at rest at the background pressure: over the first step
    the vertical momentum changes by the buoyancy -g (rho - rho_bar) dt
    (the pressure stays hydrostatic to the reconstruction's accuracy), with
    the sign that lifts the warm (lighter) air."""
    w = I.bubble(63, 6)
    ph = dict(w["phys"], N=0, mu=0.0, cfl=0.9)
    Q = O.fv_ic(ph, w["mesh"], "bubbles", w["bubbles"])
    Qb = O.fv_ic(ph, w["mesh"], "bubbles", [])
    dt = O.fv_dt(ph, w["mesh"], Q)
    out = O.fv_step(ph, w["mesh"], Q, dt)
    buoy = -ph["g"] * (Q[:, 0] - Qb[:, 0]) * dt
    core = np.abs(buoy) > 0.5 * np.abs(buoy).max()
    assert core.sum() > 20
    ratio = out[core, 2] / buoy[core]
    assert np.all(np.abs(ratio - 1) < 0.02), (ratio.min(), ratio.max())
    assert np.all(out[core, 2] > 0)
    # the Hancock half step moves the face values by half a step of the full
    # equation, source included: the face values' vertical momentum is half
    # the buoyancy impulse
    E, inc = O.fv_predict(ph, w["mesh"], Q, dt)
    for f in range(4):
        r = E[core, f, 2] / (0.5 * buoy[core])
        assert np.all(np.abs(r - 1) < 0.02), (f, r.min(), r.max())
