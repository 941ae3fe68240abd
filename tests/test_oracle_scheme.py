"""Pins of the oracle's ADER-DG step against what the mathematics fixes:
exact preservation of constant states, exactness of the space-time predictor
for linear advection of polynomial data, conservation on periodic grids,
reflection and x<->z symmetry, order of convergence on a manufactured
solution, and hydrostatic balance of the resting atmosphere."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I


def cfd(N, mu=0.01, mms=0):
    return dict(I.CFD, N=N, picard_iters=0, mu=mu, mms=mms, cfl=0.5)


def periodic(nx, nz=None):
    return dict(nx=nx, nz=nz or nx, max_level=0, x0=0.0, z0=0.0, Lx=1.0, Lz=1.0 * (nz or nx) / nx,
                bc=[I.BC_PERIODIC] * 4)


@pytest.mark.parametrize("N", range(1, 8))
def test_constant_state_is_preserved(N):
    n = N + 1
    mesh = periodic(3)
    Q = np.zeros((9, 4, n, n))
    Q[:, 0], Q[:, 1], Q[:, 2], Q[:, 3] = 1.1, 0.3, -0.2, 2.7
    out = O.step(cfd(N, mu=0.05), mesh, Q, 0.0, 1e-2)
    assert np.max(np.abs(out - Q)) <= 1e-13 * 2.7


@pytest.mark.parametrize("N", range(1, 6))
@pytest.mark.parametrize("axis", [0, 1])
def test_predictor_exact_for_linear_advection(N, axis):
    """mu = 0, constant velocity a along one axis, constant pressure, density a
    polynomial of degree N along that axis: the space-time solution
    rho(x - a t) is a polynomial of degree N in (x, t), and the Picard sweep
    is nilpotent on it, so N+1 sweeps reproduce it exactly; the time-averaged
    face values then equal the exact time average of rho at the face."""
    n = N + 1
    b = O.basis(N)
    xi = b["xi"]
    nx = 3
    h = 1.0 / nx
    a, p = 0.7, 1.0
    coef = np.array([1.0, 0.1, 0.05, -0.02, 0.01, 0.004])[: N + 1]
    rho_f = lambda s: np.polynomial.polynomial.polyval(s, coef)
    Q = np.zeros((nx * nx, 4, n, n))
    for c in range(nx * nx):
        i, j = c % nx, c // nx
        s = (i if axis == 0 else j) * h + h * xi
        r = np.repeat(rho_f(s)[None, :], n, 0) if axis == 0 else np.repeat(rho_f(s)[:, None], n, 1)
        Q[c, 0] = r
        Q[c, 1 + axis] = a * r
        Q[c, 3] = p / 0.4 + 0.5 * r * a * a
    dt = 0.02
    _, FD = O.predictor(cfd(N, mu=0.0), periodic(nx), Q, 0.0, dt)
    # cell 0, upper face along the axis (+x: face 1, +z: face 3)
    exact = sum(b["w"][k] * rho_f(h - a * dt * xi[k]) for k in range(n))
    face = 1 if axis == 0 else 3
    assert np.max(np.abs(FD[0, face, 0, 0, :] - exact)) <= 2e-14
    # mass flux at the face = a * average density
    assert np.max(np.abs(FD[0, face, 1, 0, :] - a * exact)) <= 2e-14


@pytest.mark.parametrize("N", [2, 4])
def test_periodic_conservation(N):
    n = N + 1
    nx = 4
    mesh = periodic(nx)
    Q = I.random_state_cfd(nx * nx, N, seed=11 + N)
    b = O.basis(N)
    W = np.outer(b["w"], b["w"]) / nx ** 2
    before = np.einsum("cvji,ji->v", Q, W)
    out = O.step(cfd(N, mu=0.02), mesh, Q, 0.0, 2e-3)
    after = np.einsum("cvji,ji->v", out, W)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())
    assert np.max(np.abs(out - Q)) > 1e-6   # the state did change


def test_reflection_and_transpose_symmetry():
    """Mirroring x -> 1-x (momentum_x negated) and swapping x <-> z (momenta
    swapped) commute with the step: catches swapped indices and sign slips."""
    N, nx = 3, 3
    mesh = periodic(nx)
    Q = I.random_state_cfd(nx * nx, N, seed=5)
    phys = cfd(N, mu=0.03)
    dt = 2e-3
    out = O.step(phys, mesh, Q, 0.0, dt)
    grid = lambda A: A.reshape(nx, nx, 4, N + 1, N + 1)          # [j][i][v][jz][ix]
    flat = lambda G: np.ascontiguousarray(G).reshape(nx * nx, 4, N + 1, N + 1)
    # mirror in x
    G = grid(Q)[:, ::-1, :, :, ::-1].copy()
    G[:, :, 1] *= -1
    outm = grid(O.step(phys, mesh, flat(G), 0.0, dt))[:, ::-1, :, :, ::-1].copy()
    outm[:, :, 1] *= -1
    assert np.max(np.abs(flat(outm) - out)) <= 1e-13
    # transpose x <-> z
    G = grid(Q).transpose(1, 0, 2, 4, 3)[:, :, [0, 2, 1, 3]]
    outt = grid(O.step(phys, mesh, flat(G), 0.0, dt)).transpose(1, 0, 2, 4, 3)[:, :, [0, 2, 1, 3]]
    assert np.max(np.abs(flat(outt) - out)) <= 1e-13


def _mms_error(N, nx, mu, T=0.05):
    w = I.mms_small(N=N, nx=nx, mu=mu)
    phys = w["phys"]
    # asymmetric wave: different speeds and wave numbers along x and z
    phys.update(mms_u=0.5, mms_w=0.25, mms_kx=2 * math.pi, mms_kz=4 * math.pi)
    Q = O.ic(phys, w["mesh"], "mms")
    ns = int(math.ceil(T / O.dt(phys, w["mesh"], Q)))
    Q, _ = O.run(phys, w["mesh"], Q, 0.0, ns, T / ns)
    Qe = O.ic(phys, w["mesh"], "mms", t0=T)
    b = O.basis(N)
    W = np.outer(b["w"], b["w"]) / nx ** 2
    return math.sqrt(np.sum(W[None] * (Q[:, 0] - Qe[:, 0]) ** 2))


def _orders(errs, grids):
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1)), errs
    return [math.log(errs[k] / errs[k + 1], grids[k + 1] / grids[k]) for k in range(len(errs) - 1)]


# lower bounds of the observed order on the finest pair of three grids
# (8, 16, 32 cells), about 0.3 below the measured values and above N, so a
# one-order loss fails: the Rusanov speed |v.n| + c (far above the speed of
# the advected density wave, |v.n| <= 0.5 against c ~ 1.2) makes even orders
# pre-asymptotic at these sizes (N = 2 measures 2.2-2.5 here and rises to
# 2.7 at 128 cells; with c ten times smaller it reaches 3.0 at 32 cells)
DENSITY_WAVE_EOC = {(1, 0.0): 2.4, (2, 0.0): 2.0, (3, 0.0): 4.0,
                    (1, 0.01): 2.7, (2, 0.01): 2.3, (3, 0.01): 3.9}


@pytest.mark.parametrize("N,mu", sorted(DENSITY_WAVE_EOC))
def test_mms_convergence_order(N, mu):
    """Order of the error in rho on the manufactured density wave (measured
    2.63 / 2.17 / 4.37 at mu = 0 and 2.97 / 2.49 / 4.23 at mu = 0.01 for
    N = 1 / 2 / 3 on 16 -> 32 cells)."""
    grids = (8, 16, 32)
    eoc = _orders([_mms_error(N, nx, mu) for nx in grids], grids)
    assert eoc[-1] >= DENSITY_WAVE_EOC[(N, mu)], eoc


def _paper_mms_error(N, nx, mu):
    """L2 error of rho at t = 0.5 on the paper's manufactured solution
    (CFD scenarios, eq. manufactured-solution): periodic [0,10]^2, CFD
    constants, Courant factor 0.5."""
    w = I.paper_mms(N, nx, mu)
    phys, mesh, T = w["phys"], w["mesh"], w["t_end"]
    Q = O.ic(phys, mesh, "paper_mms")
    ns = int(math.ceil(T / O.dt(phys, mesh, Q)))
    Q, _ = O.run(phys, mesh, Q, 0.0, ns, T / ns)
    Qe = O.ic(phys, mesh, "paper_mms", t0=T)
    b = O.basis(N)
    W = np.outer(b["w"], b["w"]) * (10.0 / nx) ** 2
    return math.sqrt(np.sum(W[None] * (Q[:, 0] - Qe[:, 0]) ** 2))


# Paper's wave without viscosity: the order N+1 of the paper's convergence
# figure on the finest of three grids (measured 2.80, 3.97, 4.57, 5.62, 7.24
# for N = 2..6; coarser pairs are pre-asymptotic, e.g. 5.31 for N = 6 on
# 4 -> 8 cells); bounds >= N + 0.6.
PAPER_WAVE_INVISCID = {2: ((8, 16, 32), 2.6), 3: ((8, 16, 32), 3.7), 4: ((4, 8, 16), 4.3),
                       5: ((4, 8, 16), 5.4), 6: ((4, 8, 16), 6.6)}


@pytest.mark.parametrize("N", sorted(PAPER_WAVE_INVISCID))
def test_paper_mms_convergence_inviscid(N):
    grids, bound = PAPER_WAVE_INVISCID[N]
    eoc = _orders([_paper_mms_error(N, nx, 0.0) for nx in grids], grids)
    assert eoc[-1] >= bound, eoc


# Paper's wave at the paper's viscosity mu = 0.1: the viscous face flux (the
# average of both sides' element-local viscous fluxes plus the state jump
# times 2 eta lambda_v, eta ~ (2N+1)/h, with no symmetrising term) converges
# at about order N here: measured 2.52 (N=1, 16->32), 2.71 (N=2, 16->32),
# 2.95 (N=3, 8->16; 2.68 on 32->64), 4.10, 4.73, 5.91 (N=4..6, 8->16); the
# paper notes diminishing returns at large orders.  Bounds ~0.3 below.
PAPER_WAVE_VISCOUS = {1: ((8, 16, 32), 2.2), 2: ((8, 16, 32), 2.4), 3: ((4, 8, 16), 2.7),
                      4: ((4, 8, 16), 3.8), 5: ((4, 8, 16), 4.4), 6: ((4, 8, 16), 5.6)}


@pytest.mark.parametrize("N", sorted(PAPER_WAVE_VISCOUS))
def test_paper_mms_convergence_viscous(N):
    grids, bound = PAPER_WAVE_VISCOUS[N]
    eoc = _orders([_paper_mms_error(N, nx, 0.1) for nx in grids], grids)
    assert eoc[-1] >= bound, eoc


@pytest.mark.parametrize("N,nx,tol", [(4, 9, 1e-12), (6, 9, 1e-12)])
def test_resting_atmosphere_stays_at_rest(N, nx, tol):
    w = I.bubble(nx, N, bubbles=[])
    Q = O.ic(w["phys"], w["mesh"], "bubbles", [])
    dt = O.dt(w["phys"], w["mesh"], Q)
    Q2, _ = O.run(w["phys"], w["mesh"], Q, 0.0, 5, dt)
    # momentum relative to rho * (sound speed ~ 350 m/s)
    assert np.max(np.abs(Q2[:, 1:3])) <= tol * 350.0
    assert np.max(np.abs(Q2[:, 0] - Q[:, 0])) <= tol


def test_resting_atmosphere_drift_shrinks_with_h():
    drift = []
    for nx in (9, 27):
        w = I.bubble(nx, 2, bubbles=[])
        Q = O.ic(w["phys"], w["mesh"], "bubbles", [])
        dt = O.dt(w["phys"], w["mesh"], Q)
        Q2, _ = O.run(w["phys"], w["mesh"], Q, 0.0, 5, dt)
        drift.append(np.max(np.abs(Q2[:, 1:3])))
    assert drift[1] < drift[0] / 9.0


def test_mesh_faces_of_uniform_grids():
    k = O.mesh_kinds(periodic(4))
    assert np.all(k == 0)
    w = I.bubble(5, 2)
    k = O.mesh_kinds(w["mesh"])
    walls = (k == 1).sum()
    assert walls == 4 * 5


def test_dof_count_matches_paper():
    """The scalability run (729x729 cells, order 6) has 'roughly 104 million'
    DOF; cells * (N+1)^2 * 4 variables gives that count."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    s = g["scalability_run"]
    dof = s["cells_per_side"] ** 2 * (s["order"] + 1) ** 2 * 4
    assert abs(dof / 1e6 - s["approx_mdof"]) < 0.5


def test_bubble_courant_factor_is_stable():
    """The bubble workloads' Courant factor keeps the order-6 scheme stable:
    300 steps of the 27x27 bubble (twice the time in which the same run at
    factor 0.5 blows up) stay bounded with a small flow (|m| < 0.1 kg/m^2/s
    for a 0.5 K bubble) and the density within the initial range."""
    w = I.bubble(27, 6)
    Q0 = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    Q, t = O.run(w["phys"], w["mesh"], Q0, 0.0, 300)
    assert t > 0.3
    assert np.isfinite(Q).all()
    assert np.max(np.abs(Q[:, 1:3])) < 0.1
    assert Q[:, 0].min() > Q0[:, 0].min() - 1e-3 and Q[:, 0].max() < Q0[:, 0].max() + 1e-3
