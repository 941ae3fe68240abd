"""GPU parity of the three-dimensional step against the oracle's 3D scheme,
through the C ABI (``include/adg3.h``).

Metric (per variable v): max |gpu - oracle| / S_v, S_v = max |oracle_v| for
density and energy and at least the acoustic momentum scale
sqrt(max rho * max E) for the momenta; the bar is 1e-11 in FP64 for the
predictor outputs, one step and the time step, as in two dimensions.  At the
full 25^3 size of the 3D bubble the step is checked on sampled cells, each
against the oracle on the 3 x 3 x 3 block of cells around it (a cell's new
state depends only on its own and its six neighbours' predictors)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1905_05524_amd import adg
from paper_1905_05524_amd import inputs as I

import parity as P

pytestmark = pytest.mark.gpu

TOL = 1e-11
WALL, PER = I.BC_WALL, I.BC_PERIODIC


def scales(b):
    b = np.asarray(b).reshape(b.shape[0], 5, -1)
    mx = [np.max(np.abs(b[:, v])) for v in range(5)]
    ac = math.sqrt(mx[0] * mx[4])
    return np.array([mx[0], max(mx[1], ac), max(mx[2], ac), max(mx[3], ac), mx[4]])


def relerr(a, b, scale=None):
    a = np.asarray(a).reshape(a.shape[0], 5, -1)
    b = np.asarray(b).reshape(b.shape[0], 5, -1)
    sc = scales(b) if scale is None else scale
    return np.array([np.max(np.abs(a[:, v] - b[:, v])) / (sc[v] if sc[v] > 0 else 1.0) for v in range(5)])


def fd_err(got, ref):
    """Face data [C][6][2][5][n][n]: state part scaled like the state, flux
    part by the largest flux magnitude of each variable."""
    got, ref = np.asarray(got), np.asarray(ref)
    C = ref.shape[0]
    qs = np.moveaxis(ref[:, :, 0], 2, 1).reshape(C, 5, -1)
    e_state = relerr(np.moveaxis(got[:, :, 0], 2, 1), np.moveaxis(ref[:, :, 0], 2, 1), scales(qs))
    fs = np.array([max(np.max(np.abs(ref[:, :, 1, v])), 1e-300) for v in range(5)])
    e_flux = np.array([np.max(np.abs(got[:, :, 1, v] - ref[:, :, 1, v])) / fs[v] for v in range(5)])
    return np.maximum(e_state, e_flux)


def cfd(N, mu=0.02, cfl=0.5):
    return dict(I.CFD, N=N, picard_iters=0, mu=mu, mms=0, cfl=cfl)


def grid(nx, ny, nz, h, bc):
    return dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, h=h, bc=list(bc))


def atmo_case(N, nx, ny, nz, seed, mu=5.0):
    """Warm bubble in a walled box of 1000 m cells scaled to the grid, with
    momentum noise so that every flux term is active."""
    phys = dict(I.ATMO, N=N, picard_iters=0, mu=mu, mms=0, cfl=0.4)
    h = 1000.0 / max(nx, nz)
    m = grid(nx, ny, nz, h, [WALL] * 6)
    Q = O.ic3(phys, m, "bubbles", [I.cosine_bubble3(a=400.0, xc=0.5 * nx * h, yc=0.5 * ny * h, zc=0.35 * nz * h)])
    return phys, m, I.perturb3(Q, seed=seed, rel=1e-3, vel=0.5)


def cfd_case(N, nx, ny, nz, bc, seed, mu=0.02):
    m = grid(nx, ny, nz, 1.0 / nx, bc)
    return cfd(N, mu), m, I.random_state_cfd3(nx * ny * nz, N, seed)


CASES = [
    # (id, builder)
    ("cfd_per_N1", lambda: cfd_case(1, 5, 3, 2, [PER] * 6, 1)),
    ("cfd_per_N2", lambda: cfd_case(2, 5, 3, 2, [PER] * 6, 2)),
    ("cfd_per_N3", lambda: cfd_case(3, 5, 3, 2, [PER] * 6, 3)),
    ("cfd_wall_N3", lambda: cfd_case(3, 3, 3, 3, [WALL] * 6, 4)),
    ("cfd_mixed_N2", lambda: cfd_case(2, 3, 2, 4, [PER, PER, WALL, WALL, PER, PER], 5)),
    ("atmo_N1", lambda: atmo_case(1, 4, 3, 4, 6)),
    ("atmo_N3", lambda: atmo_case(3, 3, 2, 3, 7)),
    ("cfd_per_N4", lambda: cfd_case(4, 2, 2, 2, [PER] * 6, 8)),
    ("atmo_N5", lambda: atmo_case(5, 2, 1, 2, 9)),
]


@pytest.fixture(params=CASES, ids=[c[0] for c in CASES])
def case(request):
    return request.param[1]()


def test_predictor_matches_oracle(case):
    phys, m, Q = case
    dt = 0.5 * O.dt3(phys, m, Q)
    Qs_ref, FD_ref = O.predictor3(phys, m, Q, dt)
    g = adg.Mesh3(phys, m, fixed_dt=True)
    g.set_state(Q, t=0.0, dt=dt)
    g.predictor()
    torch.cuda.synchronize()
    e_qs = relerr(g.qstar().cpu().numpy(), Qs_ref)
    e_fd = fd_err(g.face_data().cpu().numpy(), FD_ref)
    assert np.all(e_qs <= TOL), e_qs
    assert np.all(e_fd <= TOL), e_fd


def test_step_and_time_step_match_oracle(case):
    phys, m, Q = case
    dt = 0.5 * O.dt3(phys, m, Q)
    ref = O.step3(phys, m, Q, 0.0, dt)
    g = adg.Mesh3(phys, m)
    g.set_state(Q, t=0.0, dt=dt)
    g.step()
    torch.cuda.synchronize()
    got = g.Q.cpu().numpy()
    P.assert_step(got, ref, Q, V=5)
    # clock: t advanced by dt, one step, dt replaced by the CFL step of the new state
    clock = g.clock.cpu().numpy()
    assert clock[0] == dt and clock[3] == 1.0
    assert abs(clock[1] - O.dt3(phys, m, ref)) <= 1e-12 * clock[1]


def test_compute_dt_matches_oracle(case):
    phys, m, Q = case
    g = adg.Mesh3(phys, m)
    g.set_state(Q)
    g.compute_dt()
    assert abs(g.dt - O.dt3(phys, m, Q)) <= 1e-13 * g.dt


@pytest.mark.parametrize("bc", [PER, WALL])
def test_single_cell_grid(bc):
    """One cell: with periodic faces every neighbour is the cell itself."""
    phys, m, Q = cfd_case(3, 1, 1, 1, [bc] * 6, 11)
    dt = 0.5 * O.dt3(phys, m, Q)
    ref = O.step3(phys, m, Q, 0.0, dt)
    g = adg.Mesh3(phys, m, fixed_dt=True)
    g.set_state(Q, t=0.0, dt=dt)
    g.step()
    P.assert_step(g.Q.cpu().numpy(), ref, Q, V=5)


def test_multi_step_run_matches_oracle():
    """Five steps with the time step chosen by the CFL rule on each side."""
    phys, m, Q = atmo_case(2, 3, 3, 3, 12)
    Qo, t = O.run3(phys, m, Q, 0.0, 5)
    g = adg.Mesh3(phys, m)
    g.set_state(Q, t=0.0)
    g.compute_dt()
    for _ in range(5):
        g.step()
    torch.cuda.synchronize()
    assert abs(g.t - t) <= 1e-12 * t
    P.assert_step(g.Q.cpu().numpy(), Qo, Q, V=5, tol=5 * TOL, tol_inc=5 * P.TOL_INC)


@pytest.mark.parametrize("N", [1, 3])
def test_bubble_initial_state_matches_oracle(N):
    w = I.bubble3d(n=5, N=N)
    g = adg.Mesh3(w["phys"], w["mesh"])
    g.init_state("bubbles", w["bubbles"])
    torch.cuda.synchronize()
    ref = O.ic3(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    assert np.all(relerr(g.Q.cpu().numpy(), ref) <= 1e-14)
    g.check_health()


def test_abc_initial_state_matches_oracle():
    w = I.abc3d(n=4)
    g = adg.Mesh3(w["phys"], w["mesh"])
    g.init_state("abc", t0=0.05)
    torch.cuda.synchronize()
    ref = O.ic3(w["phys"], w["mesh"], "abc", t0=0.05)
    assert np.all(relerr(g.Q.cpu().numpy(), ref) <= 1e-14)


def test_resting_atmosphere_stays_at_rest():
    """Hydrostatic background, no bubble, walls: the momenta stay at rounding
    level over 20 steps (the 3D oracle pin holds the same bound)."""
    w = I.bubble3d(n=6, N=3)
    g = adg.Mesh3(w["phys"], w["mesh"])
    g.init_state("bubbles", [])
    Q0 = g.Q.clone()
    g.compute_dt()
    for _ in range(20):
        g.step()
    g.check_health()
    assert torch.max(torch.abs(g.Q[:, 1:4])).item() <= 1e-12 * 350.0
    assert torch.max(torch.abs(g.Q[:, 0] - Q0[:, 0])).item() <= 1e-12


def sub_block(m, cell, size=3):
    """The block of cells around cell (i, j, k) (clamped to the grid) as an
    oracle mesh with wall faces, and the index of the cell in it."""
    lo, loc = [], []
    dims = (m["nx"], m["ny"], m["nz"])
    for p, d in zip(cell, dims):
        s = min(max(p - 1, 0), max(d - size, 0))
        lo.append(s)
        loc.append(p - s)
    sz = [min(size, d) for d in dims]
    h = m["h"]
    sm = dict(nx=sz[0], ny=sz[1], nz=sz[2], x0=m["x0"] + lo[0] * h, y0=m["y0"] + lo[1] * h,
              z0=m["z0"] + lo[2] * h, h=h, bc=[WALL] * 6)
    return sm, lo, loc


def test_full_size_bubble_step_on_sampled_cells():
    """The 3D bubble at its full size (25^3 cells of 40 m, N = 3), perturbed,
    one step with the oracle's time step in the launch configuration the
    benchmark times; sampled cells (corners, edges, faces, interior, random)
    against the oracle on the 3 x 3 x 3 block around each."""
    w = I.bubble3d()
    phys, m = w["phys"], w["mesh"]
    Q = I.perturb3(O.ic3(phys, m, "bubbles", w["bubbles"]), seed=25, rel=1e-4, vel=0.05)
    dt = O.dt3(phys, m, Q)
    g = adg.Mesh3(phys, m, fixed_dt=True)
    g.set_state(Q, t=0.0, dt=dt)
    g.step()
    torch.cuda.synchronize()
    got = g.Q.cpu().numpy()
    n, nx, ny, nz = phys["N"] + 1, m["nx"], m["ny"], m["nz"]
    rng = np.random.default_rng(3)
    cells = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny // 2, nz - 1), (nx // 2, 0, 0), (12, 12, 8)]
    cells += [tuple(int(v) for v in rng.integers(0, 25, 3)) for _ in range(3)]
    G = Q.reshape(nz, ny, nx, 5, n, n, n)
    for (i, j, k) in cells:
        sm, lo, loc = sub_block(m, (i, j, k))
        sub = G[lo[2]:lo[2] + sm["nz"], lo[1]:lo[1] + sm["ny"], lo[0]:lo[0] + sm["nx"]].reshape(-1, 5, n, n, n)
        out = O.step3(phys, sm, np.ascontiguousarray(sub), 0.0, dt)
        ref = out[(loc[2] * sm["ny"] + loc[1]) * sm["nx"] + loc[0]][None]
        c = (k * ny + j) * nx + i
        P.assert_step(got[c][None], ref, Q[c][None], V=5, state_scale=scales(Q), what=(i, j, k))


def test_large_grid_step_on_sampled_cells():
    """64^3 cells at N = 3 (262,144 cells, 671 MB of state): one step,
    sampled cells against the oracle on the 3 x 3 x 3 block around each."""
    phys = dict(I.ATMO, N=3, picard_iters=0, mu=0.005, mms=0, cfl=0.4)
    m = I.mesh3(64, 1000.0)
    Q = O.ic3(phys, m, "bubbles", [I.cosine_bubble3()])
    Q = I.perturb3(Q, seed=64, rel=1e-4, vel=0.05)
    dt = O.dt3(phys, m, Q)
    g = adg.Mesh3(phys, m, fixed_dt=True)
    g.set_state(Q, t=0.0, dt=dt)
    g.step()
    torch.cuda.synchronize()
    n = 4
    G = Q.reshape(64, 64, 64, 5, n, n, n)
    rng = np.random.default_rng(5)
    cells = [(0, 0, 0), (63, 63, 63), (63, 0, 31)] + [tuple(int(v) for v in rng.integers(0, 64, 3)) for _ in range(3)]
    for (i, j, k) in cells:
        sm, lo, loc = sub_block(m, (i, j, k))
        sub = G[lo[2]:lo[2] + sm["nz"], lo[1]:lo[1] + sm["ny"], lo[0]:lo[0] + sm["nx"]].reshape(-1, 5, n, n, n)
        out = O.step3(phys, sm, np.ascontiguousarray(sub), 0.0, dt)
        ref = out[(loc[2] * sm["ny"] + loc[1]) * sm["nx"] + loc[0]][None]
        c = (k * 64 + j) * 64 + i
        got = g.Q[c].cpu().numpy()[None]
        P.assert_step(got, ref, Q[c][None], V=5, state_scale=scales(Q), what=(i, j, k))
