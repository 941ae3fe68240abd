"""Pins of the oracle's 3D scheme (uniform grids of cubes, periodic or wall
boundaries): reduction to the pinned 2D scheme for states that do not depend
on y, invariance under a cyclic permutation of the axes, exactness of the
predictor for linear advection along each axis, preservation of constant
states, conservation on periodic grids, and a resting atmosphere."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I

WALL, PER = I.BC_WALL, I.BC_PERIODIC


def cfd(N, mu=0.02):
    return dict(I.CFD, N=N, picard_iters=0, mu=mu, mms=0, cfl=0.5)


def mesh3(nx, ny, nz, h, bc):
    return dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, h=h, bc=list(bc))


def lift_2d(Q2, nx, nz, ny):
    """3D state constant in y with zero y momentum from a 2D state [c][4][z][x]."""
    C2, _, n, _ = Q2.shape
    Q3 = np.zeros((nx * ny * nz, 5, n, n, n))
    for k in range(nz):
        for i in range(nx):
            q = Q2[k * nx + i]
            for j in range(ny):
                c = (k * ny + j) * nx + i
                for v3, v2 in ((0, 0), (1, 1), (3, 2), (4, 3)):
                    Q3[c, v3] = q[v2][:, None, :]
    return Q3


@pytest.mark.parametrize("N", [1, 3])
def test_y_independent_states_follow_the_2d_scheme(N):
    """A warm bubble in a walled x-z box, constant along a periodic y: one 3D
    step equals the pinned 2D step in every y-plane (gravity, walls with the
    background heat flux, viscosity and heat conduction all active)."""
    w = I.bubble(4, N, bubbles=[I.cosine_bubble(a=400.0)])
    phys = dict(w["phys"], mu=5.0)
    mesh2 = w["mesh"]
    Q2 = I.perturb(O.ic(phys, mesh2, "bubbles", w["bubbles"]), seed=N)
    h = mesh2["Lx"] / mesh2["nx"]
    m3 = mesh3(4, 2, 4, h, [WALL, WALL, PER, PER, WALL, WALL])
    Q3 = lift_2d(Q2, 4, 4, 2)
    dt = 0.5 * O.dt(phys, mesh2, Q2)
    out2 = O.step(phys, mesh2, Q2, 0.0, dt)
    out3 = O.step3(phys, m3, Q3, 0.0, dt)
    ref3 = lift_2d(out2, 4, 4, 2)
    scale = np.abs(ref3).reshape(len(ref3), 5, -1).max(axis=(0, 2))
    scale[1:4] = np.maximum(scale[1:4], np.sqrt(scale[0] * scale[4]))
    err = np.abs(out3 - ref3).reshape(len(ref3), 5, -1).max(axis=(0, 2)) / scale
    assert np.all(err <= 1e-13), err
    assert np.max(np.abs(out3[:, 2])) <= 1e-12 * scale[2]


def rotate(Q, nx, ny, nz):
    """Cyclic permutation of the axes x -> y -> z -> x: the new field at
    (x', y', z') = (z, x, y); momenta (mx, my, mz) -> (mz, mx, my) accordingly."""
    n = Q.shape[-1]
    G = Q.reshape(nz, ny, nx, 5, n, n, n)                  # [K][J][I][v][k][j][i]
    # new grid: X' = Z, Y' = X, Z' = Y  ->  new dims (nx', ny', nz') = (nz, nx, ny)
    R = G.transpose(1, 2, 0, 3, 5, 6, 4)                    # [J][I][K][v][j][i][k] = [K'][J'][I'][v][k'][j'][i']
    R = R[:, :, :, [0, 3, 1, 2, 4]]
    return np.ascontiguousarray(R.reshape(nx * ny * nz, 5, n, n, n))


@pytest.mark.parametrize("N", [1, 2])
@pytest.mark.parametrize("bc", [PER, WALL])
def test_cyclic_axis_permutation_commutes_with_the_step(N, bc):
    nx, ny, nz = 3, 2, 2
    C = nx * ny * nz
    n = N + 1
    rng = np.random.default_rng(7 + N)
    Q = np.zeros((C, 5, n, n, n))
    Q[:, 0] = 1.0 + 0.2 * rng.uniform(-1, 1, Q[:, 0].shape)
    Q[:, 1:4] = 0.3 * rng.uniform(-1, 1, Q[:, 1:4].shape)
    Q[:, 4] = 2.5 + 0.3 * rng.uniform(-1, 1, Q[:, 4].shape)
    phys = cfd(N, mu=0.05)
    m = mesh3(nx, ny, nz, 0.25, [bc] * 6)
    mr = mesh3(nz, nx, ny, 0.25, [bc] * 6)
    dt = 0.5 * O.dt3(phys, m, Q)
    a = rotate(O.step3(phys, m, Q, 0.0, dt), nx, ny, nz)
    b = O.step3(phys, mr, rotate(Q, nx, ny, nz), 0.0, dt)
    assert np.max(np.abs(a - b)) <= 1e-13 * 3.0


@pytest.mark.parametrize("N", [1, 3])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_predictor_exact_for_linear_advection_3d(N, axis):
    """mu = 0, constant velocity along one axis, constant pressure, density a
    polynomial of degree N along it: the time-averaged face values equal the
    exact time average of rho(x - a t) at the face."""
    n = N + 1
    b = O.basis(N)
    xi = b["xi"]
    nc, h, a, p = 2, 0.5, 0.7, 1.0
    coef = np.array([1.0, 0.1, 0.05, -0.02])[: N + 1]
    rho_f = lambda s: np.polynomial.polynomial.polyval(s, coef)
    C = nc ** 3
    Q = np.zeros((C, 5, n, n, n))
    for c in range(C):
        i, j, k = c % nc, (c // nc) % nc, c // (nc * nc)
        s = (i, j, k)[axis] * h + h * xi
        shape = [1, 1, 1]
        shape[2 - axis] = n                    # node axes are (z, y, x)
        r = np.broadcast_to(rho_f(s).reshape(shape), (n, n, n))
        Q[c, 0] = r
        Q[c, 1 + axis] = a * r
        Q[c, 4] = p / 0.4 + 0.5 * r * a * a
    dt = 0.02
    _, FD = O.predictor3(cfd(N, mu=0.0), mesh3(nc, nc, nc, h, [PER] * 6), Q, dt)
    exact = sum(b["w"][k] * rho_f(h - a * dt * xi[k]) for k in range(n))
    face = 2 * axis + 1
    assert np.max(np.abs(FD[0, face, 0, 0] - exact)) <= 2e-14
    assert np.max(np.abs(FD[0, face, 1, 0] - a * exact)) <= 2e-14


def test_constant_state_and_conservation():
    N = 2
    n = N + 1
    m = mesh3(3, 2, 2, 1.0 / 3, [PER] * 6)
    C = 12
    Q = np.zeros((C, 5, n, n, n))
    Q[:, 0], Q[:, 1], Q[:, 2], Q[:, 3], Q[:, 4] = 1.2, 0.3, -0.2, 0.1, 2.6
    out = O.step3(cfd(N), m, Q, 0.0, 1e-3)
    assert np.max(np.abs(out - Q)) <= 1e-13 * 2.6
    rng = np.random.default_rng(5)
    Q[:, 0] += 0.1 * rng.uniform(-1, 1, Q[:, 0].shape)
    Q[:, 1:4] += 0.1 * rng.uniform(-1, 1, Q[:, 1:4].shape)
    Q[:, 4] += 0.1 * rng.uniform(-1, 1, Q[:, 4].shape)
    b = O.basis(N)
    W = np.einsum("k,j,i->kji", b["w"], b["w"], b["w"])
    dt = 0.5 * O.dt3(cfd(N), m, Q)
    out = O.step3(cfd(N), m, Q, 0.0, dt)
    before = np.einsum("cvkji,kji->v", Q, W)
    after = np.einsum("cvkji,kji->v", out, W)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())
    assert np.max(np.abs(out - Q)) > 1e-8


def test_resting_atmosphere_3d():
    """A resting hydrostatic atmosphere in a box with walls on all six faces
    stays at rest to the bound of the 2D pin (N = 4, cells of 111 m)."""
    phys = dict(I.ATMO, N=4, picard_iters=0, mu=1e-3, mms=0, cfl=0.4)
    m = mesh3(9, 2, 9, 1000.0 / 9, [WALL] * 6)
    Q = O.ic3(phys, m, "bubbles", [])
    Q2, t = O.run3(phys, m, Q, 0.0, 5)
    assert t > 0
    assert np.max(np.abs(Q2[:, 1:4])) <= 1e-12 * 350.0
    assert np.max(np.abs(Q2[:, 0] - Q[:, 0])) <= 1e-12


def test_abc_flow_initial_state():
    """The ABC velocity field is divergence free and periodic on [-pi, pi]^3;
    its nodal interpolant has (to rounding) zero mean momentum."""
    phys = dict(I.CFD, N=3, picard_iters=0, mu=0.01, mms=0, cfl=0.5, gamma=1.4)
    L = 2 * np.pi
    m = dict(nx=3, ny=3, nz=3, x0=-np.pi, y0=-np.pi, z0=-np.pi, h=L / 3, bc=[PER] * 6)
    Q = O.ic3(phys, m, "abc")
    b = O.basis(3)
    W = np.einsum("k,j,i->kji", b["w"], b["w"], b["w"])
    mom = np.einsum("cvkji,kji->v", Q[:, 1:4], W) / 27
    assert np.all(np.abs(mom) <= 1e-3)
    assert np.allclose(Q[:, 0], 1.0)
