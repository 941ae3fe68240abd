"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds workload descriptions and random draws only: physical
constants, mesh sizes, bubble lists, scenario draws and random perturbations.
It contains none of the method's arithmetic (no equation of state, no flux, no
quadrature); each side (GPU library, oracle) builds its states from these
descriptions with its own code.

Workloads follow the paper's scenarios (Krenz, Rannabauer, Bader 2019):
  * ``mms_small``   periodic unit square 9x9, N=2, advected density wave with
                    its manufactured heat-flux source (CFD constants gamma=1.4,
                    Pr=0.7, c_v=1 of the convergence section)
  * ``paper_mms``   the paper's manufactured solution: periodic [0,10]^2,
                    mu = 0.1, to t = 0.5, orders 1..6
  * ``bubble81``    2D cosine warm bubble (stratified-flow section) on 81x81
                    cells of 12.35 m, N=6, no-slip walls, Courant factor 0.4
  * ``amr27``       the same box on 27x27 coarse cells with one 3-way
                    refinement level and a second, cold Gaussian bubble
  * ``amr9``        colliding bubbles on 9x9 coarse cells with two 3-way
                    refinement levels (the paper's AMR run)
  * ``bubble27``    81x81's box on 27x27 cells (adjoint workload)
  * ``batch64``     64 random bubble scenarios (grids 9..81, N in 3..6)
  * ``fv630``       the colliding bubbles with the finite-volume scheme: 7^2
                    patches of 90^2 cells = 630x630 cells of 1.59 m, inviscid
  * ``bubble3d``    3D cosine bubble in the 1000 m cube on 25^3 cells of 40 m,
                    N=3, mu = 0.005, no-slip walls
  * ``abc3d``       the ABC flow on the periodic cube [-pi, pi]^3, 27^3
                    cells, N=3, mu = 0.01
"""
from __future__ import annotations

import math

import numpy as np

BC_PERIODIC, BC_WALL = 0, 1
SHAPE_COSINE, SHAPE_PLATEAU_GAUSS = 0, 1

# physical constants --------------------------------------------------------
# CFD scenarios: gamma = 1.4, Pr = 0.7, c_v = 1 -> R = c_p - c_v = 0.4
CFD = dict(gamma=1.4, Pr=0.7, R=0.4, cp=1.4, p0=1.0, theta_bg=1.0, g=0.0, gravity=0)
# atmosphere: gamma, Pr and p0 of the stratified-flow section; g, R, c_p and
# the background potential temperature of the bubble workloads
ATMO = dict(gamma=1.4, Pr=0.71, R=287.0, cp=1005.0, p0=1.0e5, theta_bg=300.0, g=9.81, gravity=1)


def mms_small(N: int = 2, nx: int = 9, mu: float = 0.01):
    phys = dict(CFD, N=N, picard_iters=0, mu=mu, mms=1, mms_amp=0.1, mms_u=0.5, mms_w=0.5,
                mms_kx=2.0 * math.pi, mms_kz=2.0 * math.pi, mms_p=1.0, cfl=0.5)
    mesh = dict(nx=nx, nz=nx, max_level=0, x0=0.0, z0=0.0, Lx=1.0, Lz=1.0, bc=[BC_PERIODIC] * 4)
    return dict(name=f"mms{nx}x{nx}_N{N}", phys=phys, mesh=mesh, ic="mms", bubbles=[], steps=10)


def paper_mms(N: int, nx: int, mu: float = 0.1, t_end: float = 0.5):
    """The paper's manufactured-solution run (CFD scenarios): periodic
    [0,10]^2 on nx x nx cells, CFD constants, mu = 0.1, to t = 0.5; the
    fields and their source are fixed by the paper (kind 'paper_mms')."""
    phys = dict(CFD, N=N, picard_iters=0, mu=mu, mms=2, cfl=0.5)
    mesh = dict(nx=nx, nz=nx, max_level=0, x0=0.0, z0=0.0, Lx=10.0, Lz=10.0, bc=[BC_PERIODIC] * 4)
    return dict(name=f"paper_mms{nx}x{nx}_N{N}", phys=phys, mesh=mesh, ic="paper_mms", bubbles=[],
                t_end=t_end)


# Grids of the convergence study on the paper's manufactured solution, per
# order (three or four grids each, coarse enough for the CPU oracle)
PAPER_MMS_GRIDS = {1: (4, 8, 16, 32), 2: (4, 8, 16, 32), 3: (4, 8, 16, 32),
                   4: (2, 4, 8, 16), 5: (2, 4, 8, 16), 6: (2, 4, 8, 16)}


def cosine_bubble(A=0.5, a=250.0, xc=500.0, zc=350.0):
    return (SHAPE_COSINE, A, a, 0.0, xc, zc)


def cold_bubble(A=-0.15, a=0.0, s=50.0, xc=560.0, zc=640.0):
    return (SHAPE_PLATEAU_GAUSS, A, a, s, xc, zc)


# Courant factor of the bubble workloads.  With the time-step rule
# dt = cfl h / (2 (2N+1) (lambda + 2 lambda_v (2N+1) / h)), the order-6 scheme
# is unstable at cfl = 0.5 (the 81x81 bubble blows up after about 200 steps,
# 27x27 after about 150) and stable at 0.45 and below over thousands of
# steps; 0.4 keeps a margin.
BUBBLE_CFL = 0.4


def bubble(nx: int = 81, N: int = 6, mu: float = 1e-3, bubbles=None, steps: int = 100):
    phys = dict(ATMO, N=N, picard_iters=0, mu=mu, mms=0, cfl=BUBBLE_CFL)
    mesh = dict(nx=nx, nz=nx, max_level=0, x0=0.0, z0=0.0, Lx=1000.0, Lz=1000.0,
                bc=[BC_WALL] * 4)
    bl = [cosine_bubble()] if bubbles is None else list(bubbles)
    return dict(name=f"bubble{nx}x{nx}_N{N}", phys=phys, mesh=mesh, ic="bubbles", bubbles=bl,
                steps=steps)


def bubble81():
    return bubble(81, 6)


def bubble27():
    return bubble(27, 6, steps=50)


def amr27():
    """27x27 coarse cells of 37.04 m, one 3-way refinement level, warm cosine
    and cold Gaussian bubbles, N=6; regrid every 10 steps with the TV of theta.
    Thresholds: T_refine = 0, T_coarsen = -0.4 (T_refine refines 153 coarse
    cells of the initial state: 1953 leaves)."""
    w = bubble(27, 6, bubbles=[cosine_bubble(), cold_bubble()], steps=200)
    w["mesh"]["max_level"] = 1
    w["mesh"]["leaves"] = uniform_leaves(27, 27)
    w["name"] = "amr27x27_L1_N6"
    w["T_refine"], w["T_coarsen"], w["regrid_every"] = 0.0, -0.4, 10
    return w


def warm_plateau_bubble(A=0.5, a=150.0, s=50.0, xc=500.0, zc=300.0):
    return (SHAPE_PLATEAU_GAUSS, A, a, s, xc, zc)


def amr9():
    """Colliding bubbles (stratified-flow section): warm plateau bubble
    A = 0.5 K, a = 150 m, s = 50 m at (500, 300) m and cold bubble
    A = -0.15 K, s = 50 m at (560, 640) m; 9x9 coarse cells of 111.1 m with
    two 3-way refinement levels (37.04 m, 12.35 m), N=6, mu = 1e-3 (the
    paper's AMR run) with the paper's thresholds T_refine = 2.5,
    T_coarsen = -0.5.  The initial mesh is refined from the analytic state in
    three passes; regrid every 10 steps."""
    w = bubble(9, 6, bubbles=[warm_plateau_bubble(), cold_bubble()], steps=200)
    w["mesh"]["max_level"] = 2
    w["mesh"]["leaves"] = uniform_leaves(9, 9)
    w["name"] = "amr9x9_L2_N6"
    w["T_refine"], w["T_coarsen"], w["regrid_every"] = 2.5, -0.5, 10
    w["initial_passes"] = 3
    return w


def paper_grid():
    """The grid of the paper's performance runs: the colliding bubbles (the
    warm plateau and cold bubbles of ``amr9``) on a uniform 729 x 729 grid
    of 1.37 m cells, N = 6 (531,441 cells, 104,162,436 DOF), 20 steps."""
    w = bubble(729, 6, bubbles=[warm_plateau_bubble(), cold_bubble()], steps=20)
    w["name"] = "colliding729x729_N6"
    return w


def uniform_leaves(nx: int, nz: int, level: int = 0):
    """Leaf list (level, i, j) of a uniform grid in cell order c = j*nx + i."""
    return [(level, i, j) for j in range(nz) for i in range(nx)]


def batch_scenarios(count: int = 64, seed: int = 190505524):
    """Random bubble scenarios: k x k grid on the 1000 m box, k in 9..81,
    N in {3,4,5,6}, cosine bubble centre in [300,700]x[250,450] m, amplitude
    in [0.2,1.0] K; everything else as the 81x81 bubble."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        k = int(rng.integers(9, 82))
        N = int(rng.integers(3, 7))
        xc = float(rng.uniform(300.0, 700.0))
        zc = float(rng.uniform(250.0, 450.0))
        A = float(rng.uniform(0.2, 1.0))
        w = bubble(k, N, bubbles=[cosine_bubble(A=A, xc=xc, zc=zc)])
        w["name"] = f"scen{s}_{k}x{k}_N{N}"
        out.append(w)
    return out


def fd_directions(count: int, size: int, seed: int = 4):
    """Unit-norm Gaussian directions for finite-difference checks."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, size))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def random_state_cfd(C: int, N: int, seed: int):
    """Random conserved state in CFD units with a safely positive pressure:
    rho in [0.8,1.2], momenta in [-0.3,0.3], energy in [2.2,2.8]."""
    rng = np.random.default_rng(seed)
    n = N + 1
    Q = np.empty((C, 4, n, n))
    Q[:, 0] = 1.0 + 0.2 * rng.uniform(-1, 1, (C, n, n))
    Q[:, 1] = 0.3 * rng.uniform(-1, 1, (C, n, n))
    Q[:, 2] = 0.3 * rng.uniform(-1, 1, (C, n, n))
    Q[:, 3] = 2.5 + 0.3 * rng.uniform(-1, 1, (C, n, n))
    return Q


def perturb(Q: np.ndarray, seed: int, rel: float = 1e-3, vel: float = 0.5):
    """Seeded noise on a given state: relative noise `rel` on density and
    energy, momentum noise of `vel` times the local density."""
    rng = np.random.default_rng(seed)
    P = np.array(Q, dtype=np.float64, copy=True)
    P[:, 0] *= 1.0 + rel * rng.uniform(-1, 1, P[:, 0].shape)
    P[:, 3] *= 1.0 + rel * rng.uniform(-1, 1, P[:, 3].shape)
    P[:, 1] += vel * Q[:, 0] * rng.uniform(-1, 1, P[:, 1].shape)
    P[:, 2] += vel * Q[:, 0] * rng.uniform(-1, 1, P[:, 2].shape)
    return P


def refined_leaves(nx: int, nz: int, refine):
    """Leaf list (level, i, j) of an nx x nz coarse grid where the coarse
    cells in `refine` (iterable of (i, j)) are split into 3x3 children.
    Coarse cells come first in row-major order, then children family by
    family."""
    rs = set(tuple(r) for r in refine)
    out = [(0, i, j) for j in range(nz) for i in range(nx) if (i, j) not in rs]
    for (i, j) in sorted(rs, key=lambda t: (t[1], t[0])):
        out += [(1, 3 * i + a, 3 * j + b) for b in range(3) for a in range(3)]
    return out


# ------------------------------------------------------------ finite volume
# Courant factor of the finite-volume workloads (the N = 0 rule
# dt = cfl h / (2 lambda)).
FV_CFL = 0.9


def fv_bubbles(n: int = 630, steps: int = 50):
    """Colliding bubbles (warm plateau and cold Gaussian bubble of the AMR
    run) with the MUSCL-Hancock scheme: 7^2 patches of 90^2 cells on the
    1000 m box (n = 630: cells of 1.59 m), no viscosity, no-slip walls."""
    phys = dict(ATMO, N=0, picard_iters=0, mu=0.0, mms=0, cfl=FV_CFL)
    mesh = dict(nx=n, nz=n, max_level=0, x0=0.0, z0=0.0, Lx=1000.0, Lz=1000.0, bc=[BC_WALL] * 4)
    return dict(name=f"fv{n}x{n}", phys=phys, mesh=mesh, ic="bubbles",
                bubbles=[warm_plateau_bubble(), cold_bubble()], steps=steps)


# ------------------------------------------------------------------------ 3D
def cosine_bubble3(A=0.5, a=250.0, xc=500.0, yc=500.0, zc=350.0):
    """Bubble of the 3D cosine-bubble run: (shape, A, a, s, xc, yc, zc)."""
    return (SHAPE_COSINE, A, a, 0.0, xc, yc, zc)


def mesh3(n: int, L: float, x0: float = 0.0, bc: int = BC_WALL, ny: int = None):
    """n x ny x n cubes of edge L / n with lower corner (x0, x0, x0)."""
    return dict(nx=n, ny=n if ny is None else ny, nz=n, x0=x0, y0=x0, z0=x0, h=L / n, bc=[bc] * 6)


def bubble3d(n: int = 25, N: int = 3, mu: float = 0.005, steps: int = 50):
    """3D cosine bubble (stratified-flow section): the 1000 m cube with
    no-slip walls on n^3 cells (n = 25: 40 m cells), order N = 3, mu = 0.005,
    bubble A = 0.5 K, a = 250 m at (500, 500, 350) m."""
    phys = dict(ATMO, N=N, picard_iters=0, mu=mu, mms=0, cfl=BUBBLE_CFL)
    return dict(name=f"bubble3d_{n}^3_N{N}", phys=phys, mesh=mesh3(n, 1000.0), ic="bubbles",
                bubbles=[cosine_bubble3()], steps=steps)


def abc3d(n: int = 27, N: int = 3, mu: float = 0.01):
    """ABC flow (CFD section): periodic cube [-pi, pi]^3 on n^3 cells, order
    N = 3, mu = 0.01, CFD gas constants; the paper compares at t = 0.1."""
    phys = dict(CFD, N=N, picard_iters=0, mu=mu, mms=0, cfl=0.5)
    return dict(name=f"abc3d_{n}^3_N{N}", phys=phys, mesh=mesh3(n, 2.0 * math.pi, x0=-math.pi, bc=BC_PERIODIC),
                ic="abc", bubbles=[], t_end=0.1)


def random_state_cfd3(C: int, N: int, seed: int):
    """Random 3D conserved state in CFD units with a safely positive
    pressure: rho in [0.8,1.2], momenta in [-0.3,0.3], energy in [2.2,2.8]."""
    rng = np.random.default_rng(seed)
    n = N + 1
    Q = np.empty((C, 5, n, n, n))
    Q[:, 0] = 1.0 + 0.2 * rng.uniform(-1, 1, (C, n, n, n))
    Q[:, 1:4] = 0.3 * rng.uniform(-1, 1, (C, 3, n, n, n))
    Q[:, 4] = 2.5 + 0.3 * rng.uniform(-1, 1, (C, n, n, n))
    return Q


def perturb3(Q: np.ndarray, seed: int, rel: float = 1e-3, vel: float = 0.5):
    """Seeded noise on a 3D state: relative noise `rel` on density and
    energy, momentum noise of `vel` times the local density."""
    rng = np.random.default_rng(seed)
    P = np.array(Q, dtype=np.float64, copy=True)
    P[:, 0] *= 1.0 + rel * rng.uniform(-1, 1, P[:, 0].shape)
    P[:, 4] *= 1.0 + rel * rng.uniform(-1, 1, P[:, 4].shape)
    for v in (1, 2, 3):
        P[:, v] += vel * Q[:, 0] * rng.uniform(-1, 1, P[:, v].shape)
    return P
