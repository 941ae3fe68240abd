"""Pins of the oracle's 1:3 non-conforming faces (adaptive meshes with one
refinement level): face detection, exact preservation of constant states,
conservation on periodic adaptive grids, and agreement with the uniform grid
when every cell is refined."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I


def amr_periodic(nx, refine):
    return dict(nx=nx, nz=nx, max_level=1, x0=0.0, z0=0.0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4,
                leaves=I.refined_leaves(nx, nx, refine))


def cfd(N, mu=0.02):
    return dict(I.CFD, N=N, picard_iters=0, mu=mu, mms=0, cfl=0.5)


def weights(mesh, N):
    b = O.basis(N)
    W = np.outer(b["w"], b["w"])
    h = np.array([mesh["Lx"] / mesh["nx"] / 3 ** l for (l, _, _) in mesh["leaves"]])
    return W[None] * (h ** 2)[:, None, None]


def test_face_kinds():
    mesh = amr_periodic(3, [(1, 1)])
    k = O.mesh_kinds(mesh)
    # coarse cells next to the refined one see 3 fine neighbours (kind 3)
    assert (k == 3).sum() == 4
    # fine cells on the family boundary see a coarse neighbour (kind 2)
    assert (k == 2).sum() == 12
    assert (k == 1).sum() == 0


@pytest.mark.parametrize("N", [1, 3])
def test_constant_state_on_adaptive_grid(N):
    mesh = amr_periodic(3, [(1, 1), (0, 2)])
    C = len(mesh["leaves"])
    n = N + 1
    Q = np.zeros((C, 4, n, n))
    Q[:, 0], Q[:, 1], Q[:, 2], Q[:, 3] = 1.2, 0.3, -0.1, 2.6
    out = O.step(cfd(N), mesh, Q, 0.0, 1e-3)
    assert np.max(np.abs(out - Q)) <= 1e-13 * 2.6


@pytest.mark.parametrize("N", [2, 3])
def test_conservation_on_adaptive_grid(N):
    mesh = amr_periodic(4, [(1, 1), (2, 1), (3, 3)])
    C = len(mesh["leaves"])
    Q = I.random_state_cfd(C, N, seed=31 + N)
    W = weights(mesh, N)
    dt = 0.5 * O.dt(cfd(N), mesh, Q)
    before = np.einsum("cvji,cji->v", Q, W)
    out = O.step(cfd(N), mesh, Q, 0.0, dt)
    after = np.einsum("cvji,cji->v", out, W)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())
    assert np.max(np.abs(out - Q)) > 1e-8


def test_fully_refined_equals_uniform_fine_grid():
    """All coarse cells refined: every face is conforming at level 1, so the
    step equals the uniform grid of 3x the resolution (same cells, reordered)."""
    N = 2
    nx = 2
    mesh = amr_periodic(nx, [(i, j) for j in range(nx) for i in range(nx)])
    fine = dict(nx=3 * nx, nz=3 * nx, max_level=0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4)
    Qf = I.random_state_cfd(9 * nx * nx, N, seed=4)
    # map leaf order -> uniform order c = j*nx + i
    idx = [j * 3 * nx + i for (_, i, j) in mesh["leaves"]]
    dt = 0.5 * O.dt(cfd(N), fine, Qf)
    ref = O.step(cfd(N), fine, Qf, 0.0, dt)
    out = O.step(cfd(N), mesh, Qf[idx], 0.0, dt)
    assert np.max(np.abs(out - ref[idx])) <= 1e-13 * np.max(np.abs(ref))


def test_interior_fine_cell_updates_as_on_uniform_grid():
    """The centre child of a refined family sees only fine neighbours, and the
    predictor is element-local, so its update equals the uniform fine grid's
    (same operations in the same order)."""
    N, nx = 3, 3
    mesh = amr_periodic(nx, [(1, 1)])
    fine = dict(nx=3 * nx, nz=3 * nx, max_level=0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4)
    Qf = I.random_state_cfd(9 * nx * nx, N, seed=12)
    idx = [j * 3 * nx + i for (_, i, j) in mesh["leaves"]]
    Q = np.zeros((len(idx), 4, N + 1, N + 1))
    for c, (l, i, j) in enumerate(mesh["leaves"]):
        if l == 1:
            Q[c] = Qf[j * 3 * nx + i]
        else:   # coarse cells: any valid state
            Q[c] = I.random_state_cfd(1, N, seed=100 + c)[0]
    dt = 0.25 * O.dt(cfd(N), fine, Qf)
    out = O.step(cfd(N), mesh, Q, 0.0, dt)
    ref = O.step(cfd(N), fine, Qf, 0.0, dt)
    centre = mesh["leaves"].index((1, 4, 4))
    assert np.max(np.abs(out[centre] - ref[4 * 3 * nx + 4])) <= 1e-14 * np.max(np.abs(ref))


def test_smooth_field_across_levels_matches_uniform_closely():
    """A resolved smooth state on an adaptive grid evolves close to the same
    state on the uniform fine grid (consistency of the non-conforming
    coupling), for the refined family next to coarse cells."""
    N, nx = 3, 9
    mesh = amr_periodic(nx, [(4, 4)])
    phys = dict(I.mms_small(N=N)["phys"])
    Q = O.ic(phys, mesh, "mms")
    fine = dict(nx=3 * nx, nz=3 * nx, max_level=0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4)
    Qf = O.ic(phys, fine, "mms")
    dt = 0.5 * O.dt(phys, fine, Qf)
    out = O.step(phys, mesh, Q, 0.0, dt)
    ref = O.step(phys, fine, Qf, 0.0, dt)
    fam = [c for c, (l, _, _) in enumerate(mesh["leaves"]) if l == 1]
    idx = [j * 3 * nx + i for (l, i, j) in mesh["leaves"] if l == 1]
    d = np.max(np.abs((out[fam] - Q[fam]) - (ref[idx] - Qf[idx])))
    assert d <= 0.05 * np.max(np.abs(ref[idx] - Qf[idx]))
