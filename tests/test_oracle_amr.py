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


# ------------------------------------------------------------------ regrid
def poly_state(mesh, N, deg):
    """Nodal values of a fixed polynomial field of total degree deg."""
    b = O.basis(N)
    out = []
    for (l, i, j) in mesh["leaves"]:
        h = mesh["Lx"] / mesh["nx"] / 3 ** l
        X = i * h + h * b["xi"][None, :]
        Z = j * h + h * b["xi"][:, None]
        f = lambda k: sum((0.3 + 0.1 * a + 0.05 * k) * X ** a * Z ** (min(deg, 3) - a if a <= min(deg, 3) else 0)
                          for a in range(deg + 1)) + 1.0
        out.append(np.stack([f(0), f(1), f(2), 2.0 + f(3)]))
    return np.array(out)


def test_regrid_refine_is_exact_on_polynomials():
    N = 3
    mesh = dict(nx=3, nz=3, max_level=1, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4, leaves=I.uniform_leaves(3, 3))
    Q = poly_state(mesh, N, 3)
    flags = np.zeros(9, dtype=np.int8)
    flags[[1, 4]] = 1
    leaves, Qn = O.regrid(cfd(N), mesh, Q, flags)
    assert len(leaves) == 9 - 2 + 18
    expect = poly_state(dict(mesh, leaves=leaves), N, 3)
    assert np.max(np.abs(Qn - expect)) <= 1e-13


def test_regrid_coarsen_is_l2_projection_and_conservative():
    N = 2
    leaves = I.refined_leaves(3, 3, [(1, 1), (0, 2)])
    mesh = dict(nx=3, nz=3, max_level=1, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4, leaves=leaves)
    Q = I.random_state_cfd(len(leaves), N, seed=8)
    flags = np.zeros(len(leaves), dtype=np.int8)
    fam = [c for c, (l, i, j) in enumerate(leaves) if l == 1 and i // 3 == 1 and j // 3 == 1]
    flags[fam] = -1
    new, Qn = O.regrid(cfd(N), mesh, Q, flags)
    assert len(new) == len(leaves) - 8
    W0, W1 = weights(mesh, N), weights(dict(mesh, leaves=new), N)
    assert np.allclose(np.einsum("cvji,cji->v", Q, W0), np.einsum("cvji,cji->v", Qn, W1), rtol=0, atol=1e-14)
    # a polynomial state is reproduced exactly by the projection
    P = poly_state(mesh, N, 2)
    _, Pn = O.regrid(cfd(N), mesh, P, flags)
    assert np.max(np.abs(Pn - poly_state(dict(mesh, leaves=new), N, 2))) <= 1e-13


def test_regrid_refine_then_coarsen_is_identity():
    N = 4
    mesh = dict(nx=2, nz=2, max_level=1, Lx=1.0, Lz=1.0, bc=[I.BC_WALL] * 4, leaves=I.uniform_leaves(2, 2))
    Q = I.random_state_cfd(4, N, seed=3)
    l1, Q1 = O.regrid(cfd(N), mesh, Q, np.array([1, 0, 1, 0], dtype=np.int8))
    f2 = np.array([-1 if l == 1 else 0 for (l, _, _) in l1], dtype=np.int8)
    l2, Q2 = O.regrid(cfd(N), dict(mesh, leaves=l1), Q1, f2)
    assert l2 == [(0, i, j) for j in range(2) for i in range(2)]
    assert np.max(np.abs(Q2 - Q)) <= 1e-13 * np.max(np.abs(Q))


def test_regrid_rules():
    N = 1
    leaves = I.refined_leaves(2, 2, [(0, 0)])
    mesh = dict(nx=2, nz=2, max_level=1, Lx=1.0, Lz=1.0, bc=[I.BC_WALL] * 4, leaves=leaves)
    Q = I.random_state_cfd(len(leaves), N, seed=1)
    # 8 of 9 siblings flagged: nothing merges; refine at max level dropped;
    # coarsen at level 0 dropped
    f = np.array([-1 if l == 0 else (1 if (i, j) == (0, 0) else -1) for (l, i, j) in leaves], dtype=np.int8)
    new, Qn = O.regrid(cfd(N), mesh, Q, f)
    assert new == leaves
    assert np.array_equal(Qn, Q)
    # all nine flagged: merged at the position of the first child
    f = np.array([0 if l == 0 else -1 for (l, i, j) in leaves], dtype=np.int8)
    new, _ = O.regrid(cfd(N), mesh, Q, f)
    assert new == [(0, 1, 0), (0, 0, 1), (0, 1, 1), (0, 0, 0)]


# ------------------------------------------------------------ two levels
def two_level(leaves, nx=3):
    return dict(nx=nx, nz=nx, max_level=2, x0=0.0, z0=0.0, Lx=1.0, Lz=1.0, bc=[I.BC_WALL] * 4,
                leaves=leaves)


def _children(l, i, j):
    return [(l + 1, 3 * i + a, 3 * j + b) for b in range(3) for a in range(3)]


def _state(leaves, N=1, seed=3):
    return I.random_state_cfd(len(leaves), N, seed=seed)


def test_refinement_ripples_to_keep_levels_balanced():
    """Refining the left-middle child of the refined centre cell would put a
    level-2 cell next to the level-0 cell on its left: that cell is refined
    too, and nothing else."""
    base = [(0, i, j) for j in range(3) for i in range(3) if (i, j) != (1, 1)] + _children(0, 1, 1)
    mesh = two_level(base)
    flags = np.zeros(len(base), dtype=np.int8)
    flags[base.index((1, 3, 4))] = 1
    leaves, _ = O.regrid(cfd(1), mesh, _state(base), flags)
    expect = []
    for lf in base:
        if lf in ((0, 0, 1), (1, 3, 4)):
            expect += _children(*lf)
        else:
            expect.append(lf)
    assert leaves == expect
    assert len(leaves) == 33
    O.mesh_kinds(dict(mesh, leaves=leaves))   # a valid (balanced) mesh


def _two_level_base():
    """3x3 coarse cells; the left-middle and the centre cell refined, the
    centre's left-middle child refined again."""
    leaves = []
    for j in range(3):
        for i in range(3):
            if (i, j) in ((0, 1), (1, 1)):
                continue
            leaves.append((0, i, j))
    leaves += _children(0, 0, 1)
    for ch in _children(0, 1, 1):
        leaves += _children(*ch) if ch == (1, 3, 4) else [ch]
    return leaves


def test_coarsening_that_breaks_balance_is_cancelled():
    base = _two_level_base()
    mesh = two_level(base)
    O.mesh_kinds(mesh)
    flags = np.zeros(len(base), dtype=np.int8)
    for ch in _children(0, 0, 1):       # the left family asks to coarsen
        flags[base.index(ch)] = -1
    leaves, Qn = O.regrid(cfd(1), mesh, _state(base), flags)
    assert leaves == base               # its parent would touch level 2: kept
    assert np.array_equal(Qn, _state(base))


def test_coarsenings_that_restore_balance_together_are_accepted():
    base = _two_level_base()
    mesh = two_level(base)
    flags = np.zeros(len(base), dtype=np.int8)
    for ch in _children(0, 0, 1) + _children(1, 3, 4):
        flags[base.index(ch)] = -1
    leaves, _ = O.regrid(cfd(1), mesh, _state(base), flags)
    expect = [(0, i, j) for j in range(3) for i in range(3) if (i, j) != (1, 1)]
    got = set(leaves)
    assert got == set(expect) | set(_children(0, 1, 1))
    assert len(leaves) == 8 + 9


def test_unbalanced_mesh_is_rejected():
    """The validity check used below: a level-2 cell next to a level-0 cell."""
    leaves = [(0, i, j) for j in range(3) for i in range(3) if (i, j) != (1, 1)]
    for ch in _children(0, 1, 1):
        leaves += _children(*ch) if ch == (1, 3, 4) else [ch]
    with pytest.raises(Exception):
        O.mesh_kinds(two_level(leaves))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_two_level_regrids_stay_balanced(seed):
    """Random flags on random two-level meshes: the result is a valid mesh
    (neighbours differ by at most one level), every leaf flagged refine below
    the top level is refined, and a family coarsens only when all nine
    siblings asked for it."""
    rng = np.random.default_rng(seed)
    leaves = [(0, i, j) for j in range(4) for i in range(4)]
    mesh = dict(nx=4, nz=4, max_level=2, x0=0.0, z0=0.0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC, I.BC_PERIODIC,
                I.BC_WALL, I.BC_WALL], leaves=leaves)
    for rnd in range(4):
        C = len(leaves)
        flags = rng.choice(np.array([-1, 0, 1], dtype=np.int8), size=C, p=[0.4, 0.3, 0.3])
        new, _ = O.regrid(cfd(1), mesh, _state(leaves, seed=rnd), flags)
        O.mesh_kinds(dict(mesh, leaves=new))
        newset = set(new)
        for lf, fl in zip(leaves, flags):
            if fl == 1 and lf[0] < 2:
                assert set(_children(*lf)) <= newset
            if lf not in newset and lf[0] > 0 and not set(_children(*lf)) <= newset:
                # coarsened: its whole family asked for it
                fam = [s for s in leaves if s[0] == lf[0] and (s[1] // 3, s[2] // 3) == (lf[1] // 3, lf[2] // 3)]
                assert len(fam) == 9
                assert all(flags[leaves.index(s)] == -1 for s in fam)
        leaves = new
        mesh = dict(mesh, leaves=leaves)


def _levels(leaves, L):
    c = [0] * (L + 1)
    for (l, _, _) in leaves:
        c[l] += 1
    return c


def test_paper_thresholds_track_the_colliding_bubbles():
    """The paper's AMR run (stratified-flow section: colliding bubbles, 9x9
    coarse cells, two levels, T_refine = 2.5, T_coarsen = -0.5) shows cells of
    all three sizes.  With the indicator read as the mean gradient norm over
    the cell, three initial passes reach level 2, and the mesh then stays
    unchanged over regrids every 10 steps (no refine/coarsen cycle: a refined
    family carries its parent's TV)."""
    w = I.amr9()
    phys, mesh = w["phys"], dict(w["mesh"])
    Q = O.ic(phys, mesh, "bubbles", w["bubbles"])
    for _ in range(w["initial_passes"]):
        _, fl, _ = O.tv(phys, mesh, Q, O.VAR_THETA, w["T_refine"], w["T_coarsen"])
        leaves, _ = O.regrid(phys, mesh, Q, fl)
        mesh["leaves"] = leaves
        Q = O.ic(phys, mesh, "bubbles", w["bubbles"])
    lv = _levels(mesh["leaves"], 2)
    assert lv == [71, 84, 54], lv
    t = 0.0
    for _ in range(2):
        Q, t = O.run(phys, mesh, Q, t, 10)
        _, fl, _ = O.tv(phys, mesh, Q, O.VAR_THETA, w["T_refine"], w["T_coarsen"])
        leaves, Q = O.regrid(phys, mesh, Q, fl)
        assert leaves == mesh["leaves"]
