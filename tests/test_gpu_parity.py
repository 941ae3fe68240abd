"""GPU parity: every kernel of the HIP path against the CPU oracle on the same
seeded inputs, through the C ABI.

Metric (per variable v): max |gpu - oracle| / S_v over all nodes, S_v = max
|oracle_v| for density and energy and at least the acoustic momentum scale
sqrt(max rho * max E) for the momenta; the bar is 1e-11 per step in FP64.  The
increment Q^{n+1} - Q^n is checked with the same normwise metric at 1e-9,
since the state is dominated by the hydrostatic background.  Flags must agree exactly except for cells whose TV
lies within a relative 1e-12 of a threshold."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1905_05524_amd import adg
from paper_1905_05524_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-11
TOL_INC = 1e-9


def _scales(b):
    """Per-variable error scale of a reference state [C][4][...]: max |rho| and
    max |E| for density and energy; for the momenta the larger of max |m| and
    the acoustic momentum scale sqrt(max rho * max E) (a flow at rest has no
    momentum scale of its own)."""
    b = np.asarray(b).reshape(b.shape[0], 4, -1)
    mx = [np.max(np.abs(b[:, v])) for v in range(4)]
    ac = math.sqrt(mx[0] * mx[3])
    return np.array([mx[0], max(mx[1], ac), max(mx[2], ac), mx[3]])


def relerr(a, b, scale=None):
    a = np.asarray(a).reshape(a.shape[0], 4, -1)
    b = np.asarray(b).reshape(b.shape[0], 4, -1)
    sc = _scales(b) if scale is None else scale
    return np.array([np.max(np.abs(a[:, v] - b[:, v])) / (sc[v] if sc[v] > 0 else 1.0) for v in range(4)])


def increment_err(got, ref, Q0, state_scale=None):
    """Normwise error of the increment Q^{n+1} - Q^n, each variable scaled by
    max |increment| floored at 1e-6 of the state scale (the hydrostatic
    cancellation p - p_bar limits the increment's own precision)."""
    dref = np.asarray(ref) - np.asarray(Q0)
    dgot = np.asarray(got) - np.asarray(Q0)
    inc = np.array([np.max(np.abs(dref.reshape(dref.shape[0], 4, -1)[:, v])) for v in range(4)])
    sc = np.maximum(inc, 1e-6 * (_scales(ref) if state_scale is None else state_scale))
    return relerr(dgot, dref, scale=sc)


# predictor kernels: one wavefront per cell; one workgroup per cell whose
# wavefronts own one time level each, or share them two or four ways
KERNELS = {"cell": (1, 1), "level": (0, 1), "level2": (0, 2), "level4": (0, 4)}


def mesh_of(w, kernel=None, **kw):
    m = adg.Mesh(w["phys"], w["mesh"], **kw)
    if kernel is not None:
        m.set_launch(*KERNELS[kernel])
    return m


def bubble_small(nx, N, mu=1e-3, walls=True):
    w = I.bubble(nx, N, mu=mu)
    if not walls:
        w["mesh"]["bc"] = [I.BC_PERIODIC] * 4
    return w


def cfd_periodic(nx, nz, N, mms=1, mu=0.02):
    w = I.mms_small(N=N, nx=nx, mu=mu)
    w["phys"]["mms"] = mms
    w["phys"].update(mms_u=0.5, mms_w=0.25, mms_kx=2 * math.pi, mms_kz=4 * math.pi)
    w["mesh"]["nz"] = nz
    w["mesh"]["Lz"] = nz / nx
    return w


def test_basis_matches_oracle():
    for N in range(1, 8):
        w = I.mms_small(N=N, nx=2)
        m = mesh_of(w)
        b, ob = m.basis(), O.basis(N)
        assert np.max(np.abs(b["xi"] - ob["xi"])) <= 4e-16
        assert np.max(np.abs(b["w"] - ob["w"])) <= 4e-16
        assert np.max(np.abs(b["D"] - ob["D"])) <= 1e-13 * max(1, np.max(np.abs(ob["D"])))
        assert np.max(np.abs(b["P"] - ob["P"])) <= 1e-14


@pytest.mark.parametrize("N", [2, 6])
def test_initial_state_matches_oracle(N):
    w = I.bubble(9, N, bubbles=[I.cosine_bubble(), I.cold_bubble()])
    m = mesh_of(w)
    m.init_state("bubbles", w["bubbles"])
    ref = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    assert np.all(relerr(m.Q.cpu().numpy(), ref) <= 1e-14)
    w = I.mms_small(N=N, nx=5)
    m = mesh_of(w)
    m.init_state("mms", t0=0.3)
    ref = O.ic(w["phys"], w["mesh"], "mms", t0=0.3)
    assert np.all(relerr(m.Q.cpu().numpy(), ref) <= 1e-14)


def _state(w, seed):
    if w["ic"] == "mms" or not w["phys"]["gravity"]:
        Q = I.random_state_cfd(w["mesh"]["nx"] * w["mesh"]["nz"], w["phys"]["N"], seed)
        return Q
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    return I.perturb(Q, seed)


CASES = [("bubble", 4, N) for N in range(1, 8)] + [("cfd", 3, N) for N in (1, 2, 4, 7)] + \
        [("cfd_ragged", 5, 3), ("cfd_1x1", 1, 2), ("bubble_1x1", 1, 3)]


def _case(kind, nx, N):
    if kind == "bubble":
        return bubble_small(nx, N)
    if kind == "bubble_1x1":
        return bubble_small(1, N)
    if kind == "cfd":
        return cfd_periodic(nx, nx, N)
    if kind == "cfd_ragged":
        return cfd_periodic(nx, 3, N)
    if kind == "cfd_1x1":
        return cfd_periodic(1, 1, N)
    raise ValueError(kind)


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("kind,nx,N", CASES)
def test_predictor_matches_oracle(kind, nx, N, kernel):
    w = _case(kind, nx, N)
    Q = _state(w, seed=1000 + 10 * N + nx)
    dt = 0.5 * O.dt(w["phys"], w["mesh"], Q)
    t = 0.37
    m = mesh_of(w, kernel, fixed_dt=True)
    m.set_state(Q, t=t, dt=dt)
    m.predictor()
    torch.cuda.synchronize()
    Qs, FD = O.predictor(w["phys"], w["mesh"], Q, t, dt)
    e = relerr(m.qstar().cpu().numpy(), Qs)
    assert np.all(e <= TOL), e
    ei = increment_err(m.qstar().cpu().numpy(), Qs, Q)
    assert np.all(ei <= TOL_INC), ei
    fd = m.face_data().cpu().numpy()
    for k in range(2):   # averaged state, averaged normal flux
        a = fd[:, :, k].transpose(0, 2, 1, 3)    # [C][var][face][node]
        b = FD[:, :, k].transpose(0, 2, 1, 3)
        assert np.all(relerr(a, b) <= TOL), (k, relerr(a, b))


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("kind,nx,N", CASES)
def test_step_matches_oracle(kind, nx, N, kernel):
    w = _case(kind, nx, N)
    Q = _state(w, seed=2000 + 10 * N + nx)
    dt = 0.5 * O.dt(w["phys"], w["mesh"], Q)
    m = mesh_of(w, kernel, fixed_dt=True)
    m.set_state(Q, t=0.1, dt=dt)
    m.step()
    ref = O.step(w["phys"], w["mesh"], Q, 0.1, dt)
    got = m.Q.cpu().numpy()
    assert np.all(relerr(got, ref) <= TOL), relerr(got, ref)
    assert np.all(increment_err(got, ref, Q) <= TOL_INC), increment_err(got, ref, Q)
    clk = m.clock.cpu().numpy()
    assert clk[0] == 0.1 + dt and clk[1] == dt and clk[3] == 1.0



@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("N", [1, 3, 6, 7])
def test_paper_mms_step_matches_oracle(N, kernel):
    """The paper's manufactured solution (its source on every variable, a
    separate instantiation of each predictor kernel) on a 3x3 grid,
    one step from the exact state at t = 0.2 against the oracle, on every
    predictor kernel."""
    w = I.paper_mms(N, 3)
    Q = O.ic(w["phys"], w["mesh"], "paper_mms", t0=0.2)
    dt = 0.5 * O.dt(w["phys"], w["mesh"], Q)
    m = mesh_of(w, kernel, fixed_dt=True)
    m.set_state(Q, t=0.2, dt=dt)
    m.step()
    ref = O.step(w["phys"], w["mesh"], Q, 0.2, dt)
    got = m.Q.cpu().numpy()
    assert np.all(relerr(got, ref) <= TOL), relerr(got, ref)
    assert np.all(increment_err(got, ref, Q) <= TOL_INC), increment_err(got, ref, Q)


@pytest.mark.parametrize("nx,nz", [(73, 6), (439, 1), (768, 1), (769, 1)])
def test_automatic_kernel_choice_at_its_threshold(nx, nz):
    """N = 6 with the default launch mode: 438 cells (438 x 7 = 3066
    wavefronts) take the predictor with one wavefront per time level, 439
    and 768 cells (768 x 4 = 3072) the time levels over four wavefronts, 769
    cells the one-wavefront-per-cell predictor; all match the oracle over
    one step."""
    w = cfd_periodic(nx, nz, 6)
    Q = _state(w, seed=3000 + nx)
    dt = 0.5 * O.dt(w["phys"], w["mesh"], Q)
    m = mesh_of(w, None, fixed_dt=True)
    m.set_state(Q, t=0.2, dt=dt)
    m.step()
    ref = O.step(w["phys"], w["mesh"], Q, 0.2, dt)
    got = m.Q.cpu().numpy()
    assert np.all(relerr(got, ref) <= TOL), relerr(got, ref)
    assert np.all(increment_err(got, ref, Q) <= TOL_INC), increment_err(got, ref, Q)

def test_cfl_dt_matches_oracle():
    for w in (I.bubble(9, 6), I.mms_small(N=2)):
        m = mesh_of(w)
        if w["ic"] == "mms":
            m.init_state("mms")
        else:
            m.init_state("bubbles", w["bubbles"])
        m.compute_dt()
        ref = O.dt(w["phys"], w["mesh"], m.Q.cpu().numpy())
        assert abs(m.dt - ref) <= 1e-14 * ref


@pytest.mark.parametrize("kernel", list(KERNELS))
def test_mms_ten_steps_per_step_parity(kernel):
    """The manufactured-solution workload (9x9 periodic, N=2): 10 steps with
    the CFL rule on the GPU; each step is compared with the oracle fed the
    GPU's previous state and time step."""
    w = I.mms_small()
    m = mesh_of(w, kernel)
    m.init_state("mms")
    m.compute_dt()
    for s in range(w["steps"]):
        Q0 = m.Q.cpu().numpy().copy()
        t, dt = m.t, m.dt
        m.step()
        ref = O.step(w["phys"], w["mesh"], Q0, t, dt)
        got = m.Q.cpu().numpy()
        assert np.all(relerr(got, ref) <= TOL), (s, relerr(got, ref))
        assert np.all(increment_err(got, ref, Q0) <= TOL_INC), (s, increment_err(got, ref, Q0))
        # the next CFL step agrees with the oracle's rule on the new state
        assert abs(m.dt - O.dt(w["phys"], w["mesh"], got)) <= 1e-13 * m.dt


@pytest.mark.parametrize("perturbed", [False, True])
def test_bubble81_full_size_step(perturbed):
    """81x81 cells, N=6 (the benchmark workload), launch configuration of the
    benchmark: one CFL step from the initial bubble (and from a seeded
    perturbation of it), compared on every node."""
    w = I.bubble81()
    m = mesh_of(w)
    m.init_state("bubbles", w["bubbles"])
    if perturbed:
        m.set_state(I.perturb(m.Q.cpu().numpy(), seed=81))
    m.compute_dt()
    Q0 = m.Q.cpu().numpy().copy()
    t, dt = m.t, m.dt
    m.step()
    ref = O.step(w["phys"], w["mesh"], Q0, t, dt)
    got = m.Q.cpu().numpy()
    assert np.all(relerr(got, ref) <= TOL), relerr(got, ref)
    assert np.all(increment_err(got, ref, Q0) <= TOL_INC), increment_err(got, ref, Q0)


def test_paper_grid_step_on_sampled_cells():
    """The grid of the paper's performance runs (colliding bubbles, 729x729
    cells, N=6, 104 M DOF), perturbed: one GPU step with the oracle's time
    step, sampled cells (corners, edges, interior, random) against the
    oracle stepping the 3 x 3 block around each (a cell's update depends
    only on its face neighbours; every boundary of this grid is a wall)."""
    w = I.paper_grid()
    phys, mesh = w["phys"], w["mesh"]
    nx, nz, n = mesh["nx"], mesh["nz"], phys["N"] + 1
    Q = I.perturb(O.ic(phys, mesh, "bubbles", w["bubbles"]), seed=729)
    dt = O.dt(phys, mesh, Q)
    m = mesh_of(w, fixed_dt=True)
    m.set_state(Q, t=0.0, dt=dt)
    m.step()
    torch.cuda.synchronize()
    h = mesh["Lx"] / nx
    rng = np.random.default_rng(7)
    cells = [(0, 0), (nx - 1, nz - 1), (0, nz - 1), (nx - 1, 0), (nx // 2, 0), (364, 364)]
    cells += [tuple(int(v) for v in rng.integers(0, 729, 2)) for _ in range(4)]
    for (i, j) in cells:
        i0, i1, j0, j1 = max(0, i - 1), min(nx, i + 2), max(0, j - 1), min(nz, j + 2)
        sub = dict(mesh, nx=i1 - i0, nz=j1 - j0, x0=mesh["x0"] + i0 * h, z0=mesh["z0"] + j0 * h,
                   Lx=(i1 - i0) * h, Lz=(j1 - j0) * h, bc=[I.BC_WALL] * 4, max_level=0)
        blk = np.ascontiguousarray(Q.reshape(nz, nx, 4, n, n)[j0:j1, i0:i1].reshape(-1, 4, n, n))
        ref = O.step(phys, sub, blk, 0.0, dt)[(j - j0) * (i1 - i0) + (i - i0)][None]
        got = m.Q[j * nx + i].cpu().numpy()[None]
        e = relerr(got, ref, _scales(Q))
        assert np.all(e <= TOL), ((i, j), e)
        ei = increment_err(got, ref, Q[j * nx + i][None], state_scale=_scales(Q))
        assert np.all(ei <= TOL_INC), ((i, j), ei)


def _tv_compare(w, Q, var, Tr, Tc):
    m = mesh_of(w)
    m.set_state(Q)
    C = m.C
    tv = torch.zeros(C, dtype=torch.float64, device="cuda")
    fl = torch.zeros(C, dtype=torch.int8, device="cuda")
    st = torch.zeros(3, dtype=torch.float64, device="cuda")
    m.tv_indicator(var, Tr, Tc, tv, fl, st)
    torch.cuda.synchronize()
    rtv, rfl, rst = O.tv(w["phys"], w["mesh"], Q, var, Tr, Tc)
    tv, fl, st = tv.cpu().numpy(), fl.cpu().numpy(), st.cpu().numpy()
    # rounding bound: relative 1e-13 of the largest TV, plus the noise floor of
    # a constant field, ||D||_inf / h * (few ulp of max |f|) per derivative
    N = w["phys"]["N"]
    Dinf = np.max(np.sum(np.abs(O.basis(N)["D"]), axis=1))
    h = w["mesh"]["Lx"] / w["mesh"]["nx"]
    fmax = 400.0 if var == adg.ADG_VAR_THETA else np.max(np.abs(Q[:, 0]))
    bound = 1e-13 * np.max(np.abs(rtv)) + 2 * 8 * Dinf / h * 2.3e-16 * fmax
    assert np.max(np.abs(tv - rtv)) <= bound, (np.max(np.abs(tv - rtv)), bound)
    assert st[0] == rst[0]
    dmu, dsig = abs(st[1] - rst[1]), abs(st[2] - rst[2])
    assert dmu <= 1e-13 * abs(rst[1]) + bound
    assert dsig <= 1e-12 * abs(rst[2]) + bound
    # a flag may differ only where TV lies within 1e-12 (relative) of a
    # threshold, or within the rounding bound of TV, mean and sigma
    thr = [rst[1] + T * rst[2] for T in (Tr, Tc)]
    band = [max(1e-12 * abs(t), bound + dmu + abs(T) * dsig) for t, T in zip(thr, (Tr, Tc))]
    near = np.any([np.abs(rtv - t) <= b for t, b in zip(thr, band)], axis=0)
    assert np.all((fl == rfl) | near)
    return fl


@pytest.mark.parametrize("N", [2, 6])
def test_tv_indicator_matches_oracle(N):
    w = I.bubble(27, N, bubbles=[I.cosine_bubble(), I.cold_bubble()])
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    fl = _tv_compare(w, Q, adg.ADG_VAR_THETA, 1.5, -0.5)
    assert (fl == 1).sum() > 0
    # the TV distribution is skewed (most cells see a constant theta), so
    # mu - 0.5 sigma < 0 coarsens nothing; a threshold at the mean does
    fl = _tv_compare(w, Q, adg.ADG_VAR_THETA, 1.0, 0.0)
    assert (fl == 1).sum() > 0 and (fl == -1).sum() > 0
    wr = cfd_periodic(6, 6, N)
    _tv_compare(wr, I.random_state_cfd(36, N, 9), adg.ADG_VAR_RHO, 0.5, -0.5)


def test_tv_indicator_many_cells_matches_oracle():
    """Above 65,536 cells the statistics run through per-workgroup partials
    (300 x 300 = 90,000 cells, N = 2), and the TV kernel packs four cells
    per wavefront: TV, statistics and flags against the oracle."""
    w = I.bubble(300, 2, bubbles=[I.cosine_bubble(), I.cold_bubble()])
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    fl = _tv_compare(w, Q, adg.ADG_VAR_THETA, 1.0, 0.0)
    assert (fl == 1).sum() > 0 and (fl == -1).sum() > 0


def test_tv_constant_field_keeps_all():
    w = cfd_periodic(4, 4, 3)
    n = 4
    Q = np.zeros((16, 4, n, n))
    Q[:, 0], Q[:, 3] = 1.0, 2.5
    fl = _tv_compare(w, Q, adg.ADG_VAR_RHO, 1.0, -1.0)
    assert np.all(fl == 0)


def test_health_detects_bad_states():
    w = I.bubble(9, 3)
    m = mesh_of(w)
    m.init_state("bubbles", w["bubbles"])
    m.check_health()
    Q = m.Q.clone()
    m.Q[5, 0, 1, 1] = float("nan")
    with pytest.raises(adg.AdgError) as e:
        m.check_health()
    assert e.value.code == adg.ADG_ESTATE
    m.Q.copy_(Q)
    m.Q[3, 0, 0, 0] = -1.0
    with pytest.raises(adg.AdgError):
        m.check_health()
    m.Q.copy_(Q)
    m.check_health()


def test_periodic_conservation_on_gpu():
    """Property at any size: a periodic grid conserves sum h^2 w_i w_j Q."""
    w = cfd_periodic(32, 32, 5, mms=0)
    Q = I.random_state_cfd(32 * 32, 5, 77)
    m = mesh_of(w, fixed_dt=True)
    m.set_state(Q, t=0.0, dt=0.5 * O.dt(w["phys"], w["mesh"], Q))
    for _ in range(3):
        m.step()
    b = O.basis(5)
    W = np.outer(b["w"], b["w"])
    before = np.einsum("cvji,ji->v", Q, W)
    after = np.einsum("cvji,ji->v", m.Q.cpu().numpy(), W)
    assert np.all(np.isfinite(after))
    assert np.all(np.abs(after - before) <= 1e-12 * np.abs(before).max())


def test_step_is_deterministic():
    w = I.bubble(27, 6)
    a, b = mesh_of(w), mesh_of(w)
    for m in (a, b):
        m.init_state("bubbles", w["bubbles"])
        m.compute_dt()
        for _ in range(3):
            m.step()
    assert torch.equal(a.Q, b.Q) and torch.equal(a.clock, b.clock)


def test_bubble81_long_run_stays_bounded():
    """1000 steps of the 81x81, N=6 bubble at the workloads' Courant factor
    (five times the step count at which factor 0.5 blows up): the state stays
    healthy and the flow small."""
    w = I.bubble81()
    m = adg.Mesh(w["phys"], w["mesh"])
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    rho0 = m.Q[:, 0].clone()
    for _ in range(1000):
        m.step()
    m.check_health()
    Q = m.Q
    assert float(Q[:, 1:3].abs().max()) < 0.1
    assert float(Q[:, 0].min()) > float(rho0.min()) - 1e-3
    assert float(Q[:, 0].max()) < float(rho0.max()) + 1e-3
    assert m.t > 0.5
