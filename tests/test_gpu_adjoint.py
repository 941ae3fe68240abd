"""GPU tests of the hand-written adjoint through the C ABI.

* Dot-product test per step: <J v, w> from the oracle's dual-number JVP
  against <v, J^T w> from the GPU adjoint (walls and periodic, N = 1..6).
* Rollout gradient of the potential-temperature loss with respect to the
  initial perturbation (torch.autograd.Function): against the oracle's
  directional derivatives and against central differences of the GPU forward
  rollout, on the 27x27, N=6, 50-step workload with 16 seeded unit
  directions: central differences at eps = 1e-3 within 1e-6 of g.d, the
  oracle's directional derivatives within 1e-8, on every direction.  The
  Rusanov speed is a maximum over face nodes of both sides, whose exact ties
  on a hydrostatic background make the loss only piecewise smooth (see the
  test).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1905_05524_amd import adg
from paper_1905_05524_amd import inputs as I
from paper_1905_05524_amd.autodiff import theta_rollout

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _case(kind, N):
    if kind == "walls":
        w = I.bubble(4, N, bubbles=[I.cosine_bubble(a=400.0)])
        Q = I.perturb(O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"]), seed=10 + N)
        return w["phys"], w["mesh"], Q
    phys = dict(I.CFD, N=N, picard_iters=0, mu=0.05, mms=0, cfl=0.5)
    mesh = dict(nx=3, nz=3, max_level=0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4)
    return phys, mesh, I.random_state_cfd(9, N, seed=20 + N)


@pytest.mark.parametrize("kernel", [(1, 1), (0, 1), (0, 2), (0, 4)], ids=["cell", "level", "level2", "level4"])
@pytest.mark.parametrize("kind", ["walls", "periodic"])
@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_step_adjoint_dot_product(kind, N, kernel):
    """<J v, w> = <v, J^T w> against the oracle's forward-mode derivative;
    the forward predictor with the iterate store runs on every kernel (one
    wavefront per cell; one per time level, the small meshes' default; the
    levels shared by two or four wavefronts)."""
    phys, mesh, Q = _case(kind, N)
    dt = 0.5 * O.dt(phys, mesh, Q)
    rng = np.random.default_rng(100 + N)
    scale = np.array([1e-4, 0.1, 0.1, 10.0])[None, :, None, None]
    v = rng.standard_normal(Q.shape) * scale
    w = rng.standard_normal(Q.shape) / scale
    _, Jv = O.step_jvp(phys, mesh, Q, v, 0.3, dt)
    m = adg.Mesh(phys, mesh, fixed_dt=True)
    m.set_launch(*kernel)
    m.set_state(Q, t=0.3, dt=dt)
    lam_out = torch.empty_like(m.Q)
    m.step_adjoint(dev(Q), dev(w), lam_out)
    JTw = lam_out.cpu().numpy()
    a, b = float(np.sum(Jv * w)), float(np.sum(v * JTw))
    bound = np.linalg.norm(Jv) * np.linalg.norm(w)
    assert abs(a - b) <= 1e-12 * bound, (a, b, bound)
    # the adjoint leaves the bound state untouched
    assert np.array_equal(m.Q.cpu().numpy(), Q)


def _theta_nodes(w, mesh):
    """theta' of the workload's bubbles at the nodes (the oracle's initial
    state read back as T/Exner - theta_bg is avoided: evaluate the bubble
    formula through the oracle's state and invert the density relation)."""
    Q = O.ic(w["phys"], mesh, "bubbles", w["bubbles"])
    phys = w["phys"]
    b = O.basis(phys["N"])
    n = phys["N"] + 1
    C = Q.shape[0]
    h = mesh["Lx"] / mesh["nx"]
    th = np.zeros((C, n, n))
    for c in range(C):
        j = c // mesh["nx"]
        for jj in range(n):
            z = j * h + h * b["xi"][jj]
            rb, pb = O.background(phys, z)
            # rho = p_bar / (R (theta_bg + theta') pi), rho_bar = p_bar / (R theta_bg pi)
            th[c, jj, :] = phys["theta_bg"] * (rb / Q[c, 0, jj, :]) - phys["theta_bg"]
    return th


def test_rollout_gradient_matches_oracle_small():
    w = I.bubble(6, 3, bubbles=[I.cosine_bubble(a=300.0)])
    K = 5
    th0 = _theta_nodes(w, w["mesh"])
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    dt = m.dt
    th = dev(th0).requires_grad_(True)
    L = theta_rollout(th, m, K, dt)
    L.backward()
    g = th.grad.cpu().numpy()
    Lref, _ = O.rollout_jvp(w["phys"], w["mesh"], th0, None, 0.0, dt, K)
    assert abs(float(L.detach()) - Lref) <= 1e-11 * Lref
    D = I.fd_directions(3, th0.size, seed=4).reshape((3,) + th0.shape)
    for d in D:
        _, dL = O.rollout_jvp(w["phys"], w["mesh"], th0, d, 0.0, dt, K)
        assert abs(np.sum(g * d) - dL) <= 1e-10 * max(abs(dL), 1e-3 * np.linalg.norm(g)), (np.sum(g * d), dL)


def test_rollout_gradient_bubble27_fd_and_oracle():
    """27x27 cells, N=6, 50 steps, checkpoint every step: 16 seeded unit
    directions; the adjoint gradient against the oracle's directional
    derivatives (dual numbers) on every direction, and against central
    differences of the GPU forward rollout within 1e-6 per direction.

    The step is eps = 1e-3 (unit directions), the minimum of the measured
    error curve: the relative error against the adjoint, max (median) over
    the 16 directions, is 1.8e-7 (1.4e-7) at 1e-2, 9.4e-8 (1.4e-8) at 1e-3,
    1.5e-6 (2.5e-7) at 1e-4, 4.5e-5 (3.4e-6) at 1e-5, 1.2e-4 (3.3e-5) at
    1e-6 and 5.7e-3 (1.8e-4) at 1e-7.  Below 1e-4 the rollout's own rounding
    dominates: L = 92 carries a relative rounding of about 1e-12 after 50
    steps, about 1e-10 absolute, which divided by 2 eps exceeds 1e-6 |g.d|
    (|g.d| is 3.5e-3 to 5e-2 here) for every eps below about 1e-3.

    Outside the bubble the state is exactly hydrostatic, so the sound speed
    ties exactly across the nodes of every horizontal face and the Rusanov
    maximum sits on a kink, where central differences average the tied
    branches while the adjoint (like the oracle) takes the first one.  The
    check therefore adds a seeded 1e-3 K nodal perturbation to theta' that
    separates the tied speeds by far more than the finite-difference step."""
    w = I.bubble27()
    K = w["steps"]
    th0 = _theta_nodes(w, w["mesh"])
    th0 = th0 + 1e-3 * np.random.default_rng(27).uniform(-1.0, 1.0, th0.shape)
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    dt = m.dt
    th = dev(th0).requires_grad_(True)
    L = theta_rollout(th, m, K, dt)
    L.backward()
    g = th.grad.cpu().numpy()
    D = I.fd_directions(16, th0.size, seed=4).reshape((16,) + th0.shape)
    eps = 1e-3
    for k, d in enumerate(D):
        gd = float(np.sum(g * d))
        _, dL = O.rollout_jvp(w["phys"], w["mesh"], th0, d, 0.0, dt, K)
        # 50 steps of rounding-order differences stay below 1e-8
        assert abs(gd - dL) <= 1e-8 * abs(dL), (k, gd, dL)
        with torch.no_grad():
            Lp = float(theta_rollout(dev(th0 + eps * d), m, K, dt))
            Lm = float(theta_rollout(dev(th0 - eps * d), m, K, dt))
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - gd) <= 1e-6 * abs(gd), (k, fd, gd)


def test_kept_iterates_give_the_recomputed_gradient():
    """Keeping every step's Picard iterates and face data (adg_step_keep /
    adg_step_adjoint_kept) gives bit for bit the gradient of the path that
    recomputes them from the checkpoints, and the same loss."""
    w = I.bubble(9, 4)
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    dt = m.dt
    C, n = m.C, 5
    rng = np.random.default_rng(8)
    th0 = dev(0.1 + 0.05 * rng.standard_normal((C, n, n)))
    res = {}
    for keep in (False, True):
        th = th0.clone().requires_grad_(True)
        L = theta_rollout(th, m, 6, dt, keep=keep)
        L.backward()
        res[keep] = (float(L.detach()), th.grad.detach().clone())
    assert res[True][0] == res[False][0]
    assert torch.equal(res[True][1], res[False][1])


def test_rollout_needs_a_frozen_time_step():
    w = I.bubble(5, 2)
    m = adg.Mesh(w["phys"], w["mesh"])          # CFL time step after every step
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    th = dev(np.zeros((m.C, 3, 3))).requires_grad_(True)
    with pytest.raises(ValueError):
        theta_rollout(th, m, 2, m.dt)


def test_gradient_unchanged_by_another_rollout_before_backward():
    """Two losses on one mesh: the second forward rollout (and plain steps)
    between the first forward and its backward must not change the first
    gradient, with and without kept iterates."""
    w = I.bubble(7, 3)
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    dt = m.dt
    C, n = m.C, 4
    rng = np.random.default_rng(17)
    th_a = dev(0.2 + 0.05 * rng.standard_normal((C, n, n)))
    th_b = dev(-0.1 + 0.05 * rng.standard_normal((C, n, n)))
    for keep in (False, True):
        ref_th = th_a.clone().requires_grad_(True)
        La = theta_rollout(ref_th, m, 5, dt, keep=keep)
        La.backward()
        ref = ref_th.grad.detach().clone()
        # forward A, then forward B and a few plain steps, then backward A
        ta = th_a.clone().requires_grad_(True)
        La2 = theta_rollout(ta, m, 5, dt, keep=keep)
        tb = th_b.clone().requires_grad_(True)
        Lb = theta_rollout(tb, m, 3, dt, keep=keep)
        for _ in range(2):
            m.step()
        La2.backward()
        assert float(La2.detach()) == float(La.detach())
        assert torch.equal(ta.grad, ref), keep
        Lb.backward()
        assert torch.isfinite(tb.grad).all()


def test_step_to_equals_the_in_place_step():
    """adg_step_to writes the step's result into another buffer and leaves
    the bound state as it was: the same bits as adg_step (without a store)
    and as adg_step_keep (with one, also the same kept iterates and face
    data); only one of store and fd is rejected."""
    w = I.bubble27()
    ref = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    ref.init_state("bubbles", w["bubbles"])
    ref.compute_dt()
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.set_state(ref.Q.clone(), t=0.0, dt=ref.dt)
    ref.set_state(ref.Q.clone(), t=0.0, dt=ref.dt)
    Q0 = m.Q.clone()
    out = torch.empty_like(m.Q)
    m.step_to(out)
    ref.step()
    torch.cuda.synchronize()
    assert torch.equal(out, ref.Q)
    assert torch.equal(m.Q, Q0)
    assert torch.equal(m.clock, ref.clock)
    sb, fb = m.keep_bytes()
    st1 = torch.empty(sb // 8, dtype=torch.float64, device="cuda")
    fd1 = torch.empty(fb // 8, dtype=torch.float64, device="cuda")
    st2, fd2 = torch.empty_like(st1), torch.empty_like(fd1)
    m.bind_state(out)
    out2 = torch.empty_like(out)
    m.step_to(out2, st1, fd1)
    ref.step_keep(st2, fd2)
    torch.cuda.synchronize()
    m.bind()
    assert torch.equal(out2, ref.Q)
    assert torch.equal(st1, st2) and torch.equal(fd1, fd2)
    with pytest.raises(adg.AdgError):
        m.step_to(out2, st1, None)

