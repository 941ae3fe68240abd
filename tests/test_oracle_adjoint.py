"""Pins of the oracle's forward-mode derivatives (dual numbers), the
reference for the hand-written adjoint: central finite differences of the
plain double-precision oracle, and linearity."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I


def bubble_case(N, nx=3):
    w = I.bubble(nx, N, bubbles=[I.cosine_bubble(a=400.0)])
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    return w, I.perturb(Q, seed=N)


@pytest.mark.parametrize("N", [2, 3])
def test_step_jvp_matches_central_differences(N):
    w, Q = bubble_case(N)
    dt = 0.5 * O.dt(w["phys"], w["mesh"], Q)
    rng = np.random.default_rng(N)
    dQ = rng.standard_normal(Q.shape) * np.array([1e-4, 0.1, 0.1, 10.0])[None, :, None, None]
    out, jv = O.step_jvp(w["phys"], w["mesh"], Q, dQ, 0.0, dt)
    assert np.array_equal(out, O.step(w["phys"], w["mesh"], Q, 0.0, dt))
    eps = 1e-3
    fd = (O.step(w["phys"], w["mesh"], Q + eps * dQ, 0.0, dt) - O.step(w["phys"], w["mesh"], Q - eps * dQ, 0.0, dt)) / (2 * eps)
    for v in range(4):
        sc = np.max(np.abs(jv[:, v])) + 1e-300
        assert np.max(np.abs(fd[:, v] - jv[:, v])) <= 1e-6 * sc, v
    # linearity
    _, jv2 = O.step_jvp(w["phys"], w["mesh"], Q, 3.0 * dQ, 0.0, dt)
    assert np.max(np.abs(jv2 - 3.0 * jv)) <= 1e-12 * np.max(np.abs(jv))


def test_step_jvp_periodic_viscous():
    N = 3
    mesh = dict(nx=3, nz=3, max_level=0, Lx=1.0, Lz=1.0, bc=[I.BC_PERIODIC] * 4)
    phys = dict(I.CFD, N=N, mu=0.05, mms=0, cfl=0.5)
    Q = I.random_state_cfd(9, N, seed=2)
    dt = 0.5 * O.dt(phys, mesh, Q)
    dQ = np.random.default_rng(5).standard_normal(Q.shape)
    _, jv = O.step_jvp(phys, mesh, Q, dQ, 0.0, dt)
    eps = 1e-6
    fd = (O.step(phys, mesh, Q + eps * dQ, 0.0, dt) - O.step(phys, mesh, Q - eps * dQ, 0.0, dt)) / (2 * eps)
    assert np.max(np.abs(fd - jv)) <= 1e-6 * np.max(np.abs(jv))


def test_rollout_jvp_matches_central_differences():
    N, K = 2, 3
    w = I.bubble(3, N)
    n = N + 1
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    dt = O.dt(w["phys"], w["mesh"], Q)
    # theta' at the nodes: the bubble's perturbation, read back from the state
    rng = np.random.default_rng(0)
    th = 0.5 * rng.uniform(0, 1, (9, n, n))
    d = rng.standard_normal(th.shape)
    d /= np.linalg.norm(d)
    L, dL = O.rollout_jvp(w["phys"], w["mesh"], th, d, 0.0, dt, K)
    eps = 1e-5
    Lp, _ = O.rollout_jvp(w["phys"], w["mesh"], th + eps * d, None, 0.0, dt, K)
    Lm, _ = O.rollout_jvp(w["phys"], w["mesh"], th - eps * d, None, 0.0, dt, K)
    assert abs((Lp - Lm) / (2 * eps) - dL) <= 1e-6 * abs(dL)
    assert L > 0
