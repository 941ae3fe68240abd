"""GPU tests of the launch shapes, the multi-scenario batch (eager and HIP
graph) and adaptive meshes with 1:3 non-conforming faces, all through the C
ABI.  Launch shapes and batching must not change results: they are compared
bitwise with the single-mesh default shape; batched scenarios (sampled from
the 64-scenario workload, and a batch holding a 1:3 adaptive scenario) and
adaptive meshes are compared with the oracle, state and increment."""
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


def relerr(a, b):
    a = np.asarray(a).reshape(a.shape[0], 4, -1)
    b = np.asarray(b).reshape(b.shape[0], 4, -1)
    mx = [np.max(np.abs(b[:, v])) for v in range(4)]
    ac = math.sqrt(mx[0] * mx[3])
    sc = [mx[0], max(mx[1], ac), max(mx[2], ac), mx[3]]
    return np.array([np.max(np.abs(a[:, v] - b[:, v])) / sc[v] for v in range(4)])


def _run(w, Q, dt, shape=None, steps=2):
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    if shape:
        m.set_launch(*shape)
    m.set_state(Q, t=0.0, dt=dt)
    for _ in range(steps):
        m.step()
    torch.cuda.synchronize()
    return m.Q.clone()


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_launch_shapes_are_bitwise_equal(N):
    """Every packing of the one-wavefront-per-cell predictor gives the same
    bits; the predictor with one wavefront per time level (shape (0, 1), the
    default on small meshes) sums the levels in another order and agrees to
    rounding, and with the oracle."""
    w = I.bubble(7, N)      # 49 cells: ragged for every packing
    Q = I.perturb(O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"]), seed=N)
    dt = 0.5 * O.dt(w["phys"], w["mesh"], Q)
    base = _run(w, Q, dt, (1, 1))
    n = N + 1
    for cpw in (1, 2, 4):
        if cpw * n * n > 64:
            continue
        for wpb in (1, 2, 4):
            got = _run(w, Q, dt, (cpw, wpb))
            assert torch.equal(got, base), (cpw, wpb)
    lv = _run(w, Q, dt, (0, 1))
    assert torch.equal(lv, _run(w, Q, dt))
    ref = O.step(w["phys"], w["mesh"], O.step(w["phys"], w["mesh"], Q, 0.0, dt), dt, dt)
    P.assert_step(lv.cpu().numpy(), ref, Q, what="level kernel")
    P.assert_step(base.cpu().numpy(), ref, Q, what="cell kernel")
    # the time levels shared by two or four wavefronts: with as many
    # wavefronts as levels or more, the one-per-level kernel bit for bit
    for W in (2, 4):
        got = _run(w, Q, dt, (0, W))
        if W >= n:
            assert torch.equal(got, lv), W
        P.assert_step(got.cpu().numpy(), ref, Q, what=f"levels over {W} wavefronts")


def test_invalid_launch_shape_rejected():
    w = I.bubble(3, 6)
    m = adg.Mesh(w["phys"], w["mesh"])
    with pytest.raises(adg.AdgError):
        m.set_launch(2, 1)    # 2 * 49 > 64
    with pytest.raises(adg.AdgError):
        m.set_launch(1, 3)
    with pytest.raises(adg.AdgError):
        m.set_launch(0, 3)


def test_autotune_keeps_state_and_results():
    w = I.bubble(9, 3)
    m = adg.Mesh(w["phys"], w["mesh"])
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    Q0, c0 = m.Q.clone(), m.clock.clone()
    cpw, wpb = m.autotune(reps=2)
    assert torch.equal(m.Q, Q0) and torch.equal(m.clock, c0)
    assert cpw in (0, 1, 2, 4) and wpb in (1, 2, 4)
    m.step()
    ref = adg.Mesh(w["phys"], w["mesh"])
    ref.set_launch(cpw, wpb)
    ref.set_state(Q0)
    ref.clock.copy_(c0)
    ref.step()
    assert torch.equal(m.Q, ref.Q)


def _small_batch():
    ws = I.batch_scenarios(6, seed=7)
    # shrink grids to keep the test fast but keep the order mix and raggedness
    for k, w in enumerate(ws):
        nx = [5, 9, 4, 7, 3, 6][k]
        w["mesh"]["nx"] = w["mesh"]["nz"] = nx
    return ws


def test_batch_matches_single_runs_bitwise():
    ws = _small_batch()
    b = adg.Batch(ws)
    for s, w in enumerate(ws):
        b.init_state(s, "bubbles", w["bubbles"])
    b.compute_dt()
    for _ in range(3):
        b.step()
    torch.cuda.synchronize()
    for s, w in enumerate(ws):
        m = adg.Mesh(w["phys"], w["mesh"])
        m.init_state("bubbles", w["bubbles"])
        m.compute_dt()
        for _ in range(3):
            m.step()
        torch.cuda.synchronize()
        assert torch.equal(b.state(s), m.Q), s
        assert torch.equal(b.clock[s], m.clock), s


def _oracle_steps(w, Q, t, dts):
    """The oracle's state after steps of the given lengths from (Q, t)."""
    for dt in dts:
        Q = O.step(w["phys"], w["mesh"], Q, t, dt)
        t += dt
    return Q


def _batch_vs_oracle(ws, sample, steps=2, graph=False):
    """Step a batch (eagerly or as graph replays), then compare the sampled
    scenarios with the oracle run on the same inputs and the same time-step
    sequence (each scenario's own CFL step, read from its clock)."""
    b = adg.Batch(ws)
    for s, w in enumerate(ws):
        if w["ic"] == "bubbles":
            b.init_state(s, "bubbles", w["bubbles"])
    b.compute_dt()
    torch.cuda.synchronize()
    start = {s: (b.state(s).cpu().numpy().copy(), float(b.clock[s][0])) for s in sample}
    dts = {s: [] for s in sample}
    stream = torch.cuda.Stream() if graph else None
    for _ in range(steps):
        for s in sample:
            dts[s].append(float(b.clock[s][1]))
        if graph:
            with torch.cuda.stream(stream):
                b.step_graph(stream)
            stream.synchronize()
        else:
            b.step()
        torch.cuda.synchronize()
    for s in sample:
        Q0, t0 = start[s]
        print(f"batch scenario {s} ({ws[s]['name']}) vs oracle", flush=True)
        ref = _oracle_steps(ws[s], Q0, t0, dts[s])
        P.assert_step(b.state(s).cpu().numpy(), ref, Q0, what=ws[s]["name"])
        assert float(b.clock[s][0]) == pytest.approx(t0 + sum(dts[s]), rel=1e-14)


def test_full_batch_sampled_scenarios_match_oracle():
    """The 64-scenario batch (134,577 cells, orders 3-6, grids 9..81) as
    graph replays: two steps; the smallest and largest scenario of each
    order against the oracle."""
    ws = I.batch_scenarios()
    by_order = {}
    for s, w in enumerate(ws):
        by_order.setdefault(w["phys"]["N"], []).append((w["mesh"]["nx"], s))
    sample = sorted({min(v)[1] for v in by_order.values()} | {max(v)[1] for v in by_order.values()})
    _batch_vs_oracle(ws, sample, steps=2, graph=True)


def test_batch_with_adaptive_scenario_matches_oracle():
    """A batch of three scenarios of two orders, one of them on a mesh with
    1:3 non-conforming faces (the wall-bounded two-bubble case): every
    scenario against the oracle after three eager steps."""
    ws = [I.bubble(5, 3), I.bubble(6, 4, bubbles=[I.cosine_bubble(), I.cold_bubble()]), I.bubble(4, 4)]
    ws[1]["mesh"] = dict(ws[1]["mesh"], max_level=1,
                         leaves=I.refined_leaves(6, 6, [(2, 1), (3, 1), (2, 2), (0, 5), (5, 0)]))
    _batch_vs_oracle(ws, [0, 1, 2], steps=3)


def test_batch_graph_replay_equals_eager():
    ws = _small_batch()
    eager, graph = adg.Batch(ws), adg.Batch(ws)
    for b in (eager, graph):
        for s, w in enumerate(ws):
            b.init_state(s, "bubbles", w["bubbles"])
        b.compute_dt()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    for k in range(4):
        eager.step()
        with torch.cuda.stream(stream):
            graph.step_graph(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        # eager work and synchronisation between replays
        assert torch.equal(eager.Q, graph.Q), k
        assert torch.equal(eager.clock, graph.clock), k


@pytest.mark.parametrize("mixed", [False, True])
def test_persistent_mode_equals_per_order_launches(mixed):
    """The persistent work-counter predictor (one resident grid per order,
    items from a device counter) gives the bits of the per-order launches
    with one wavefront per cell, over several graph replays (the counters
    reset themselves between launches), also with a scenario on a 1:3 mesh.
    (The small groups here default to one wavefront per time level, which
    sums in another order: the per-order side is set to per-cell launches.)"""
    ws = _small_batch()
    if mixed:
        ws[1]["mesh"] = dict(I.bubble(6, ws[1]["phys"]["N"])["mesh"], max_level=1,
                             leaves=I.refined_leaves(6, 6, [(2, 1), (3, 1), (0, 5)]))
    a, b = adg.Batch(ws), adg.Batch(ws)
    for bb in (a, b):
        for s, w in enumerate(ws):
            bb.init_state(s, "bubbles", w["bubbles"])
        bb.compute_dt()
    for g in range(a.n_groups):
        a.set_launch(g, 1, 1)
    b.set_mode(adg.ADG_BATCH_PERSISTENT)
    stream = torch.cuda.Stream()
    for k in range(4):
        with torch.cuda.stream(stream):
            a.step_graph(stream)
            b.step_graph(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(a.Q, b.Q), k
        assert torch.equal(a.clock, b.clock), k
    b.step()                      # eager launch after the replays
    a.step()
    torch.cuda.synchronize()
    assert torch.equal(a.Q, b.Q)


def test_persistent_mode_at_the_extreme_orders():
    """The persistent predictor at orders 1, 2 and 7 (four, four and one
    cells per wavefront; at order 7 one wavefront per SIMD) against the
    per-order launches with one wavefront per cell, and against the oracle
    on one scenario of each order."""
    ws = []
    for N, nx in ((1, 11), (2, 7), (7, 5), (1, 4)):
        w = I.bubble(nx, N)
        ws.append(w)
    a, b = adg.Batch(ws), adg.Batch(ws)
    for bb in (a, b):
        for s, w in enumerate(ws):
            bb.init_state(s, "bubbles", w["bubbles"])
        bb.compute_dt()
    for g in range(a.n_groups):
        a.set_launch(g, 1, 1)
    b.set_mode(adg.ADG_BATCH_PERSISTENT)
    Q0 = [b.state(s).cpu().numpy() for s in range(len(ws))]
    c0 = b.clock.cpu().numpy()
    for _ in range(2):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert torch.equal(a.Q, b.Q)
    assert torch.equal(a.clock, b.clock)
    for s in range(3):
        w = ws[s]
        dt0 = c0[s, 1]
        ref = O.step(w["phys"], w["mesh"], Q0[s], 0.0, dt0)
        dt1 = O.dt(w["phys"], w["mesh"], ref)
        ref = O.step(w["phys"], w["mesh"], ref, dt0, dt1)
        P.assert_step(b.state(s).cpu().numpy(), ref, Q0[s], what=f"persistent N={w['phys']['N']}")


def test_batch_autotune_then_step_unchanged():
    ws = _small_batch()
    a, b = adg.Batch(ws), adg.Batch(ws)
    for bb in (a, b):
        for s, w in enumerate(ws):
            bb.init_state(s, "bubbles", w["bubbles"])
        bb.compute_dt()
    cpw, wpb = b.autotune(reps=2)
    assert len(cpw) == b.n_groups
    for g in range(b.n_groups):
        a.set_launch(g, cpw[g], wpb[g])
    a.step()
    b.step()
    torch.cuda.synchronize()
    assert torch.equal(a.Q, b.Q) and torch.equal(a.clock, b.clock)


def test_batch_rejects_mixed_physics():
    ws = _small_batch()
    ws[1]["phys"] = dict(ws[1]["phys"], mu=2e-3)
    with pytest.raises(adg.AdgError):
        adg.Batch(ws)


# ------------------------------------------------------------ adaptive meshes
def amr_case(kind, N):
    if kind == "periodic":
        w = I.mms_small(N=N, nx=4, mu=0.02)
        w["phys"]["mms"] = 0
        mesh = dict(w["mesh"], max_level=1, leaves=I.refined_leaves(4, 4, [(1, 1), (2, 1), (3, 3), (0, 0)]))
        return w["phys"], mesh, I.random_state_cfd(len(mesh["leaves"]), N, seed=50 + N)
    w = I.bubble(6, N, bubbles=[I.cosine_bubble(), I.cold_bubble()])
    mesh = dict(w["mesh"], max_level=1, leaves=I.refined_leaves(6, 6, [(2, 1), (3, 1), (2, 2), (0, 5), (5, 0)]))
    Q = O.ic(w["phys"], mesh, "bubbles", w["bubbles"])
    return w["phys"], mesh, I.perturb(Q, seed=60 + N)


@pytest.mark.parametrize("kind", ["periodic", "walls"])
@pytest.mark.parametrize("N", [1, 3, 6])
def test_adaptive_step_matches_oracle(kind, N):
    phys, mesh, Q = amr_case(kind, N)
    dt = 0.5 * O.dt(phys, mesh, Q)
    m = adg.Mesh(phys, mesh, fixed_dt=True)
    m.set_state(Q, t=0.2, dt=dt)
    m.step()
    ref = O.step(phys, mesh, Q, 0.2, dt)
    P.assert_step(m.Q.cpu().numpy(), ref, Q)


def test_adaptive_periodic_conservation_on_gpu():
    phys, mesh, Q = amr_case("periodic", 4)
    b = O.basis(4)
    W = np.outer(b["w"], b["w"])
    h = np.array([1.0 / 4 / 3 ** l for (l, _, _) in mesh["leaves"]])
    Wc = W[None] * (h ** 2)[:, None, None]
    m = adg.Mesh(phys, mesh, fixed_dt=True)
    m.set_state(Q, t=0.0, dt=0.5 * O.dt(phys, mesh, Q))
    for _ in range(3):
        m.step()
    before = np.einsum("cvji,cji->v", Q, Wc)
    after = np.einsum("cvji,cji->v", m.Q.cpu().numpy(), Wc)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())


def test_adaptive_initial_state_matches_oracle():
    phys, mesh, _ = amr_case("walls", 6)
    w = I.bubble(6, 6, bubbles=[I.cosine_bubble(), I.cold_bubble()])
    m = adg.Mesh(phys, mesh)
    m.init_state("bubbles", w["bubbles"])
    ref = O.ic(phys, mesh, "bubbles", w["bubbles"])
    assert np.all(relerr(m.Q.cpu().numpy(), ref) <= 1e-14)
