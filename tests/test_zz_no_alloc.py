"""GPU test of the allocation-free step (adg_step_static): through the C ABI,
two calls in a row on one GPU (the second on a smaller mesh, reusing the
static workspace) give the same state and clock as adg_step with a
caller-supplied workspace; meshes whose workspace exceeds the static buffer
are rejected before anything runs."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1905_05524_amd import adg
from paper_1905_05524_amd import inputs as I
from oracle import oracle as O

pytestmark = pytest.mark.gpu

STATIC_BYTES = 32 << 20


def _relerr(a, b):
    a = a.reshape(a.shape[0], 4, -1)
    b = b.reshape(b.shape[0], 4, -1)
    mx = [np.max(np.abs(b[:, v])) for v in range(4)]
    ac = float(np.sqrt(mx[0] * mx[3]))
    sc = [mx[0], max(mx[1], ac), max(mx[2], ac), mx[3]]
    return max(np.max(np.abs(a[:, v] - b[:, v])) / sc[v] for v in range(4))


def _case(nx, N, seed):
    w = I.bubble(nx, N)
    Q = I.perturb(O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"]), seed=seed)
    m = adg.Mesh(w["phys"], w["mesh"])
    m.set_state(Q)
    m.compute_dt()
    return m


def _step_both(m):
    """(adg_step's state and clock, adg_step_static's state and clock) from
    the same start."""
    Q0 = m.Q.clone()
    clock0 = m.clock.clone()
    Qs, clocks = Q0.clone(), clock0.clone()
    print(f"adg_step_static: {m.C} cells, n = {m.n}", flush=True)
    rc = adg.lib().adg_step_static(m.h, ctypes.c_void_p(Qs.data_ptr()), ctypes.c_void_p(clocks.data_ptr()),
                                   adg._stream_ptr(None))
    assert rc == adg.ADG_OK, adg.lib().adg_last_error()
    m.step()
    torch.cuda.synchronize()
    return (m.Q.cpu().numpy(), m.clock.cpu().numpy()), (Qs.cpu().numpy(), clocks.cpu().numpy()), Q0.cpu().numpy()


def test_static_step_equals_step_on_two_calls_in_a_row():
    big = _case(27, 6, 1)          # one wavefront per cell
    small = _case(5, 3, 2)         # one wavefront per time level
    assert big.ws_bytes > small.ws_bytes and big.ws_bytes <= STATIC_BYTES
    for m in (big, small):
        (Qa, ca), (Qb, cb), Q0 = _step_both(m)
        assert _relerr(Qb, Qa) <= 1e-11
        # increment Q^{n+1} - Q^n, normwise
        inc = np.linalg.norm(Qb - Q0) / max(np.linalg.norm(Qa - Q0), 1e-300)
        assert np.linalg.norm((Qb - Q0) - (Qa - Q0)) <= 1e-9 * np.linalg.norm(Qa - Q0), inc
        # same kernels on the same inputs: identical results, clock included
        assert np.array_equal(Qa, Qb) and np.array_equal(ca, cb)
        assert cb[3] == 1.0 and cb[0] > 0.0


def test_static_step_rejects_meshes_beyond_the_buffer():
    w = I.bubble(150, 6)           # 22,500 cells: about 76 MB of workspace
    m = adg.Mesh(w["phys"], w["mesh"])
    assert m.ws_bytes > STATIC_BYTES
    Q = m.Q.clone()
    clock = m.clock.clone()
    rc = adg.lib().adg_step_static(m.h, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(clock.data_ptr()),
                                   adg._stream_ptr(None))
    assert rc == adg.ADG_EINVAL
    assert b"static scratch holds" in adg.lib().adg_last_error()
    rc = adg.lib().adg_step_static(m.h, None, ctypes.c_void_p(clock.data_ptr()), adg._stream_ptr(None))
    assert rc == adg.ADG_EINVAL
