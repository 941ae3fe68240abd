"""Error metrics shared by the GPU parity tests (not a test module).

State error, per variable v: max |gpu - oracle| / S_v over all nodes, with
S_v = max |oracle_v| for density and energy and at least the acoustic
momentum scale sqrt(max rho * max E) for the momenta (a flow at rest has no
momentum scale of its own).  The bar is 1e-11 per step in FP64.

Increment error: the same metric on Q^{n+1} - Q^n, each variable scaled by
its own largest increment (floored at 1e-6 of the state scale: the
hydrostatic cancellation p - p_bar limits the increment's own precision),
at 1e-9.  The state of the bubble workloads is dominated by the background,
and momenta start at rest, so this is the check that sees the dynamics.

V = 4 (2D: rho, rho u, rho w, E) or 5 (3D: rho, rho u, rho v, rho w, E);
states are [C][V][...] arrays."""
import math

import numpy as np

TOL = 1e-11
TOL_INC = 1e-9


def scales(b, V=4):
    b = np.asarray(b).reshape(b.shape[0], V, -1)
    mx = [np.max(np.abs(b[:, v])) for v in range(V)]
    ac = math.sqrt(mx[0] * mx[V - 1])
    return np.array([mx[0]] + [max(mx[v], ac) for v in range(1, V - 1)] + [mx[V - 1]])


def relerr(a, b, V=4, scale=None):
    a = np.asarray(a).reshape(a.shape[0], V, -1)
    b = np.asarray(b).reshape(b.shape[0], V, -1)
    sc = scales(b, V) if scale is None else scale
    return np.array([np.max(np.abs(a[:, v] - b[:, v])) / (sc[v] if sc[v] > 0 else 1.0) for v in range(V)])


def increment_err(got, ref, Q0, V=4, state_scale=None):
    dref = np.asarray(ref) - np.asarray(Q0)
    dgot = np.asarray(got) - np.asarray(Q0)
    r = dref.reshape(dref.shape[0], V, -1)
    inc = np.array([np.max(np.abs(r[:, v])) for v in range(V)])
    ss = scales(ref, V) if state_scale is None else state_scale
    return relerr(dgot, dref, V, scale=np.maximum(inc, 1e-6 * ss))


def assert_step(got, ref, Q0, V=4, tol=TOL, tol_inc=TOL_INC, what="", state_scale=None):
    """State and increment of a step (or a few steps) against the oracle."""
    e = relerr(got, ref, V, scale=state_scale)
    assert np.all(e <= tol), (what, "state", e)
    ei = increment_err(got, ref, Q0, V, state_scale)
    assert np.all(ei <= tol_inc), (what, "increment", ei)
    return e, ei
