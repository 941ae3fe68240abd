"""Pins of the oracle's pointwise physics against an independent symbolic
transcription of the paper's equation set (sympy differentiates the fields;
the oracle uses the chain rule), the hydrostatic balance of the background and
the manufactured solution."""
import math

import numpy as np
import pytest
import sympy as sp

from oracle import oracle as O
from paper_1905_05524_amd import inputs as I


def sympy_flux(phys, q, gx, gz, x0, z0):
    """Paper eqs. equation-set, eos (geopotential read as rho*g*z),
    temperature, stress-tensor, heat-conduction-coeff (kappa = mu cp / Pr) and
    momentum-equation-split, for fields linear around (x0, z0)."""
    x, z = sp.symbols("x z", real=True)
    Qs = [sp.Float(q[v]) + sp.Float(gx[v]) * (x - x0) + sp.Float(gz[v]) * (z - z0) for v in range(4)]
    rho, jx, jz, E = Qs
    gam, R, cp, Pr, mu = (sp.Float(phys[k]) for k in ("gamma", "R", "cp", "Pr", "mu"))
    g = sp.Float(phys["g"]) if phys["gravity"] else sp.Integer(0)
    vx, vz = jx / rho, jz / rho
    p = (gam - 1) * (E - sp.Rational(1, 2) * (vx * jx + vz * jz) - rho * g * z)
    T = p / (rho * R)
    kappa = mu * cp / Pr
    X = (x, z)
    v = (vx, vz)
    div = sp.diff(vx, x) + sp.diff(vz, z)
    sig = [[mu * (sp.Rational(2, 3) * div * (1 if a == b else 0) - (sp.diff(v[b], X[a]) + sp.diff(v[a], X[b])))
            for b in range(2)] for a in range(2)]
    if phys["gravity"]:
        rb, pb = O.background(phys, z0)
        pprime = p - sp.Float(pb)
    else:
        rb, pb = 0.0, 0.0
        pprime = p
    F = []
    for a in range(2):
        Fa = [ (jx, jz)[a] ]
        for b in range(2):
            Fa.append(v[a] * (jx, jz)[b] + (pprime if a == b else 0) + sig[a][b])
        Fa.append(v[a] * (E + p) + sum(v[b] * sig[b][a] for b in range(2)) - kappa * sp.diff(T, X[a]))
        F.append(Fa)
    S = [0, 0, -g * (rho - sp.Float(rb)), 0]
    sub = {x: x0, z: z0}
    Fx = np.array([float(sp.N(f.subs(sub), 30)) for f in F[0]])
    Fz = np.array([float(sp.N(f.subs(sub), 30)) for f in F[1]])
    Sv = np.array([float(sp.N(sp.sympify(s).subs(sub), 30)) for s in S])
    return Fx, Fz, Sv


@pytest.mark.parametrize("case", ["cfd", "atmo"])
def test_pointwise_flux_against_sympy(case):
    rng = np.random.default_rng(7 if case == "cfd" else 8)
    if case == "cfd":
        phys = dict(I.CFD, N=2, mu=0.05, mms=0)
    else:
        phys = dict(I.ATMO, N=2, mu=0.7, mms=0)
    for _ in range(6):
        if case == "cfd":
            q = np.array([1.0, 0.3, -0.2, 2.5]) + 0.1 * rng.uniform(-1, 1, 4)
            gx, gz = rng.uniform(-1, 1, 4), rng.uniform(-1, 1, 4)
            x0, z0 = rng.uniform(0, 1, 2)
        else:
            z0 = rng.uniform(0, 1000)
            rb, pb = O.background(phys, z0)
            q = np.array([rb * 1.01, 2.0 * rb, -1.5 * rb, pb / 0.4 + rb * 9.81 * z0 + 5.0])
            gx = rng.uniform(-1, 1, 4) * np.array([1e-4, 1e-2, 1e-2, 10.0])
            gz = rng.uniform(-1, 1, 4) * np.array([1e-4, 1e-2, 1e-2, 10.0])
            x0 = rng.uniform(0, 1000)
        Fx, Fz, S = O.pointwise(phys, q, gx, gz, x0, z0)
        Fx2, Fz2, S2 = sympy_flux(phys, q, gx, gz, x0, z0)
        for a, b in ((Fx, Fx2), (Fz, Fz2), (S, S2)):
            scale = np.maximum(np.abs(b), 1e-300)
            # relative per component, absolute floor at the magnitude of the
            # largest term (cancellation in the momentum flux with p')
            assert np.all(np.abs(a - b) <= 1e-13 * np.maximum(scale, np.max(np.abs(b)) * 1e-3)), (a, b)


def test_background_hydrostatic_and_constant_theta():
    phys = dict(I.ATMO, N=2, mu=0.0, mms=0)
    for z in [0.0, 137.0, 500.0, 999.0]:
        h = 1e-2
        rp, pp = O.background(phys, z + h)
        rm, pm = O.background(phys, z - h)
        r0, p0 = O.background(phys, z)
        dpdz = (pp - pm) / (2 * h)
        # paper eq. hydrostatic-balance: d p_bar / dz = -g rho_bar
        assert abs(dpdz + phys["g"] * r0) <= 1e-8 * abs(phys["g"] * r0)
        # constant potential temperature: theta = T (p0/p)^(R/cp), T = p/(rho R)
        T = p0 / (r0 * phys["R"])
        theta = T * (phys["p0"] / p0) ** (phys["R"] / phys["cp"])
        assert abs(theta - phys["theta_bg"]) <= 1e-12 * phys["theta_bg"]


def test_mms_source_solves_pde():
    """The manufactured density wave with its source solves the equation set:
    dE/dt + div F_E = S_E with F from sympy, at random space-time points."""
    w = I.mms_small(N=2)
    phys = dict(w["phys"])
    phys.update(mms_u=0.5, mms_w=0.25, mms_kx=2 * math.pi, mms_kz=4 * math.pi)
    x, z, t = sp.symbols("x z t", real=True)
    A, u, ww, kx, kz, p = (sp.Float(phys[k]) for k in ("mms_amp", "mms_u", "mms_w", "mms_kx", "mms_kz", "mms_p"))
    rho = 1 + A * sp.sin(kx * (x - u * t)) * sp.sin(kz * (z - ww * t))
    gam, R, cp, Pr, mu = (sp.Float(phys[k]) for k in ("gamma", "R", "cp", "Pr", "mu"))
    E = p / (gam - 1) + rho * (u * u + ww * ww) / 2
    T = p / (rho * R)
    kappa = mu * cp / Pr
    FEx = u * (E + p) - kappa * sp.diff(T, x)
    FEz = ww * (E + p) - kappa * sp.diff(T, z)
    res = sp.diff(E, t) + sp.diff(FEx, x) + sp.diff(FEz, z)
    rng = np.random.default_rng(3)
    for _ in range(5):
        xv, zv, tv = rng.uniform(0, 1, 3)
        expect = float(res.subs({x: xv, z: zv, t: tv}))
        rhov = float(rho.subs({x: xv, z: zv, t: tv}))
        q = np.array([rhov, rhov * 0.5, rhov * 0.25, float(E.subs({x: xv, z: zv, t: tv}))])
        _, _, S = O.pointwise(phys, q, np.zeros(4), np.zeros(4), xv, zv, tv)
        assert abs(S[3] - expect) <= 1e-12 * max(1.0, abs(expect))
        assert S[0] == 0 and S[1] == 0 and S[2] == 0


def paper_mms_fields():
    """The paper's manufactured solution (CFD scenarios, eq.
    manufactured-solution) as sympy expressions: p, rho, v = v0 sin(k.x - 2 pi t)
    with v0 = (1/4, 1/4) and k = pi/5 (1, 1)."""
    x, z, t = sp.symbols("x z t", real=True)
    arg = sp.pi / 5 * x + sp.pi / 5 * z - 2 * sp.pi * t
    gam = sp.Rational(7, 5)
    p = sp.cos(arg) / 10 + 1 / gam
    rho = sp.sin(arg) / 2 + 1
    u = sp.sin(arg) / 4
    w = sp.sin(arg) / 4
    return (x, z, t), gam, p, rho, u, w


def test_paper_mms_source_solves_pde():
    """The paper's manufactured solution with the oracle's source solves the
    full equation set (no gravity): dQ/dt + div F(Q, grad Q) = S for all four
    conserved variables, F transcribed from the paper's equation set,
    stress tensor and heat flux and differentiated by sympy, at random
    space-time points.  CFD constants gamma = 1.4, Pr = 0.7, c_v = 1,
    mu = 0.1 (the paper's values for this test)."""
    (x, z, t), gam, p, rho, u, w = paper_mms_fields()
    R, cp, Pr, mu = sp.Rational(2, 5), sp.Rational(7, 5), sp.Rational(7, 10), sp.Rational(1, 10)
    E = p / (gam - 1) + rho * (u * u + w * w) / 2
    T = p / (rho * R)
    kappa = mu * cp / Pr
    X, v = (x, z), (u, w)
    div = sp.diff(u, x) + sp.diff(w, z)
    sig = [[mu * (sp.Rational(2, 3) * div * (1 if a == b else 0) - (sp.diff(v[b], X[a]) + sp.diff(v[a], X[b])))
            for b in range(2)] for a in range(2)]
    m = (rho * u, rho * w)
    F = []
    for a in range(2):
        Fa = [m[a]] + [v[a] * m[b] + (p if a == b else 0) + sig[a][b] for b in range(2)]
        Fa.append(v[a] * (E + p) + sum(v[b] * sig[b][a] for b in range(2)) - kappa * sp.diff(T, X[a]))
        F.append(Fa)
    Q = [rho, m[0], m[1], E]
    res = [sp.diff(Q[k], t) + sp.diff(F[0][k], x) + sp.diff(F[1][k], z) for k in range(4)]
    phys = dict(I.CFD, N=2, mu=0.1, mms=2)
    rng = np.random.default_rng(5)
    for _ in range(6):
        xv, zv = rng.uniform(0, 10, 2)
        tv = rng.uniform(0, 0.5)
        sub = {x: xv, z: zv, t: tv}
        expect = np.array([float(sp.N(r.subs(sub), 30)) for r in res])
        q = np.array([float(sp.N(e.subs(sub), 30)) for e in Q])
        _, _, S = O.pointwise(phys, q, np.zeros(4), np.zeros(4), xv, zv, tv)
        assert np.all(np.abs(S - expect) <= 1e-13 * max(1.0, np.max(np.abs(expect)))), (S, expect)
    # the state the oracle interpolates is the paper's field
    mesh = dict(nx=2, nz=2, max_level=0, x0=0.0, z0=0.0, Lx=10.0, Lz=10.0, bc=[I.BC_PERIODIC] * 4)
    Qo = O.ic(phys, mesh, "paper_mms", t0=0.3)
    xi = O.basis(2)["xi"]
    c, jz, ix = 3, 1, 2                       # cell (1, 1), node (z = 1, x = 2)
    sub = {x: 5.0 + 5.0 * xi[ix], z: 5.0 + 5.0 * xi[jz], t: 0.3}
    ref = np.array([float(sp.N(e.subs(sub), 30)) for e in Q])
    assert np.all(np.abs(Qo[c, :, jz, ix] - ref) <= 1e-14 * np.abs(ref).max())
