"""Gradient of a final-time potential-temperature loss with respect to the
initial perturbation, as a ``torch.autograd.Function`` over the library's
hand-written adjoint.

Forward: theta' -> initial state (hydrostatic background perturbed in theta
at fixed pressure) -> K ADER-DG steps with a frozen time step, each step
writing its new state into the next checkpoint slot in device memory -> loss
L = ||theta - theta_bg||_{L2}.  Backward: the loss adjoint, then the step
adjoints from the last step to the first, then the adjoint of the
initial-state map.  With keep=True every forward step also keeps its Picard
iterates and face data in device memory (adg_step_to with a store, the step
of adg_step_keep) and the backward
pass uses them (adg_step_adjoint_kept); otherwise each step adjoint
recomputes its predictor from its checkpoint.  Both give the same gradient.
All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import adg


class ThetaRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta_prime, mesh: "adg.Mesh", steps: int, dt: float, t0: float = 0.0, keep: bool = False):
        m = mesh
        if not m.fixed_dt:
            # the adjoint differentiates steps of one frozen length
            raise ValueError("theta_rollout needs a mesh created with fixed_dt=True")
        th = theta_prime.detach().contiguous()
        m.ic_theta(th)
        # checkpoints Q^0 .. Q^K: the loss adjoint reads the rollout's own end
        # state, whatever the mesh is used for between forward and backward
        ck = torch.empty((steps + 1,) + tuple(m.Q.shape), dtype=torch.float64, device=m.device)
        m.clock[0], m.clock[1] = float(t0), float(dt)
        stores = fds = None
        if keep:
            sb, fb = m.keep_bytes()
            stores = torch.empty((steps, sb // 8), dtype=torch.float64, device=m.device)
            fds = torch.empty((steps, fb // 8), dtype=torch.float64, device=m.device)
        # each step reads checkpoint k (bound) and writes checkpoint k + 1
        ck[0].copy_(m.Q)
        try:
            for k in range(steps):
                m.bind_state(ck[k])
                if keep:
                    m.step_to(ck[k + 1], stores[k], fds[k])
                else:
                    m.step_to(ck[k + 1])
        finally:
            m.bind()
        m.Q.copy_(ck[steps])
        loss = torch.zeros(1, dtype=torch.float64, device=m.device)
        m.loss_theta(loss)
        ctx.mesh, ctx.steps, ctx.dt, ctx.t0 = m, steps, float(dt), float(t0)
        ctx.kept = (stores, fds) if keep else None
        ctx.save_for_backward(th, ck, loss)
        return loss[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        th, ck, loss = ctx.saved_tensors
        m = ctx.mesh
        K = ctx.steps
        g = grad_out.reshape(1).to(torch.float64).contiguous()
        lam = torch.empty_like(m.Q)
        lam2 = torch.empty_like(m.Q)
        # the loss adjoint at the rollout's end state Q^K
        m.Q.copy_(ck[K])
        m.loss_theta_adjoint(loss, g, lam)
        # each step's clock (start time, frozen dt), built on the device once:
        # rebinding a row per step is a host-side pointer change, so the loop
        # enqueues kernels only (no host writes that wait for the device)
        clocks = torch.zeros((max(K, 1), 4), dtype=torch.float64, device=m.device)
        clocks[:, 0] = ctx.t0 + ctx.dt * torch.arange(max(K, 1), dtype=torch.float64, device=m.device)
        clocks[:, 1] = ctx.dt
        try:
            for k in range(K - 1, -1, -1):
                m.bind_clock(clocks[k])
                if ctx.kept is not None:
                    m.step_adjoint_kept(ck[k], ctx.kept[0][k], ctx.kept[1][k], lam, lam2)
                else:
                    m.step_adjoint(ck[k], lam, lam2)
                lam, lam2 = lam2, lam
        finally:
            m.bind()
        grad = torch.empty_like(th)
        m.ic_theta_adjoint(th, lam, grad)
        ctx.kept = None
        return grad, None, None, None, None, None


def theta_rollout(theta_prime, mesh, steps, dt, t0=0.0, keep=False):
    """Loss after `steps` frozen-dt steps from theta' (differentiable).  The
    mesh must have been created with fixed_dt=True; its bound state ends at
    the rollout's final state (forward) and again after backward."""
    return ThetaRollout.apply(theta_prime, mesh, steps, dt, t0, keep)
