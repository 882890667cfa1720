"""Gradients of displacement objectives with respect to material parameters.

``TimeHistory`` integrates N generalized-alpha steps on the GPU and keeps each
converged state (y_n, y-dot_n) on the device; ``VmsAdjoint`` wraps it in a
``torch.autograd.Function`` whose backward pass runs ``vms_adjoint_step``
once per step, newest first: the tangent is re-assembled at the checkpointed
converged state, the transposed reduced system is solved through the same
nested block preconditioner, and lam^T dG/dtheta is accumulated.

theta = (mu, kappa, k1, k2, fibre angle) as a float64 tensor of 5 entries.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from synth import fibre_field

from . import vms as V

STEP_KEYS = ("u", "p", "v", "du", "dp", "dv")


class TimeHistory:
    def __init__(self, prob, ti, n_steps, nopts=None, sopts=None, adj_opts=None, pmask=0b00011):
        self.prob = prob
        self.ti = ti
        self.n_steps = n_steps
        self.nopts = nopts or V.newton_opts(tol_R=1e-12, l_max=20)
        self.sopts = sopts or V.solver_opts(rtol=1e-12, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13)
        self.adj_opts = adj_opts or self.sopts
        self.pmask = pmask
        self.K = prob.new_matrix(mirror32=self.sopts.precision == V.MIXED)
        self.Kt = prob.new_matrix(mirror32=self.adj_opts.precision == V.MIXED)
        self.checkpoints = []

    def set_theta(self, theta):
        th = [float(x) for x in theta]
        mesh, mat = self.prob.mesh, self.prob.mat
        self.prob.set_material(dataclasses.replace(mat, mu=th[0], kappa=th[1] if th[1] > 0 else mat.kappa,
                                                   k1=th[2], k2=th[3]))
        if mesh.fibre is not None:
            fib, dfib = fibre_field(mesh, th[4])
            self.prob.set_fibres(fib, dfib)

    def timeint(self, s):
        ti = self.ti
        return V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt)

    def run(self, theta):
        """Forward integration from rest; returns u_N (device, [n][3])."""
        self.set_theta(theta)
        prob = self.prob
        st = prob.new_state()
        mesh = prob.mesh
        vm = torch.from_numpy(mesh.dir_mask[:, 0:3].astype(bool)).to(prob.dev)
        dv = torch.from_numpy(mesh.dir_vel).to(prob.dev)
        for key in ("v_n", "du_n", "v", "du"):
            st[key][vm] = dv[vm]
        self.checkpoints = [{k: st[k + "_n"].clone() for k in STEP_KEYS}]
        self.stats = []
        for s in range(self.n_steps):
            stats, _ = prob.step(st, self.timeint(s), self.nopts, self.sopts, self.K)
            self.stats.append(stats)
            self.checkpoints.append({k: st[k].clone() for k in STEP_KEYS})
            prob.roll(st)
        return self.checkpoints[-1]["u"]

    def gradient(self, dJdu):
        """dJ/dtheta (numpy, 5) given dJ/du_N (device [n][3])."""
        prob = self.prob
        n = prob.mesh.n_nodes
        ybar = torch.zeros(n, 7, dtype=torch.float64, device=prob.dev)
        ybar[:, 0:3] = dJdu.to(torch.float64)
        ydbar = torch.zeros_like(ybar)
        dJ = np.zeros(5)
        self.adj_stats = []
        for s in range(self.n_steps - 1, -1, -1):
            st = prob.new_state()
            for k in STEP_KEYS:
                st[k + "_n"].copy_(self.checkpoints[s][k])
                st[k].copy_(self.checkpoints[s + 1][k])
            ybar, ydbar, stats = prob.adjoint_step(st, self.timeint(s), self.K, self.Kt, ybar, ydbar, self.pmask,
                                                   dJ, self.adj_opts)
            self.adj_stats.append(stats)
        return dJ


class VmsAdjoint(torch.autograd.Function):
    """u_N = VmsAdjoint.apply(theta, history); backward gives dJ/dtheta.

    The forward pass keeps its own theta and checkpoint list on the autograd
    context, so a later ``history.run`` (another forward, a finite-difference
    evaluation) does not change what this graph's backward differentiates:
    backward restores both before it runs the adjoint steps.  The gradient is
    returned on theta's device and in its dtype."""

    @staticmethod
    def forward(ctx, theta, history):
        th = theta.detach().cpu().numpy().astype(np.float64).copy()
        u = history.run(th)
        ctx.history = history
        ctx.theta = th
        ctx.checkpoints = history.checkpoints
        ctx.theta_dtype = theta.dtype
        ctx.theta_device = theta.device
        return u.clone()

    @staticmethod
    def backward(ctx, grad_u):
        h = ctx.history
        h.set_theta(ctx.theta)
        h.checkpoints = ctx.checkpoints
        g = h.gradient(grad_u.contiguous())
        return torch.as_tensor(g, dtype=ctx.theta_dtype, device=ctx.theta_device), None
