"""Rollouts and their gradients on the GPU, with step checkpointing.

The time recursion of the adjoint (Sec. 5.1; framework, Sec. 4): per step t,
with (qbar, vbar) = (q_t, v_t) and g_q, g_v the loss gradients w.r.t.
(q_{t+1}, v_{t+1}),
    Acal_t^T z_t = g_q + g_v / h,
    g_q <- dL/dqbar,  g_v <- dL/dvbar          (propagated)
    dL/df_ext,t = h^2 z_t                      (final for the step)
    dL/dE, dL/dnu, dL/dmu accumulate over steps.
Every step (forward and adjoint) runs in the HIP library; this module holds
only the loop over time and the bookkeeping of checkpoints.

Checkpointing: the forward pass keeps (q, v) every `checkpoint` steps; the
backward pass recomputes each segment's converged states (and contact
records) from its checkpoint, then runs that segment's adjoint steps in
reverse.  The multiplier warm start is reset at every checkpoint boundary in
both passes, so a recomputed segment is bitwise identical to the original.
"""

from __future__ import annotations

import numpy as np
import torch

from . import native


class GpuSim:
    """A scene on the GPU plus the buffers of one step."""

    def __init__(self, spec, max_contacts=None, E=None, nu=None):
        self.spec = spec
        n = spec.n_verts
        self.max_contacts = int(max_contacts if max_contacts is not None else n * max(1, spec.planes.shape[0]))
        self.E = float(spec.E if E is None else E)
        self.nu = float(spec.nu if nu is None else nu)
        self.scene = native.Scene(spec.mesh.rest, spec.mesh.tets, spec.density, spec.h, spec.eps, self.E,
                                  self.nu, spec.gravity, spec.planes, spec.contact_margin, self.max_contacts,
                                  material=native.MATERIAL_CODES[getattr(spec, "material", "nh")])
        self.buf = native.ContactBuffers(self.max_contacts)
        self.dev = "cuda"
        # options of the adjoint solves in backward_pass (relative residual 1e-10 by default)
        self.opts = native.solve_opts(rtol=1e-10, maxit=4000, restart=64)

    def params(self, mu, requires_grad=True):
        """The (E, nu, mu) tensor of Rollout.apply for this scene."""
        return torch.tensor([self.E, self.nu, float(mu)], dtype=torch.float64, device=self.dev,
                            requires_grad=requires_grad)

    def step(self, qbar, vbar, f_ext, mu, t=None):
        """One forward step; with t given, the spec's kinematic spheres move
        from their pose at t to their pose at t + 1 during the step."""
        if t is not None and self.spec.spheres:
            native.set_spheres(self.scene, self.spec.sphere_array(t), self.spec.sphere_array(t + 1))
        q = torch.empty_like(qbar)
        v = torch.empty_like(qbar)
        native.sim_forward_step(self.scene, qbar, vbar, f_ext, mu, q, v, self.buf.state)
        return q, v, self.buf.clone()

    def reset_warm_start(self):
        native.forward_reset(self.scene)

    def adjoint(self, q, record, gq, gv, grad3, opts):
        """One adjoint step; returns (dL/dqbar, dL/dvbar, dL/df_ext, info)."""
        z = torch.zeros_like(q)
        native.adjoint_setup(self.scene, record.state, q, opts)
        info = native.adjoint_solve(self.scene, gq, gv, z, opts)
        dq, dv, df = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
        native.vjp_params(self.scene, z, gv, dq, dv, df, grad3)
        return dq, dv, df, info


def forward_pass(sim: GpuSim, q0, v0, forces, mu, checkpoint=None, keep_records=False):
    """T forward steps.  Returns (q_T, v_T, checkpoints, records).
    checkpoints: {t: (q_t, v_t)} at multiples of `checkpoint` (all steps
    when checkpoint is None)."""
    T = forces.shape[0]
    K = T if checkpoint is None else int(checkpoint)
    q, v = q0.clone(), v0.clone()
    ckpt = {0: (q.clone(), v.clone())}
    records = []
    for t in range(T):
        if t % K == 0:
            sim.reset_warm_start()
            ckpt[t] = (q.clone(), v.clone())
        q_new, v_new, rec = sim.step(q, v, forces[t], mu)
        if keep_records or checkpoint is None:
            records.append((q_new, rec))
        q, v = q_new, v_new
    return q, v, ckpt, records


def backward_pass(sim: GpuSim, forces, mu, ckpt, gq_T, gv_T, checkpoint=None, records=None, opts=None):
    """Backward recursion with segment recomputation.  Returns a dict with
    dq0, dv0, dforces (T, n, 3), grad3 = (dL/dE, dL/dnu, dL/dmu), iters."""
    T = forces.shape[0]
    K = T if checkpoint is None else int(checkpoint)
    opts = opts or sim.opts
    gq, gv = gq_T.clone(), gv_T.clone()
    grad3 = torch.zeros(3, dtype=torch.float64, device=gq.device)
    dforces = torch.zeros_like(forces)
    iters = []
    starts = list(range(0, T, K))
    for s0 in reversed(starts):
        s1 = min(s0 + K, T)
        if records is not None and len(records) == T:
            seg = records[s0:s1]
        else:
            q, v = ckpt[s0]
            sim.reset_warm_start()
            seg = []
            for t in range(s0, s1):
                q, v, rec = sim.step(q, v, forces[t], mu)
                seg.append((q, rec))
        for t in reversed(range(s0, s1)):
            q_t1, rec = seg[t - s0]
            dq, dv, df, info = sim.adjoint(q_t1, rec, gq, gv, grad3, opts)
            dforces[t] = df
            gq, gv = dq, dv
            iters.append(info.iters)
    return {"dq0": gq, "dv0": gv, "dforces": dforces, "grad3": grad3, "iters": iters}


class Rollout(torch.autograd.Function):
    """(q0, v0, forces[T, n, 3], params[3]) -> (q_T, v_T) through T implicit
    steps on the GPU; backward is the analytical adjoint with checkpointing.
    params = (E, nu, mu) as a float64 tensor (`GpuSim.params`): E and nu must
    be the scene's (its prefactored system matrix depends on them), mu is
    the friction coefficient of every step.  The gradient of params is
    (dL/dE, dL/dnu, dL/dmu) accumulated over the steps."""

    @staticmethod
    def forward(ctx, q0, v0, forces, params, sim, checkpoint):
        E, nu, mu = (float(x) for x in params.detach().cpu())
        if E != sim.E or nu != sim.nu:
            raise ValueError("params (E, nu) must be the scene's; build a GpuSim with the new values")
        qT, vT, ckpt, recs = forward_pass(sim, q0, v0, forces, mu, checkpoint)
        ctx.sim, ctx.mu, ctx.checkpoint = sim, mu, checkpoint
        ctx.ckpt, ctx.records = ckpt, (recs if checkpoint is None else None)
        ctx.save_for_backward(forces)
        return qT, vT

    @staticmethod
    def backward(ctx, gq, gv):
        (forces,) = ctx.saved_tensors
        gq = torch.zeros_like(forces[0]) if gq is None else gq.contiguous()
        gv = torch.zeros_like(forces[0]) if gv is None else gv.contiguous()
        out = backward_pass(ctx.sim, forces, ctx.mu, ctx.ckpt, gq, gv, ctx.checkpoint, ctx.records)
        return out["dq0"], out["dv0"], out["dforces"], out["grad3"], None, None


class Actuation(torch.autograd.Function):
    """a[T, G] -> forces[T, n, 3]: the external force of each step from the
    actuation parameters, f_t = Phi a_t (adj_actuation_force); backward
    dL/da_t = Phi^T dL/df_t (adj_actuation_vjp).  The scene's actuation
    tables come from native.set_actuation."""

    @staticmethod
    def forward(ctx, a, sim):
        T, G = a.shape
        f = torch.empty((T, sim.spec.n_verts, 3), dtype=torch.float64, device=a.device)
        for t in range(T):
            native.actuation_force(sim.scene, a[t].contiguous(), f[t])
        ctx.sim, ctx.G = sim, G
        return f

    @staticmethod
    def backward(ctx, gf):
        T = gf.shape[0]
        da = torch.empty((T, ctx.G), dtype=torch.float64, device=gf.device)
        for t in range(T):
            native.actuation_vjp(ctx.sim.scene, gf[t].contiguous(), da[t])
        return da, None


def rollout_with_param_grads(sim, q0, v0, forces, mu, loss_dir, checkpoint=None):
    """Forward + backward for the linear loss L = sum(loss_dir * q_T).
    Returns (L, grads) with grads = dq0, dv0, dforces, dE, dnu, dmu."""
    qT, vT, ckpt, recs = forward_pass(sim, q0, v0, forces, mu, checkpoint)
    L = float(torch.sum(loss_dir * qT))
    out = backward_pass(sim, forces, mu, ckpt, loss_dir.clone(), torch.zeros_like(loss_dir), checkpoint,
                        recs if checkpoint is None else None)
    g3 = out["grad3"].cpu().numpy()
    return L, {"dq0": out["dq0"], "dv0": out["dv0"], "dforces": out["dforces"], "dE": float(g3[0]),
               "dnu": float(g3[1]), "dmu": float(g3[2]), "iters": out["iters"]}
