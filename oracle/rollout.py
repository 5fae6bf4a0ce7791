"""Rollout and backward recursion over time (Sec. 5.1; Sec. 4 framework).
Test infrastructure only.

Per step t (qbar = q_t, vbar = v_t -> q_{t+1}, v_{t+1} = (q_{t+1} - q_t)/h):
    solve Acal_t^T z_t = g_q + g_v / h
    g_q <- dL/dqbar,  g_v <- dL/dvbar = h M z_t        (propagated)
    dL/df_ext,t = h^2 z_t                               (per step, final)
    dL/dE, dL/dnu, dL/dmu accumulate over steps          (global)
The initial-velocity gradient is dL/dv_0 = h M z_0.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .adjoint import adjoint_step
from .fem import discretise
from .forward import solve_step


@dataclasses.dataclass
class Rollout:
    qs: list
    vs: list
    records: list
    disc: object


def scene_disc(spec, E=None, nu=None):
    return discretise(spec.mesh.rest, spec.mesh.tets, spec.density,
                      spec.E if E is None else E, spec.nu if nu is None else nu, spec.h,
                      model=getattr(spec, "material", "nh"))


def run_forward(spec, steps=None, E=None, nu=None, mu=None, v0=None, q0=None, disc=None,
                forces=None) -> Rollout:
    disc = disc if disc is not None else scene_disc(spec, E, nu)
    mu = spec.mu if mu is None else mu
    q = (spec.q0 if q0 is None else q0).copy()
    v = (spec.v0 if v0 is None else v0).copy()
    T = spec.steps if steps is None else steps
    qs, vs, recs = [q], [v], []
    warm = None
    for t in range(T):
        f = spec.force(t) if forces is None else forces[t]
        q, v, rec, warm = solve_step(disc, q, v, f, spec.gravity, mu, spec.eps, spec.planes,
                                     spec.sphere_array(t), spec.sphere_array(t + 1),
                                     spec.contact_margin, warm)
        qs.append(q)
        vs.append(v)
        recs.append(rec)
    return Rollout(qs, vs, recs, disc)


@dataclasses.dataclass
class RolloutGradients:
    dq0: np.ndarray
    dv0: np.ndarray
    dfext: list
    dE: float
    dnu: float
    dmu: float
    zs: list


def backward(spec, ro: Rollout, dL_dqT, dL_dvT=None, E=None, nu=None) -> RolloutGradients:
    E = spec.E if E is None else E
    nu = spec.nu if nu is None else nu
    gq = dL_dqT.copy()
    gv = np.zeros_like(gq) if dL_dvT is None else dL_dvT.copy()
    dE = dnu = dmu = 0.0
    dfext = [None] * len(ro.records)
    zs = [None] * len(ro.records)
    for t in reversed(range(len(ro.records))):
        g = adjoint_step(ro.disc, ro.qs[t + 1], ro.records[t], gq, gv, spec.eps, E, nu)
        dE += g.dE
        dnu += g.dnu
        dmu += g.dmu_fric
        dfext[t] = g.dfext
        zs[t] = g.z
        gq, gv = g.dqbar, g.dvbar
    return RolloutGradients(gq, gv, dfext, dE, dnu, dmu, zs)


def linear_loss(spec, ro: Rollout) -> float:
    return float(np.sum(spec.loss_dir * ro.qs[-1]))
