"""Pins for the adjoint with the as-rigid-as-possible and co-rotational
local steps (App. B.2; the projection Jacobians themselves are pinned in
test_oracle_elastic.py): on a frictional step of the tiny impact scene, the
per-step gradients dL/dE, dL/dnu, dL/dmu and dL/dqbar equal central finite
differences through the converged forward step, and the forward step
balances momentum (the elastic forces of each model sum to zero)."""

import dataclasses
import functools

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle.contact import predict
from oracle.forward import solve_step
from oracle.rollout import run_forward, scene_disc
from synth import tiny_scene


@functools.lru_cache(maxsize=None)
def _run(material, steps):
    spec = dataclasses.replace(tiny_scene("impact"), material=material)
    return spec, run_forward(spec, steps=steps)


def _warm(rec):
    return {(int(rec.contacts.vid[c]), int(rec.contacts.collider[c])):
            (rec.lam[c, 0], float(np.hypot(rec.lam[c, 1], rec.lam[c, 2]))) for c in range(rec.contacts.n)}


@pytest.mark.parametrize("material", ["arap", "corot"])
def test_contact_free_momentum_balance(material):
    spec, ro = _run(material, 4)
    q, qbar, vbar = ro.qs[4], ro.qs[3], ro.vs[3]
    assert ro.records[3].contacts.n == 0
    qt = predict(qbar, vbar, np.broadcast_to(spec.gravity, qbar.shape), spec.h)
    lhs = np.sum(ro.disc.mass[:, None] * (q - qt), axis=0)
    assert np.max(np.abs(lhs)) <= 1e-12 * np.max(ro.disc.mass) * np.max(np.abs(q - qbar))


@pytest.mark.slow
@pytest.mark.parametrize("material", ["arap", "corot"])
def test_step_gradients_match_fd(material):
    step = 13
    spec, ro = _run(material, step)
    disc = ro.disc
    qbar, vbar = ro.qs[-1], ro.vs[-1]
    warm = _warm(ro.records[-1])
    f = spec.force(step)
    q, v, rec, _ = solve_step(disc, qbar, vbar, f, spec.gravity, spec.mu, spec.eps, spec.planes,
                              margin=spec.contact_margin, warm=warm)
    assert rec.residual < 1e-9
    assert rec.contacts.fric.any()
    rng = np.random.default_rng(70)
    g = rng.standard_normal(qbar.shape)
    gv = 1e-3 * rng.standard_normal(qbar.shape)
    grads = adj.adjoint_step(disc, q, rec, g, gv, spec.eps, spec.E, spec.nu)

    def loss(d, qb, mu):
        q_, v_, r_, _ = solve_step(d, qb, vbar, f, spec.gravity, mu, spec.eps, spec.planes,
                                   margin=spec.contact_margin, warm=warm)
        return float(np.sum(g * q_) + np.sum(gv * v_)), r_

    def fd(fun, eta):
        for _ in range(6):
            (lp, rp), (lm, rm) = fun(eta), fun(-eta)
            if all(np.array_equal(r.contacts.vid, rec.contacts.vid) and np.array_equal(r.contacts.fric,
                                                                                        rec.contacts.fric)
                   for r in (rp, rm)):
                return (lp - lm) / (2 * eta)
            eta /= 10.0
        raise AssertionError("contact state changes under every probe step")

    dE = fd(lambda e: loss(scene_disc(spec, E=spec.E + e), qbar, spec.mu), 1e-5 * spec.E)
    dnu = fd(lambda e: loss(scene_disc(spec, nu=spec.nu + e), qbar, spec.mu), 1e-6)
    dmu = fd(lambda e: loss(disc, qbar, spec.mu + e), 1e-5)
    dq = rng.standard_normal(qbar.shape)
    dqb = fd(lambda e: loss(disc, qbar + e * dq, spec.mu), 1e-9)
    print(f"{material}: dE {grads.dE:.6e} / {dE:.6e}, dnu {grads.dnu:.6e} / {dnu:.6e}, "
          f"dmu {grads.dmu_fric:.6e} / {dmu:.6e}, dqbar {np.sum(grads.dqbar * dq):.6e} / {dqb:.6e}")
    assert abs(grads.dE - dE) <= 1e-5 * abs(dE) + 1e-14
    assert abs(grads.dnu - dnu) <= 1e-5 * abs(dnu) + 1e-12
    assert abs(grads.dmu_fric - dmu) <= 1e-3 * abs(dmu) + 1e-9
    assert abs(np.sum(grads.dqbar * dq) - dqb) <= 1e-4 * abs(dqb) + 1e-9
