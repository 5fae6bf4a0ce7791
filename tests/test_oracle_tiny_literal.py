"""Tiny cube, literal reading of its workload: dropped from 5 mm at rest with
tangential velocities, 20 steps of 1 ms, which never reach the ground.

Pins that hold for any correct implementation of the free-falling elastic
body (no contact, so Sec. 5.1's recursion reduces to the elastic blocks):
* no contact candidate in any step, so dL/dmu is exactly zero;
* the centre of mass follows the discrete free fall of implicit Euler with a
  lumped mass exactly (internal elastic forces sum to zero);
* translation invariance of the elastic energy: adding the same velocity c to
  every vertex moves q_T by T h c, and moving every vertex by c moves q_T by
  c, so sum_v dL/dv0_v = T h sum_v r_v and sum_v dL/dq0_v = sum_v r_v;
* dL/dE and dL/dnu against central differences of the rollout."""

import functools

import numpy as np
import pytest

from oracle.rollout import backward, linear_loss, run_forward
from synth import tiny_scene


@functools.lru_cache(maxsize=None)
def _literal():
    spec = tiny_scene("literal")
    ro = run_forward(spec)
    return spec, ro, backward(spec, ro, spec.loss_dir)


def _masses(ro):
    return np.asarray(ro.disc.mass).reshape(-1)


def test_no_contact_and_zero_friction_gradient():
    spec, ro, g = _literal()
    assert len(ro.records) == spec.steps == 20
    assert all(r.contacts.n == 0 for r in ro.records)
    assert g.dmu == 0.0


def test_centre_of_mass_is_discrete_free_fall():
    spec, ro, _ = _literal()
    m = _masses(ro)
    T, h = spec.steps, spec.h
    xc0 = (m[:, None] * spec.q0).sum(0) / m.sum()
    vc0 = (m[:, None] * spec.v0).sum(0) / m.sum()
    expect = xc0 + T * h * vc0 + h * h * spec.gravity * T * (T + 1) / 2
    xcT = (m[:, None] * ro.qs[-1]).sum(0) / m.sum()
    assert np.max(np.abs(xcT - expect)) <= 1e-13


def test_translation_invariance_of_the_gradient():
    spec, ro, g = _literal()
    T, h = spec.steps, spec.h
    r = spec.loss_dir
    np.testing.assert_allclose(g.dv0.sum(0), T * h * r.sum(0), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g.dq0.sum(0), r.sum(0), rtol=1e-10, atol=1e-12)


@pytest.mark.slow
def test_material_gradients_match_central_differences():
    spec, ro, g = _literal()
    L = lambda **kw: linear_loss(spec, run_forward(spec, **kw))  # noqa: E731
    dE = (L(E=spec.E * (1 + 1e-5)) - L(E=spec.E * (1 - 1e-5))) / (2e-5 * spec.E)
    dnu = (L(nu=spec.nu + 1e-6) - L(nu=spec.nu - 1e-6)) / 2e-6
    assert abs(g.dE - dE) <= 1e-5 * abs(dE), (g.dE, dE)
    assert abs(g.dnu - dnu) <= 1e-5 * abs(dnu), (g.dnu, dnu)
