"""Pins for the bilateral bindings of the oracle (Sec. 3.2 eq:binding;
Sec. 5.1 eq:differential_2 for the gradients): a tiny cube hung by four
top-face vertices, no ground, so every step is smooth.

* momentum balance at the converged step: the elastic forces sum to zero, so
  sum_v m_v (q_v - qtilde_v) = h^2 sum_b lambda_b with the binding forces
  lambda_b = -(q_b - d_b) / E_b, and gravity enters through qtilde;
* stiff bindings hold their vertices at the targets;
* dL/dd_b, dL/dE_b and dL/dqbar of the adjoint against central finite
  differences through the converged forward step.
"""

import dataclasses
import functools

import numpy as np

from oracle import adjoint as adj
from oracle.contact import predict
from oracle.fem import Bindings, discretise
from oracle.forward import solve_step
from synth import tiny_scene

NO_PLANES = np.zeros((0, 4))


def _spec():
    return dataclasses.replace(tiny_scene("impact"), planes=NO_PLANES)


def _bindings(spec, E=1e-4):
    rest = spec.mesh.rest
    top = np.flatnonzero(np.isclose(rest[:, 2], rest[:, 2].max()))
    xy = rest[top, :2]
    corners = [top[np.argmin(xy @ d)] for d in (np.array([1, 1]), np.array([-1, 1]), np.array([1, -1]),
                                                np.array([-1, -1]))]
    vid = np.array(sorted(corners))
    return Bindings(vid, np.full(vid.size, E))


def _disc(spec, bindings):
    return discretise(spec.mesh.rest, spec.mesh.tets, spec.density, spec.E, spec.nu, spec.h, bindings)


def _targets(spec, b):
    # held 1 mm to the side of their rest positions
    return spec.mesh.rest[b.vid] + np.array([1e-3, 0.0, 0.0])


def _step(spec, disc, qbar, vbar, targets):
    return solve_step(disc, qbar, vbar, np.zeros_like(qbar), spec.gravity, spec.mu, spec.eps, NO_PLANES,
                      margin=spec.contact_margin, targets=targets)


@functools.lru_cache(maxsize=None)
def _hanging(steps=3):
    spec = _spec()
    b = _bindings(spec)
    disc = _disc(spec, b)
    d = _targets(spec, b)
    q, v = spec.mesh.rest.copy(), np.zeros_like(spec.mesh.rest)
    states = [(q, v)]
    for _ in range(steps):
        q, v, rec, _ = _step(spec, disc, q, v, d)
        assert rec.residual < 1e-9
        states.append((q, v))
    return spec, b, disc, d, states


def test_binding_forces_balance_momentum():
    spec, b, disc, d, states = _hanging()
    (qbar, vbar), (q, v) = states[-2], states[-1]
    h = spec.h
    qtilde = predict(qbar, vbar, np.broadcast_to(spec.gravity, qbar.shape), h)
    lam_b = -(q[b.vid] - d) / b.E[:, None]
    lhs = np.sum(disc.mass[:, None] * (q - qtilde), axis=0)
    rhs = h * h * lam_b.sum(axis=0)
    assert np.allclose(lhs, rhs, rtol=1e-7, atol=1e-14 * np.abs(lhs).max())
    # one step from rest the bound vertices are still short of their targets
    # (1 mm in +x): every binding pulls in +x
    q1 = states[1][0]
    lam1 = -(q1[b.vid] - d) / b.E[:, None]
    assert np.all(lam1[:, 0] > 0)


def test_stiff_bindings_hold_their_vertices():
    spec = _spec()
    # compliance 1e-7 m/N: the ~N-sized forces that hold a corner 1 mm off its
    # rest position stretch the binding by ~1e-7 m
    b = _bindings(spec, E=1e-7)
    disc = _disc(spec, b)
    d = _targets(spec, b)
    q, v, rec, _ = _step(spec, disc, spec.mesh.rest.copy(), np.zeros_like(spec.mesh.rest), d)
    assert rec.residual < 1e-6
    assert np.max(np.abs(q[b.vid] - d)) < 1e-5


def test_binding_gradients_match_fd():
    spec, b, disc, d, states = _hanging()
    qbar, vbar = states[-2]
    q, v, rec, _ = _step(spec, disc, qbar, vbar, d)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(q.shape)
    gv = 1e-3 * rng.standard_normal(q.shape)
    grads = adj.adjoint_step(disc, q, rec, g, gv, spec.eps, spec.E, spec.nu)

    def loss(disc_, qbar_, targets_):
        q_, v_, r_, _ = _step(spec, disc_, qbar_, vbar, targets_)
        assert r_.residual < 1e-9
        return float(np.sum(g * q_) + np.sum(gv * v_))

    dd = rng.standard_normal(d.shape)
    eta = 1e-7
    fd_d = (loss(disc, qbar, d + eta * dd) - loss(disc, qbar, d - eta * dd)) / (2 * eta)
    assert abs(np.sum(grads.dtarget * dd) - fd_d) <= 1e-5 * abs(fd_d) + 1e-12

    for k in range(b.vid.size):
        e = np.zeros(b.vid.size)
        e[k] = 1e-4 * b.E[k]
        fp = loss(_disc(spec, Bindings(b.vid, b.E + e)), qbar, d)
        fm = loss(_disc(spec, Bindings(b.vid, b.E - e)), qbar, d)
        fd_e = (fp - fm) / (2 * e[k])
        assert abs(grads.dE_bind[k] - fd_e) <= 1e-5 * abs(fd_e) + 1e-9, k

    dq = rng.standard_normal(qbar.shape)
    eta = 1e-9
    fd_q = (loss(disc, qbar + eta * dq, d) - loss(disc, qbar - eta * dq, d)) / (2 * eta)
    assert abs(np.sum(grads.dqbar * dq) - fd_q) <= 1e-4 * abs(fd_q) + 1e-9


def test_woodbury_with_bindings_in_the_elastic_matrix():
    """The binding term belongs to the constant (prefactored) system matrix:
    with it in A, A - dA = Acal on a contact-free step."""
    spec, b, disc, d, states = _hanging()
    (qbar, vbar), (q, v) = states[-2], states[-1]
    rec = _step(spec, disc, qbar, vbar, d)[2]
    sysm = adj.assemble(disc, q, rec, spec.eps)
    no_b = _disc(spec, None)
    sysm0 = adj.assemble(no_b, q, rec, spec.eps)
    diff = (sysm.Acal - sysm0.Acal).toarray()
    assert np.allclose(diff, b.matrix(disc.n_verts, spec.h).toarray(), rtol=0, atol=1e-12 * np.abs(diff).max())
    assert np.allclose((disc.A - no_b.A).toarray(), diff, rtol=0, atol=1e-12 * np.abs(diff).max())
