"""Pins for the active stress of the actuated workload (the quadruped; the
paper's per-tet actuation of a soft body): the force matrix is the negative
gradient of the active energy (central differences), internal active forces
carry no net force and, at rest, no net torque (P_a symmetric), and the
gradient of a rollout loss with respect to the actuation parameters, dL/da_t
= Phi^T dL/df_t from the adjoint recursion, equals central differences
through the converged rollout (with a loss on the deformation: internal
forces alone do not move the centre of mass of a body in free flight)."""

import dataclasses

import numpy as np

from oracle import actuation as act
from oracle.rollout import backward, run_forward, scene_disc
from synth import tiny_scene
from synth.configs import actuation_groups, actuation_params


def _tiny():
    spec = dataclasses.replace(tiny_scene("impact"), E=2e5)
    group, fibre = actuation_groups(spec.mesh)
    return spec, scene_disc(spec), group, fibre


def test_force_matrix_is_minus_energy_gradient():
    spec, disc, group, fibre = _tiny()
    rng = np.random.default_rng(3)
    a = rng.uniform(-1e4, 1e4, 64)
    Phi = act.force_matrix(disc, group, fibre, 64)
    f = (Phi @ a).reshape(-1, 3)
    q = spec.mesh.rest + 1e-3 * rng.standard_normal(spec.mesh.rest.shape)
    for _ in range(3):
        dq = rng.standard_normal(q.shape)
        eta = 1e-6
        fd = (act.active_energy(disc, group, fibre, a, q + eta * dq) -
              act.active_energy(disc, group, fibre, a, q - eta * dq)) / (2 * eta)
        assert abs(-np.sum(f * dq) - fd) <= 1e-7 * abs(fd) + 1e-12


def test_no_net_force_or_torque_at_rest():
    spec, disc, group, fibre = _tiny()
    a = np.random.default_rng(4).uniform(-1e4, 1e4, 64)
    f = (act.force_matrix(disc, group, fibre, 64) @ a).reshape(-1, 3)
    scale = np.abs(f).sum()
    assert np.all(np.abs(f.sum(axis=0)) <= 1e-12 * scale)
    torque = np.cross(spec.mesh.rest, f).sum(axis=0)
    assert np.all(np.abs(torque) <= 1e-12 * scale * np.abs(spec.mesh.rest).max())


def test_rollout_actuation_gradient_matches_fd():
    spec, disc, group, fibre = _tiny()
    T = 6
    Phi = act.force_matrix(disc, group, fibre, 64)
    a = actuation_params(T, amplitude=2e3)
    n = spec.n_verts

    def rollout(aa):
        forces = [(Phi @ aa[t]).reshape(n, 3) for t in range(T)]
        return run_forward(spec, steps=T, disc=disc, forces=forces)

    # a loss on the deformation (internal active forces alone cannot move
    # the centre of mass of a body in free flight)
    def loss(ro):
        return float(np.sum(spec.loss_dir * ro.qs[-1]))

    ro = rollout(a)
    g = backward(spec, ro, spec.loss_dir)
    da = np.stack([Phi.T @ g.dfext[t].reshape(-1) for t in range(T)])
    rng = np.random.default_rng(5)
    for _ in range(2):
        d = rng.standard_normal(a.shape)
        eta = 1e-2
        fd = (loss(rollout(a + eta * d)) - loss(rollout(a - eta * d))) / (2 * eta)
        assert abs(fd) > 1e-12
        assert abs(np.sum(da * d) - fd) <= 1e-5 * abs(fd), (np.sum(da * d), fd)
