"""Actuation by per-tet active stress (the actuated workload, the quadruped):
the GPU force map f = Phi a and its transpose against the oracle's force
matrix on the full quadruped mesh; the gradient of a rollout loss with
respect to the actuation parameters through the autograd layers (Actuation
then Rollout) against the oracle's recursion on the tiny cube; and on the
quadruped, that gradient against central differences of the GPU rollout
(losses on the final positions)."""

import dataclasses
import time

import numpy as np
import pytest

from gpu_helpers import rel, torch_cuda
from oracle import actuation as act
from oracle.rollout import backward, run_forward, scene_disc
from synth import tiny_scene
from synth.configs import actuation_groups, actuation_params, quadruped_scene

pytestmark = pytest.mark.gpu


def test_actuation_map_matches_oracle_on_quadruped():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    from paper_2603_16478_amd.rollout import GpuSim
    spec = quadruped_scene()
    group, fibre = actuation_groups(spec.mesh)
    disc = scene_disc(spec)
    Phi = act.force_matrix(disc, group, fibre, 64)
    sim = GpuSim(spec, max_contacts=400)
    native.set_actuation(sim.scene, group, fibre, 64)
    rng = np.random.default_rng(8)
    a = rng.uniform(-1e4, 1e4, 64)
    g = rng.standard_normal(3 * spec.n_verts)
    f = torch.empty(3 * spec.n_verts, dtype=torch.float64, device="cuda")
    da = torch.empty(64, dtype=torch.float64, device="cuda")
    native.actuation_force(sim.scene, torch.tensor(a, device="cuda"), f)
    native.actuation_vjp(sim.scene, torch.tensor(g, device="cuda"), da)
    torch.cuda.synchronize()
    e_f, e_a = rel(f.cpu().numpy(), Phi @ a), rel(da.cpu().numpy(), Phi.T @ g)
    print(f"quadruped ({spec.n_tets} tets): force err {e_f:.1e}, transpose err {e_a:.1e}", flush=True)
    assert e_f <= 1e-13
    assert e_a <= 1e-12


def test_actuated_rollout_gradient_matches_oracle():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    from paper_2603_16478_amd.rollout import Actuation, GpuSim, Rollout
    spec = dataclasses.replace(tiny_scene("impact"), E=2e5)
    T = 6
    group, fibre = actuation_groups(spec.mesh)
    disc = scene_disc(spec)
    Phi = act.force_matrix(disc, group, fibre, 64)
    a_np = actuation_params(T, amplitude=2e3)
    w = spec.loss_dir  # a loss on the deformation (the cube is in free flight)
    ro = run_forward(spec, steps=T, disc=disc, forces=[(Phi @ a_np[t]).reshape(-1, 3) for t in range(T)])
    g = backward(spec, ro, w)
    da_ref = np.stack([Phi.T @ g.dfext[t].reshape(-1) for t in range(T)])
    sim = GpuSim(spec, max_contacts=64)
    native.set_actuation(sim.scene, group, fibre, 64)
    a = torch.tensor(a_np, device="cuda", requires_grad=True)
    q0 = torch.tensor(spec.q0, device="cuda")
    v0 = torch.tensor(spec.v0, device="cuda")
    qT, vT = Rollout.apply(q0, v0, Actuation.apply(a, sim), sim.params(spec.mu), sim, 3)
    loss = torch.sum(torch.tensor(w, device="cuda") * qT)
    loss.backward()
    L_ref = float(np.sum(w * ro.qs[-1]))
    e_L = abs(float(loss.detach()) - L_ref) / abs(L_ref)
    e_g = rel(a.grad.cpu().numpy(), da_ref)
    print(f"tiny actuated rollout: loss err {e_L:.1e}, dL/da err {e_g:.1e}", flush=True)
    assert e_L <= 1e-9
    assert e_g <= 1e-7


def test_quadruped_actuation_gradient_matches_fd():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    from paper_2603_16478_amd.rollout import Actuation, GpuSim, Rollout
    spec = quadruped_scene()
    T, K = 8, 4
    group, fibre = actuation_groups(spec.mesh)
    # the workload's loss is the centre-of-mass shift; over the few steps of
    # a test that is too small a number for central differences, so the
    # check uses a seeded linear loss on the final positions
    w = torch.tensor(np.random.default_rng(10).standard_normal(spec.q0.shape), device="cuda")
    sim = GpuSim(spec, max_contacts=400)
    native.set_actuation(sim.scene, group, fibre, 64)
    q0 = torch.tensor(spec.q0, device="cuda")
    # The quadruped slides at 0.2 m/s along x: a foot that stands still under
    # almost no tangential load converges with a friction magnitude s of
    # either sign, decided by the slip direction of the first Newton iterate,
    # and the forward demotes a contact with s < 0 to normal-only, so probes
    # of 1e-8 relative switch branches there.  Sliding feet carry s = mu
    # lambda_n, far from that switch, for the whole test.
    v0 = torch.zeros_like(q0)
    v0[:, 0] = 0.2
    a0 = torch.tensor(actuation_params(T, amplitude=2e3), device="cuda")

    def loss_of(a):
        qT, _ = Rollout.apply(q0, v0, Actuation.apply(a, sim), sim.params(spec.mu, False), sim, K)
        return torch.sum(w * qT)

    t0 = time.perf_counter()
    a = a0.clone().requires_grad_(True)
    L = loss_of(a)
    L.backward()
    print(f"quadruped: {T} steps forward + backward {time.perf_counter() - t0:.1f} s, loss {float(L.detach()):.6e}",
          flush=True)
    from paper_2603_16478_amd.rollout import forward_pass

    def run(a):
        """Loss and the per-step contact state (vertices, friction flags)
        of the forward with the gradient's checkpoint schedule."""
        qT, _, _, recs = forward_pass(sim, q0, v0, Actuation.apply(a, sim), spec.mu, K, keep_records=True)
        state = [(r.vid[:r.n].cpu().numpy().tobytes(), r.fric[:r.n].cpu().numpy().tobytes()) for _, r in recs]
        return float(torch.sum(w * qT)), state

    L0, base = run(a0)
    _, again = run(a0)
    assert again == base  # the forward rollout is deterministic
    rng = np.random.default_rng(9)
    checked = 0
    with torch.no_grad():
        for i in range(8):
            d = torch.tensor(rng.standard_normal(a0.shape), device="cuda")
            ad = float(torch.sum(a.grad * d))
            # central differences where neither side changes a contact's
            # frictional flag or the contact set (the step map is not
            # differentiable across those changes); parameters are ~2e3 Pa.
            # A direction along which every probe step changes the contact
            # state (a contact at its switching threshold) is skipped.
            for eta in (0.02, 0.002, 0.0002, 0.00002):
                (lp, sp), (lm, sm) = run(a0 + eta * d), run(a0 - eta * d)
                if sp == base and sm == base:
                    break
            else:
                bad = [t for t in range(T) if sp[t] != base[t] or sm[t] != base[t]]
                print(f"  direction {i}: the contact state changes at steps {bad} under every probe step", flush=True)
                continue
            fd = (lp - lm) / (2 * eta)
            print(f"  direction {i}: adjoint {ad:.6e}, central difference {fd:.6e} (step {eta} Pa)", flush=True)
            assert abs(ad - fd) <= 1e-5 * abs(fd)
            checked += 1
            if checked == 3:
                break
    assert checked == 3
