"""GPU forward step against the oracle's converged states, and a full GPU
rollout gradient (forward + adjoint recursion) against the oracle's and
central finite differences."""

import functools

import numpy as np
import pytest

from gpu_helpers import rel, torch_cuda
from oracle.rollout import backward, linear_loss, run_forward
from synth import tiny_scene

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _tiny(steps):
    spec = tiny_scene("impact")
    return spec, run_forward(spec, steps=steps)


@pytest.mark.parametrize("step", [4, 9, 12, 16])
def test_forward_step_matches_oracle(step):
    """One step from the oracle's (qbar, vbar), both sides started cold (no
    multiplier warm start): same contact list and flags (bit-exact) and the
    same converged positions and multipliers.  The cold start matters: with
    friction the step can have several solutions, and a warm-started solve
    may keep a contact frictional that a cold-started one demotes."""
    torch = torch_cuda()
    from oracle import forward as fw
    from paper_2603_16478_amd.rollout import GpuSim
    spec, ro = _tiny(20)
    q_ref, _, ref, _ = fw.solve_step(ro.disc, ro.qs[step], ro.vs[step], spec.force(step), spec.gravity, spec.mu,
                                     spec.eps, spec.planes, margin=spec.contact_margin)
    sim = GpuSim(spec, max_contacts=64)
    dev = "cuda"
    qbar = torch.tensor(ro.qs[step], device=dev)
    vbar = torch.tensor(ro.vs[step], device=dev)
    f = torch.tensor(spec.force(step), device=dev)
    q, v, rec = sim.step(qbar, vbar, f, spec.mu)
    n = rec.n
    print(f"step {step}: contacts {n} (oracle {ref.contacts.n}), frictional "
          f"{int(rec.fric[:n].sum())} (oracle {int(ref.contacts.fric.sum())})", flush=True)
    assert n == ref.contacts.n
    np.testing.assert_array_equal(rec.vid[:n].cpu().numpy(), ref.contacts.vid)
    np.testing.assert_array_equal(rec.fric[:n].cpu().numpy().astype(bool), ref.contacts.fric)
    np.testing.assert_array_equal(rec.frame[:n].cpu().numpy().reshape(-1, 3, 3), ref.contacts.frame)
    du = q.cpu().numpy() - ro.qs[step]
    du_ref = q_ref - ro.qs[step]
    assert rel(du, du_ref) <= 1e-7, rel(du, du_ref)
    if n:
        assert rel(rec.lam[:n].cpu().numpy(), ref.lam) <= 1e-6


def test_gpu_rollout_gradient_matches_oracle():
    """20-step tiny-impact rollout entirely on the GPU (forward steps + adjoint
    recursion): dL/dE, dL/dnu, dL/dv0 against the oracle's recursion and
    against central differences of the GPU loss."""
    torch = torch_cuda()
    from paper_2603_16478_amd.rollout import GpuSim, rollout_with_param_grads
    spec, ro = _tiny(20)
    g_ref = backward(spec, ro, spec.loss_dir)
    L_ref = linear_loss(spec, ro)
    dev = "cuda"
    q0 = torch.tensor(spec.q0, device=dev)
    v0 = torch.tensor(spec.v0, device=dev)
    forces = torch.zeros((spec.steps, spec.n_verts, 3), dtype=torch.float64, device=dev)
    r = torch.tensor(spec.loss_dir, device=dev)
    sim = GpuSim(spec, max_contacts=64)
    L, g = rollout_with_param_grads(sim, q0, v0, forces, spec.mu, r)
    print("L", L, L_ref, "dE", g["dE"], g_ref.dE, "dnu", g["dnu"], g_ref.dnu, flush=True)
    assert abs(L - L_ref) <= 1e-9 * abs(L_ref)
    assert abs(g["dE"] - g_ref.dE) <= 1e-6 * abs(g_ref.dE)
    assert abs(g["dnu"] - g_ref.dnu) <= 1e-6 * abs(g_ref.dnu)
    assert rel(g["dv0"].cpu().numpy(), g_ref.dv0) <= 1e-6
    # central differences of the GPU rollout in E
    def L_of(E):
        s2 = GpuSim(spec, max_contacts=64, E=E)
        from paper_2603_16478_amd.rollout import forward_pass
        qT, _, _, _ = forward_pass(s2, q0, v0, forces, spec.mu)
        return float(torch.sum(r * qT))
    eta = 1e-6 * spec.E
    fd = (L_of(spec.E + eta) - L_of(spec.E - eta)) / (2 * eta)
    assert abs(g["dE"] - fd) <= 1e-5 * abs(fd), (g["dE"], fd)


def test_checkpointed_backward_is_bitwise_equal():
    """Checkpointing every 5 steps (recomputing segments) gives bitwise the
    same gradients as keeping every step's record (same reset schedule)."""
    torch = torch_cuda()
    from paper_2603_16478_amd.rollout import GpuSim, backward_pass, forward_pass
    spec, _ = _tiny(20)
    dev = "cuda"
    q0 = torch.tensor(spec.q0, device=dev)
    v0 = torch.tensor(spec.v0, device=dev)
    forces = torch.zeros((spec.steps, spec.n_verts, 3), dtype=torch.float64, device=dev)
    r = torch.tensor(spec.loss_dir, device=dev)
    sim = GpuSim(spec, max_contacts=64)
    _, _, ck, recs = forward_pass(sim, q0, v0, forces, spec.mu, checkpoint=5, keep_records=True)
    a = backward_pass(sim, forces, spec.mu, ck, r.clone(), torch.zeros_like(r), 5, records=recs)
    b = backward_pass(sim, forces, spec.mu, ck, r.clone(), torch.zeros_like(r), 5, records=None)
    assert torch.equal(a["dv0"], b["dv0"]) and torch.equal(a["dq0"], b["dq0"])
    assert torch.equal(a["grad3"], b["grad3"]) and torch.equal(a["dforces"], b["dforces"])
