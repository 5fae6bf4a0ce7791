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


def _oracle_records(recs, mu):
    """The GPU's step records in the oracle's format, so that the oracle's
    recursion runs on the GPU's own converged states."""
    from oracle.contact import ContactSet
    from oracle.forward import StepRecord
    out = []
    for _, r in recs:
        n = r.n
        cs = ContactSet(r.vid[:n].cpu().numpy().astype(np.int32), np.zeros(n, np.int32),
                        r.frame[:n].cpu().numpy().reshape(n, 3, 3), r.d_n[:n].cpu().numpy(),
                        r.d_f[:n].cpu().numpy(), r.fric[:n].cpu().numpy().astype(bool))
        out.append(StepRecord(cs, r.delta[:n].cpu().numpy().copy(), r.lam[:n].cpu().numpy().copy(),
                              mu))
    return out


@functools.lru_cache(maxsize=None)
def _oracle_rollout(variant):
    spec = tiny_scene(variant)
    return spec, run_forward(spec)


@pytest.mark.parametrize("variant", ["impact", "literal"])
def test_gpu_rollout_gradient_matches_oracle(variant):
    """20-step tiny rollout entirely on the GPU (forward steps + adjoint
    recursion through the Rollout autograd layer): every gradient (E, nu,
    mu, q0, v0 and the per-step external forces) against the oracle's
    recursion run on the GPU's own converged states at 1e-9, so that the
    forward solves' tolerance does not enter; the GPU forward against the
    oracle's forward; dL/dE against central differences of the GPU loss.
    The literal variant never touches the ground: dL/dmu is exactly 0."""
    torch = torch_cuda()
    from oracle.rollout import Rollout as OracleRollout
    from oracle.rollout import scene_disc
    from paper_2603_16478_amd import native
    from paper_2603_16478_amd.rollout import GpuSim, Rollout, forward_pass
    spec, ro = _oracle_rollout(variant)
    dev = "cuda"
    q0 = torch.tensor(spec.q0, device=dev, requires_grad=True)
    v0 = torch.tensor(spec.v0, device=dev, requires_grad=True)
    forces = torch.zeros((spec.steps, spec.n_verts, 3), dtype=torch.float64, device=dev, requires_grad=True)
    r = torch.tensor(spec.loss_dir, device=dev)
    sim = GpuSim(spec, max_contacts=64)
    sim.opts = native.solve_opts(rtol=1e-13, maxit=4000, restart=64)
    params = sim.params(spec.mu)
    qT, _ = Rollout.apply(q0, v0, forces, params, sim, None)
    L = torch.sum(r * qT)
    L.backward()
    # the same forward again (bitwise: same warm-start schedule), keeping its records
    _, _, _, recs = forward_pass(sim, q0.detach(), v0.detach(), forces.detach(), spec.mu, None, keep_records=True)
    qs = [spec.q0] + [q.cpu().numpy() for q, _ in recs]
    ro_gpu = OracleRollout(qs, None, _oracle_records(recs, spec.mu), scene_disc(spec))
    g = backward(spec, ro_gpu, spec.loss_dir)
    pg = params.grad.cpu().numpy()
    errs = {"dE": abs(pg[0] - g.dE) / abs(g.dE), "dnu": abs(pg[1] - g.dnu) / abs(g.dnu),
            "dq0": rel(q0.grad.cpu().numpy(), g.dq0), "dv0": rel(v0.grad.cpu().numpy(), g.dv0),
            "dfext": rel(forces.grad.cpu().numpy(), np.stack(g.dfext))}
    if variant == "literal":
        assert all(rr.n == 0 for _, rr in recs)
        assert pg[2] == 0.0 and g.dmu == 0.0
    else:
        errs["dmu"] = abs(pg[2] - g.dmu) / abs(g.dmu)
    print(variant, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= 1e-9, (k, e)
    # the GPU forward against the oracle's forward
    L_ref = linear_loss(spec, ro)
    assert abs(float(L.detach()) - L_ref) <= 1e-9 * abs(L_ref)
    # central differences of the GPU rollout in E
    def L_of(E):
        s2 = GpuSim(spec, max_contacts=64, E=E)
        qT2, _, _, _ = forward_pass(s2, q0.detach(), v0.detach(), forces.detach(), spec.mu)
        return float(torch.sum(r * qT2))
    eta = 1e-6 * spec.E
    fd = (L_of(spec.E + eta) - L_of(spec.E - eta)) / (2 * eta)
    assert abs(pg[0] - fd) <= 1e-5 * abs(fd), (pg[0], fd)


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
