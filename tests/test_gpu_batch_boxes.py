"""The batched workload in reduced form: eight boxes of uneven size (540 to
1,680 vertices), E from 1e4 to 6e6 Pa, nu up to 0.48, mu from 0.27 to 0.88,
resting on the ground with a seeded tangential velocity (one in eight
hovers, contact-free).  One GPU forward step per scene gives the converged
states; the batched adjoint of all eight must equal each scene's
single-scene adjoint (1e-9) and, for a sample, the FP64 oracle (1e-9)."""

import functools

import numpy as np
import pytest

from gpu_helpers import rel, torch_cuda
from oracle import adjoint as adj
from oracle.contact import ContactSet
from oracle.forward import StepRecord
from oracle.rollout import scene_disc
from synth.configs import batched_scenes

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _states():
    torch = torch_cuda()
    from paper_2603_16478_amd.rollout import GpuSim
    scenes = batched_scenes(8, seed=3, tmax=8000)
    out = []
    for spec in scenes:
        sim = GpuSim(spec, max_contacts=spec.n_verts)
        q0 = torch.tensor(spec.q0, device="cuda")
        v0 = torch.tensor(spec.v0, device="cuda")
        f = torch.zeros_like(q0)
        q, v, rec = sim.step(q0, v0, f, spec.mu)
        out.append((spec, sim, q, rec))
        print(f"{spec.name}: verts {spec.n_verts}, contacts {rec.n}, frictional {int(rec.fric[:rec.n].sum())}",
              flush=True)
    return out


def _oracle_record(rec, mu):
    n = rec.n
    cs = ContactSet(rec.vid[:n].cpu().numpy().astype(np.int64), np.zeros(n, dtype=np.int64),
                    rec.frame[:n].cpu().numpy().reshape(n, 3, 3), rec.d_n[:n].cpu().numpy(),
                    rec.d_f[:n].cpu().numpy(), rec.fric[:n].cpu().numpy().astype(bool))
    return StepRecord(cs, rec.delta[:n].cpu().numpy(), rec.lam[:n].cpu().numpy(), mu)


def test_batched_boxes_match_single_scene_and_oracle():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    states = _states()
    spec0 = states[0][0]
    batch = native.Batch([(s.mesh.rest, s.mesh.tets, s.E, s.nu) for s, _, _, _ in states], spec0.density, spec0.h,
                         spec0.eps, spec0.gravity, spec0.planes, spec0.contact_margin,
                         [max(1, r.n) for _, _, _, r in states])
    dev = "cuda"
    q = torch.cat([qq for _, _, qq, _ in states])
    gq = torch.tensor(np.concatenate([s.loss_dir for s, _, _, _ in states]), device=dev)
    gv = torch.zeros_like(gq)
    z = torch.zeros_like(gq)
    opts = native.solve_opts(rtol=1e-12, maxit=3000)
    native.batch_setup(batch, [r.state for _, _, _, r in states], q, opts)
    native.batch_check_status(batch)
    infos = native.batch_solve(batch, gq, gv, z, opts, raise_noconv=False)
    dq, dv, df = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
    grad = torch.zeros(3 * len(states), dtype=torch.float64, device=dev)
    native.batch_vjp(batch, z, gv, dq, dv, df, grad)
    torch.cuda.synchronize()
    zb, dqb, g = z.cpu().numpy(), dq.cpu().numpy(), grad.cpu().numpy().reshape(-1, 3)
    voff = batch.voff
    for k, (spec, sim, qk, rec) in enumerate(states):
        v0, v1 = voff[k], voff[k + 1]
        info = infos[k]
        assert info.relres <= 1e-11, (k, info.relres)
        # the same scene alone
        zs = torch.zeros_like(qk)
        native.adjoint_setup(sim.scene, rec.state, qk, opts)
        gqk = torch.tensor(spec.loss_dir, device=dev)
        native.adjoint_solve(sim.scene, gqk, torch.zeros_like(gqk), zs, opts, raise_noconv=False)
        g3 = torch.zeros(3, dtype=torch.float64, device=dev)
        d1, d2, d3 = torch.empty_like(qk), torch.empty_like(qk), torch.empty_like(qk)
        native.vjp_params(sim.scene, zs, torch.zeros_like(gqk), d1, d2, d3, g3)
        err = rel(zb[v0:v1], zs.cpu().numpy())
        print(f"scene {k}: contacts {rec.n}, iters {info.iters}, relres {info.relres:.2e}, batch vs single {err:.2e}",
              flush=True)
        assert err <= 1e-9
        assert rel(dqb[v0:v1], d1.cpu().numpy()) <= 1e-9
        assert np.allclose(g[k], g3.cpu().numpy(), rtol=1e-9, atol=1e-12 * np.abs(g3.cpu().numpy()).max())
        if k in (0, 4, 7):  # oracle sample: stiff, soft, contact-free
            ref = adj.adjoint_step(scene_disc(spec), qk.cpu().numpy(), _oracle_record(rec, spec.mu), spec.loss_dir,
                                   np.zeros_like(spec.loss_dir), spec.eps, spec.E, spec.nu)
            e2 = rel(zb[v0:v1], ref.z)
            print(f"  oracle z err {e2:.2e}", flush=True)
            assert e2 <= 1e-9
            assert abs(g[k][0] - ref.dE) <= 1e-9 * np.abs(ref.dE_tet).sum()
            assert abs(g[k][2] - ref.dmu_fric) <= 1e-9 * max(abs(ref.dmu_fric), 1e-30) + 1e-20
    batch.close()
