"""The batched workload over its full range of scene sizes: the first 16
boxes of the seeded 256-box set (2,058 to 97,650 tets, 69,590 vertices in
all; two hover above the ground), each at a seeded deformed state with the
ground contacts the detection finds there and seeded sticking contact
values, solved as one batch in FP64 (the Woodbury correction goes through
S^T S of the union at this size).  Checked per scene at any size: the GPU z
satisfies the oracle's assembled system to the solve's tolerance, and the
oracle's gradient contractions from that z equal the GPU's (FP64 bar)."""

import numpy as np
import pytest

from gpu_helpers import contact_tensors, rel, torch_cuda
from oracle import adjoint as adj
from oracle.contact import detect, predict
from oracle.forward import StepRecord
from oracle.rollout import scene_disc
from synth.configs import batched_scenes, contact_values, perturbed_state

pytestmark = pytest.mark.gpu


def test_batched_boxes_full_range_properties():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    specs = batched_scenes(16, seed=3, tmax=1e5)
    cases = []
    for k, spec in enumerate(specs):
        q = perturbed_state(spec, seed=100 + k)
        qt = predict(q, np.zeros_like(q), np.broadcast_to(spec.gravity, q.shape), spec.h)
        cs = detect(q, qt, spec.planes, np.zeros((0, 4)), np.zeros((0, 4)), spec.contact_margin)
        delta, lam = contact_values(cs.n, spec.mu, seed=200 + k)
        cases.append((spec, q, StepRecord(cs, delta, lam, spec.mu)))
    s0 = specs[0]
    print(f"{len(specs)} boxes, {sum(s.n_tets for s in specs)} tets, {sum(s.n_verts for s in specs)} vertices, "
          f"contacts {[c[2].contacts.n for c in cases]}; building the batch", flush=True)
    batch = native.Batch([(s.mesh.rest, s.mesh.tets, s.E, s.nu) for s in specs], s0.density, s0.h, s0.eps,
                         s0.gravity, s0.planes, s0.contact_margin, [max(1, c[2].contacts.n) for c in cases])
    keep, states = [], []
    for spec, q, rec in cases:
        tens = contact_tensors(rec)
        keep.append(tens)
        states.append(native.make_contact_state(rec.contacts.n, tens["vid"], tens["fric"], tens["frame"],
                                                tens["delta"], tens["lam"], rec.mu))
    rng = np.random.default_rng(300)
    gqs = [rng.standard_normal(c[1].shape) for c in cases]
    gvs = [1e-3 * rng.standard_normal(c[1].shape) for c in cases]
    dev = "cuda"
    qd = torch.tensor(np.concatenate([c[1] for c in cases]), device=dev)
    gq = torch.tensor(np.concatenate(gqs), device=dev)
    gv = torch.tensor(np.concatenate(gvs), device=dev)
    opts = native.solve_opts(rtol=1e-10, maxit=1000, restart=64)
    native.batch_setup(batch, states, qd, opts)
    native.batch_check_status(batch)
    z = torch.zeros_like(qd)
    infos = native.batch_solve(batch, gq, gv, z, opts, raise_noconv=False)
    dq, dv, df = torch.empty_like(qd), torch.empty_like(qd), torch.empty_like(qd)
    grad = torch.zeros(3 * len(cases), dtype=torch.float64, device=dev)
    native.batch_vjp(batch, z, gv, dq, dv, df, grad)
    native.batch_check_status(batch)
    torch.cuda.synchronize()
    voff = batch.voff
    out = {"z": z.cpu().numpy(), "dqbar": dq.cpu().numpy(), "dvbar": dv.cpu().numpy(), "dfext": df.cpu().numpy()}
    g3 = grad.cpu().numpy().reshape(-1, 3)
    batch.close()
    for k, (spec, q, rec) in enumerate(cases):
        v0, v1 = voff[k], voff[k + 1]
        disc = scene_disc(spec)
        sysm = adj.assemble(disc, q, rec, spec.eps)
        zk = out["z"][v0:v1].reshape(-1)
        b = gqs[k].reshape(-1) + gvs[k].reshape(-1) / spec.h
        res = np.linalg.norm(sysm.Acal.T @ zk - b) / np.linalg.norm(b)
        ref = adj.vjp(disc, sysm, q, rec, zk, gvs[k], spec.E, spec.nu)
        errs = {key: rel(out[key][v0:v1], getattr(ref, key)) for key in ("dqbar", "dvbar", "dfext")}
        print(f"box {k}: {spec.n_tets} tets, {rec.contacts.n} contacts, iters {infos[k].iters}, relres "
              f"{infos[k].relres:.1e}, oracle residual {res:.1e}, "
              + ", ".join(f"{key} {e:.1e}" for key, e in errs.items()), flush=True)
        assert infos[k].relres <= 1e-8
        assert res <= 1e-8
        for key, e in errs.items():
            assert e <= 1e-9, (k, key)
        dE_tet, dnu_tet = ref.dE_tet, ref.dnu_tet
        assert abs(g3[k][0] - ref.dE) <= 1e-9 * np.abs(dE_tet).sum()
        assert abs(g3[k][1] - ref.dnu) <= 1e-9 * np.abs(dnu_tet).sum()
        assert abs(g3[k][2] - ref.dmu_fric) <= 1e-9 * max(abs(ref.dmu_fric), 1e-30) + 1e-20
