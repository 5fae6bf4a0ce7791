"""The batched workload over its full range of scene sizes: the first 16
boxes of the seeded 256-box set (2,058 to 97,650 tets, 69,590 vertices in
all; two hover above the ground), each at a seeded deformed state with the
ground contacts the detection finds there and seeded sticking contact
values, solved as one batch (the Woodbury correction goes through S^T S of
the union at this size).  Compared element by element with the oracle's
adjoint solutions stored in tests/golden/boxes16_z.npz (written by
tests/golden/make_oracle_z.py): z in FP64 at 1e-9 and in mixed precision at
1e-4, and the gradient contractions against the oracle's contractions of
its own z."""

import os
import sys

import numpy as np
import pytest

from conftest import ROOT
from gpu_helpers import contact_tensors, rel, torch_cuda
from oracle import adjoint as adj
from oracle.rollout import scene_disc

sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
from make_oracle_z import boxes_cases  # noqa: E402

pytestmark = pytest.mark.gpu


def test_batched_boxes_full_range_against_stored_oracle():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    d = np.load(os.path.join(ROOT, "tests", "golden", "boxes16_z.npz"))
    cases = boxes_cases(16)
    specs = [c[0] for c in cases]
    s0 = specs[0]
    print(f"{len(specs)} boxes, {sum(s.n_tets for s in specs)} tets, {sum(s.n_verts for s in specs)} vertices, "
          f"contacts {[c[2].contacts.n for c in cases]}; building the batch", flush=True)
    batch = native.Batch([(s.mesh.rest, s.mesh.tets, s.E, s.nu) for s in specs], s0.density, s0.h, s0.eps,
                         s0.gravity, s0.planes, s0.contact_margin, [max(1, c[2].contacts.n) for c in cases])
    assert list(batch.voff) == list(d["voff"])
    keep, states = [], []
    for spec, q, rec, _, _ in cases:
        tens = contact_tensors(rec)
        keep.append(tens)
        states.append(native.make_contact_state(rec.contacts.n, tens["vid"], tens["fric"], tens["frame"],
                                                tens["delta"], tens["lam"], rec.mu))
    dev = "cuda"
    qd = torch.tensor(np.concatenate([c[1] for c in cases]), device=dev)
    gq = torch.tensor(np.concatenate([c[3] for c in cases]), device=dev)
    gv = torch.tensor(np.concatenate([c[4] for c in cases]), device=dev)
    outs = {}
    for prec in (native.ADJ_FP64, native.ADJ_MIXED):
        opts = native.solve_opts(rtol=1e-12 if prec == native.ADJ_FP64 else 1e-8, maxit=1000, restart=64,
                                 prec=prec, max_refine=8, precond=native.PRECOND_WOODBURY_NO_Z)
        native.batch_setup(batch, states, qd, opts)
        z = torch.zeros_like(qd)
        infos = native.batch_solve(batch, gq, gv, z, opts, raise_noconv=False)
        dq, dv, df = torch.empty_like(qd), torch.empty_like(qd), torch.empty_like(qd)
        grad = torch.zeros(3 * len(cases), dtype=torch.float64, device=dev)
        native.batch_vjp(batch, z, gv, dq, dv, df, grad)
        native.batch_check_status(batch)
        torch.cuda.synchronize()
        outs[prec] = ({"z": z.cpu().numpy(), "dqbar": dq.cpu().numpy(), "dvbar": dv.cpu().numpy(),
                       "dfext": df.cpu().numpy()}, grad.cpu().numpy().reshape(-1, 3), infos)
    voff = batch.voff
    batch.close()
    zref_all = d["z"]
    for k, (spec, q, rec, gqk, gvk) in enumerate(cases):
        v0, v1 = voff[k], voff[k + 1]
        zref = zref_all[v0:v1]
        disc = scene_disc(spec)
        sysm = adj.assemble(disc, q, rec, spec.eps)
        ref = adj.vjp(disc, sysm, q, rec, zref.reshape(-1), gvk, spec.E, spec.nu)
        for prec, bar in ((native.ADJ_FP64, 1e-9), (native.ADJ_MIXED, 1e-4)):
            out, g3, infos = outs[prec]
            errs = {"z": rel(out["z"][v0:v1], zref)}
            errs |= {key: rel(out[key][v0:v1], getattr(ref, key)) for key in ("dqbar", "dvbar", "dfext")}
            errs["dE"] = abs(g3[k][0] - ref.dE) / max(np.abs(ref.dE_tet).sum(), 1e-300)
            errs["dnu"] = abs(g3[k][1] - ref.dnu) / max(np.abs(ref.dnu_tet).sum(), 1e-300)
            if rec.contacts.n:
                errs["dmu"] = abs(g3[k][2] - ref.dmu_fric) / max(abs(ref.dmu_fric), 1e-300)
            print(f"box {k} prec {prec}: {spec.n_tets} tets, {rec.contacts.n} contacts, iters {infos[k].iters}, "
                  f"relres {infos[k].relres:.1e}, " + ", ".join(f"{key} {e:.1e}" for key, e in errs.items()),
                  flush=True)
            assert infos[k].relres <= 1e-8
            for key, e in errs.items():
                assert e <= bar, (k, prec, key, e)
