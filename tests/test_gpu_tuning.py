"""Launch-shape tuning and the autotuner: every tuning gives the same
adjoint (to rounding of the reordered sums) as the default, graph replay of
the Krylov chunks included, and the autotuner returns a member of the
supported set."""

import numpy as np
import pytest

from gpu_helpers import contact_tensors, make_scene, rel, torch_cuda
from oracle import adjoint as adj

pytestmark = pytest.mark.gpu


def _beam(mu=0.4, t=3):
    import os
    from conftest import ROOT
    from oracle.contact import ContactSet
    from oracle.forward import StepRecord
    from synth import beam_scene
    path = os.path.join(ROOT, "tests", "golden", f"beam_states_mu{mu}.npz")
    if not os.path.exists(path):
        pytest.skip(f"missing fixture {path}")
    d = np.load(path)
    cs = ContactSet(d[f"vid{t}"], d[f"collider{t}"], d[f"frame{t}"], d[f"d_n{t}"], d[f"d_f{t}"],
                    d[f"fric{t}"].astype(bool))
    return beam_scene(mu=mu), d[f"q{t}"], StepRecord(cs, d[f"delta{t}"], d[f"lam{t}"], mu)


TUNINGS = [dict(gs_rows=64, bsr_lanes=16, chunk=8, graph=0, gj_wide_min=2048, a_inv=0, lu_min=4608, lu_pipe=1,
                sweep_fuse=0),
           dict(gs_rows=128, bsr_lanes=8, chunk=4, graph=0, gj_wide_min=2048, a_inv=2, lu_min=128, lu_pipe=1,
                sweep_fuse=0),
           dict(gs_rows=128, bsr_lanes=8, chunk=4, graph=0, gj_wide_min=2048, a_inv=2, lu_min=128, lu_pipe=0,
                sweep_fuse=3),
           dict(gs_rows=128, bsr_lanes=8, chunk=4, graph=0, gj_wide_min=2048, a_inv=2, lu_min=4608, lu_pipe=1,
                sweep_fuse=64),
           dict(gs_rows=256, bsr_lanes=32, chunk=16, graph=0, gj_wide_min=128, a_inv=1, lu_min=4608, lu_pipe=1,
                sweep_fuse=-1),
           dict(gs_rows=64, bsr_lanes=4, chunk=8, graph=1, gj_wide_min=2048, a_inv=2, lu_min=128, lu_pipe=1,
                sweep_fuse=5),
           dict(gs_rows=128, bsr_lanes=16, chunk=32, graph=1, gj_wide_min=128, a_inv=0, lu_min=4608, lu_pipe=0,
                sweep_fuse=-1)]


def test_tunings_agree_with_oracle():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    spec, q, rec = _beam()
    from oracle.rollout import scene_disc
    ref = adj.adjoint_step(scene_disc(spec), q, rec, spec.loss_dir, np.zeros_like(q), spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=rec.contacts.n)
    tens = contact_tensors(rec)
    cs = native.make_contact_state(rec.contacts.n, tens["vid"], tens["fric"], tens["frame"], tens["delta"],
                                   tens["lam"], rec.mu)
    qd = torch.tensor(q, device="cuda")
    gq = torch.tensor(spec.loss_dir, device="cuda")
    gv = torch.zeros_like(gq)
    opts = native.solve_opts(rtol=1e-12, maxit=2000)
    for t in TUNINGS:
        native.set_tuning(scene, **t)
        assert native.get_tuning(scene) == t
        native.adjoint_setup(scene, cs, qd, opts)
        for rep in range(3):  # graph mode: capture on the first solve, replay after
            z = torch.zeros_like(gq)
            info = native.adjoint_solve(scene, gq, gv, z, opts)
            err = rel(z.cpu().numpy(), ref.z)
            print(f"tuning {t} rep {rep}: iters {info.iters}, z err {err:.2e}", flush=True)
            assert err <= 1e-9


def test_autotune_returns_supported_shape():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    spec, q, rec = _beam()
    scene = make_scene(spec, max_contacts=rec.contacts.n)
    tens = contact_tensors(rec)
    cs = native.make_contact_state(rec.contacts.n, tens["vid"], tens["fric"], tens["frame"], tens["delta"],
                                   tens["lam"], rec.mu)
    qd = torch.tensor(q, device="cuda")
    gq = torch.tensor(spec.loss_dir, device="cuda")
    gv = torch.zeros_like(gq)
    z = torch.zeros_like(gq)
    opts = native.solve_opts(rtol=1e-8, maxit=2000)
    native.adjoint_setup(scene, cs, qd, opts)
    best = native.autotune(scene, gq, gv, z, opts, reps=2)
    print("autotuned", best, flush=True)
    assert best["gs_rows"] in (64, 128, 256) and best["bsr_lanes"] in (4, 8, 16, 32)
    assert 1 <= best["chunk"] <= 64 and best["graph"] in (0, 1) and best["a_inv"] in (0, 1, 2)
    assert native.get_tuning(scene) == best
    with pytest.raises(native.AdjError):
        native.set_tuning(scene, gs_rows=96)
