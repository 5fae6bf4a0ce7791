"""GPU parity of the conjugate-gradient path (Sec. 5.4: CG when the adjoint
system is symmetric positive definite).  Frictionless contact (mu = 0, every
contact normal-only) and contact-free steps of the tiny impact scene:
the automatically chosen method must be PCG and its outputs must match the
FP64 oracle at 1e-9, and GMRES forced on the same system must agree."""

import dataclasses
import functools

import numpy as np
import pytest

from gpu_helpers import make_scene, rel, run_adjoint, torch_cuda
from oracle import adjoint as adj
from oracle.rollout import run_forward
from synth import tiny_scene

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


@functools.lru_cache(maxsize=None)
def _frictionless():
    spec = dataclasses.replace(tiny_scene("impact"), mu=0.0)
    return spec, run_forward(spec, steps=20)


@pytest.mark.parametrize("step", [2, 6, 13, 19])
def test_pcg_frictionless_matches_oracle(step):
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _frictionless()
    rec, q = ro.records[step], ro.qs[step + 1]
    rng = np.random.default_rng(300 + step)
    gq = rng.standard_normal(q.shape)
    gv = 1e-3 * rng.standard_normal(q.shape)
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=64)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, want_tet=True)
    info = out["info"]
    print(f"pcg step {step}: contacts {rec.contacts.n}, iters {info.iters}, relres {info.relres:.2e}, "
          f"z err {rel(out['z'], ref.z):.2e}", flush=True)
    assert info.method == native.ADJ_PCG
    for k in ("z", "dqbar", "dvbar", "dfext", "dE_tet", "dnu_tet"):
        assert rel(out[k], getattr(ref, k)) <= TOL_FP64, k
    g = out["grad3"]
    assert abs(g[0] - ref.dE) <= TOL_FP64 * np.abs(ref.dE_tet).sum()
    assert abs(g[1] - ref.dnu) <= TOL_FP64 * np.abs(ref.dnu_tet).sum()
    gm = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, method=native.ADJ_GMRES)
    assert gm["info"].method == native.ADJ_GMRES
    assert rel(gm["z"], out["z"]) <= TOL_FP64


def test_pcg_rejected_on_frictional_system():
    """Forcing PCG on a frictional (non-symmetric) system is an argument error."""
    torch_cuda()
    from paper_2603_16478_amd import native
    spec = tiny_scene("impact")
    ro = run_forward(spec, steps=12)
    rec, q = ro.records[10], ro.qs[11]
    assert rec.contacts.fric.any() and rec.mu > 0
    scene = make_scene(spec, max_contacts=64)
    with pytest.raises(native.AdjError):
        run_adjoint(scene, rec, q, np.ones_like(q), np.zeros_like(q), method=native.ADJ_PCG)


@pytest.mark.parametrize("prec_name", ["ADJ_MIXED", "ADJ_MIXED_PC"])
def test_pcg_mixed_precision_matches_oracle(prec_name):
    """Mixed precision with PCG inside the FP64 refinement loop: 1e-4
    (PCG takes ADJ_MIXED_PC as ADJ_MIXED)."""
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _frictionless()
    step = 13
    rec, q = ro.records[step], ro.qs[step + 1]
    gq = np.random.default_rng(7).standard_normal(q.shape)
    gv = np.zeros_like(q)
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=64)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, prec=getattr(native, prec_name))
    print(f"pcg mixed: iters {out['info'].iters}, refine {out['info'].refine_steps}, "
          f"z err {rel(out['z'], ref.z):.2e}", flush=True)
    assert out["info"].method == native.ADJ_PCG
    assert rel(out["z"], ref.z) <= 1e-4
    assert rel(out["dqbar"], ref.dqbar) <= 1e-4
