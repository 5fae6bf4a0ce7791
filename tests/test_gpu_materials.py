"""GPU parity for the as-rigid-as-possible and co-rotational local steps
(App. B.2): on the tiny impact run of each model, the GPU adjoint (single
scene and batched) reaches the oracle's gradients at the FP64 bar, the
assembled matrix matches, and one GPU forward step matches the oracle's
(both started cold)."""

import dataclasses
import functools

import numpy as np
import pytest

from gpu_helpers import contact_tensors, make_scene, rel, run_adjoint, torch_cuda
from oracle import adjoint as adj
from oracle.forward import solve_step
from oracle.rollout import run_forward
from synth import tiny_scene

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9
MATERIALS = ["arap", "corot"]


@functools.lru_cache(maxsize=None)
def _run(material):
    spec = dataclasses.replace(tiny_scene("impact"), material=material)
    return spec, run_forward(spec, steps=16)


@pytest.mark.parametrize("step", [3, 12, 15])
@pytest.mark.parametrize("material", MATERIALS)
def test_adjoint_matches_oracle(material, step):
    torch_cuda()
    spec, ro = _run(material)
    rec, q = ro.records[step], ro.qs[step + 1]
    rng = np.random.default_rng(300 + step)
    gq, gv = rng.standard_normal(q.shape), 1e-3 * rng.standard_normal(q.shape)
    print(f"{material} step {step}: contacts {rec.contacts.n} frictional {int(rec.contacts.fric.sum())}",
          flush=True)
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=64)
    out = run_adjoint(scene, rec, q, gq, gv, want_tet=True)
    errs = {k: rel(out[k], getattr(ref, k)) for k in ("z", "dqbar", "dvbar", "dfext", "dE_tet", "dnu_tet")}
    print(f"  iters {out['info'].iters}, relres {out['info'].relres:.2e}, "
          + ", ".join(f"{k} {e:.1e}" for k, e in errs.items()), flush=True)
    for k, e in errs.items():
        assert e <= TOL_FP64, k
    g = out["grad3"]
    assert abs(g[0] - ref.dE) <= TOL_FP64 * max(abs(ref.dE), np.abs(ref.dE_tet).sum())
    assert abs(g[1] - ref.dnu) <= TOL_FP64 * max(abs(ref.dnu), np.abs(ref.dnu_tet).sum())
    assert abs(g[2] - ref.dmu_fric) <= TOL_FP64 * max(abs(ref.dmu_fric), 1e-30) + 1e-20
    scene.close()


@pytest.mark.parametrize("material", MATERIALS)
def test_assembled_matrix_matches_oracle(material):
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _run(material)
    step = 12
    rec, q = ro.records[step], ro.qs[step + 1]
    ref = adj.assemble(ro.disc, q, rec, spec.eps).Acal.T.toarray()
    scene = make_scene(spec, max_contacts=64)
    run_adjoint(scene, rec, q, np.ones_like(q), np.zeros_like(q))
    val = native.debug_export(scene, 0).reshape(-1, 3, 3)
    rp = native.debug_export(scene, 1)
    col = native.debug_export(scene, 2)
    n = spec.n_verts
    dense = np.zeros((3 * n, 3 * n))
    for r in range(n):
        for p in range(rp[r], rp[r + 1]):
            dense[3 * r:3 * r + 3, 3 * col[p]:3 * col[p] + 3] = val[p]
    e = rel(dense, ref)
    print(f"{material}: assembled matrix err {e:.2e}", flush=True)
    assert e <= 1e-12
    scene.close()


@pytest.mark.parametrize("material", MATERIALS)
def test_batched_adjoint_matches_oracle(material):
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _run(material)
    steps = (12, 15)
    b = native.Batch([(spec.mesh.rest, spec.mesh.tets, spec.E, spec.nu)] * len(steps), spec.density, spec.h,
                     spec.eps, spec.gravity, spec.planes, spec.contact_margin, [64] * len(steps),
                     material=native.MATERIAL_CODES[material])
    keep, css = [], []
    for t in steps:
        tens = contact_tensors(ro.records[t])
        keep.append(tens)
        css.append(native.make_contact_state(ro.records[t].contacts.n, tens["vid"], tens["fric"], tens["frame"],
                                             tens["delta"], tens["lam"], ro.records[t].mu))
    rng = np.random.default_rng(400)
    gq = [rng.standard_normal(ro.qs[t + 1].shape) for t in steps]
    gv = [1e-3 * rng.standard_normal(ro.qs[t + 1].shape) for t in steps]
    dev = "cuda"
    q = torch.tensor(np.concatenate([ro.qs[t + 1] for t in steps]), device=dev)
    gqd = torch.tensor(np.concatenate(gq), device=dev)
    gvd = torch.tensor(np.concatenate(gv), device=dev)
    opts = native.solve_opts(rtol=1e-13, maxit=3000, restart=64)
    native.batch_setup(b, css, q, opts)
    z = torch.zeros_like(gqd)
    infos = native.batch_solve(b, gqd, gvd, z, opts, raise_noconv=False)
    dq, dv, df = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
    grad = torch.zeros(3 * len(steps), dtype=torch.float64, device=dev)
    native.batch_vjp(b, z, gvd, dq, dv, df, grad)
    native.batch_check_status(b)
    torch.cuda.synchronize()
    n = spec.n_verts
    zz = z.cpu().numpy().reshape(-1, 3)
    for k, t in enumerate(steps):
        ref = adj.adjoint_step(ro.disc, ro.qs[t + 1], ro.records[t], gq[k], gv[k], spec.eps, spec.E, spec.nu)
        e = rel(zz[k * n:(k + 1) * n], ref.z)
        print(f"{material} batch scene {k} (step {t}): iters {infos[k].iters}, relres {infos[k].relres:.2e}, "
              f"z err {e:.2e}", flush=True)
        assert infos[k].relres <= 1e-11
        assert e <= TOL_FP64
    b.close()


@pytest.mark.parametrize("material", MATERIALS)
def test_forward_step_matches_oracle(material):
    torch = torch_cuda()
    from paper_2603_16478_amd.rollout import GpuSim
    spec, ro = _run(material)
    step = 12
    q_ref, _, ref, _ = solve_step(ro.disc, ro.qs[step], ro.vs[step], spec.force(step), spec.gravity, spec.mu,
                                  spec.eps, spec.planes, margin=spec.contact_margin)
    sim = GpuSim(spec, max_contacts=64)
    q, v, rec = sim.step(torch.tensor(ro.qs[step], device="cuda"), torch.tensor(ro.vs[step], device="cuda"),
                         torch.tensor(spec.force(step), device="cuda"), spec.mu)
    n = rec.n
    assert n == ref.contacts.n
    np.testing.assert_array_equal(rec.vid[:n].cpu().numpy(), ref.contacts.vid)
    np.testing.assert_array_equal(rec.fric[:n].cpu().numpy().astype(bool), ref.contacts.fric)
    e = rel(q.cpu().numpy() - ro.qs[step], q_ref - ro.qs[step])
    print(f"{material} forward step {step}: contacts {n}, step displacement err {e:.2e}", flush=True)
    assert e <= 1e-7
    if n:
        assert rel(rec.lam[:n].cpu().numpy(), ref.lam) <= 1e-6
