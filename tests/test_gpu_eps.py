"""The smoothing parameter on the GPU path (Sec. 5.2; Sec. 6, smoothing
parameter sensitivity; the appendix on forward-backward smoothing
consistency), on the slope cube.

* Forward parity: one GPU step from the oracle's state after ten steps
  matches the oracle's step (both started cold) at 2 eps^2 from 1e-15 to
  1e-6, sliding and sticking.
* Backward parity with the smoothing matched and mismatched (the scene's eps
  is the backward's): the GPU adjoint reaches the oracle's at the same eps_b
  at the FP64 bar in both cases, and a mismatched backward moves the
  sticking cube's dL/dmu to the sliding cube's scale.
* A one-second sweep on the GPU forward: at 2 eps^2 = 1e-12 the sliding cube
  outruns the sticking one many times over; at 1e-6 the two move alike.
"""

import dataclasses
import functools

import numpy as np
import pytest

from gpu_helpers import make_scene, rel, run_adjoint, torch_cuda
from oracle import adjoint as adj
from oracle.forward import solve_step
from oracle.rollout import scene_disc
from synth import slope_scene

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


@functools.lru_cache(maxsize=None)
def _oracle_run(side, two_eps2, steps):
    spec = slope_scene(side, two_eps2)
    disc = scene_disc(spec)
    q, v, warm = spec.q0.copy(), spec.v0.copy(), None
    for _ in range(steps):
        q, v, rec, warm = solve_step(disc, q, v, np.zeros_like(q), spec.gravity, spec.mu, spec.eps, spec.planes,
                                     margin=spec.contact_margin, warm=warm)
    return spec, disc, q, v, warm


@pytest.mark.parametrize("side", ["slip", "stick"])
@pytest.mark.parametrize("two_eps2", [1e-15, 1e-12, 1e-9, 1e-6])
def test_forward_step_matches_oracle(two_eps2, side):
    torch = torch_cuda()
    from paper_2603_16478_amd.rollout import GpuSim
    spec, disc, qbar, vbar, _ = _oracle_run(side, two_eps2, 10)
    q_ref, _, ref, _ = solve_step(disc, qbar, vbar, np.zeros_like(qbar), spec.gravity, spec.mu, spec.eps,
                                  spec.planes, margin=spec.contact_margin)
    sim = GpuSim(spec, max_contacts=64)
    print(f"slope {side}, 2eps^2 {two_eps2:g}: one step from the oracle's step-10 state", flush=True)
    q, v, rec = sim.step(torch.tensor(qbar, device="cuda"), torch.tensor(vbar, device="cuda"),
                         torch.zeros(qbar.shape, dtype=torch.float64, device="cuda"), spec.mu)
    n = rec.n
    assert n == ref.contacts.n
    np.testing.assert_array_equal(rec.vid[:n].cpu().numpy(), ref.contacts.vid)
    np.testing.assert_array_equal(rec.fric[:n].cpu().numpy().astype(bool), ref.contacts.fric)
    du, du_ref = q.cpu().numpy() - qbar, q_ref - qbar
    e_q, e_l = rel(du, du_ref), rel(rec.lam[:n].cpu().numpy(), ref.lam)
    print(f"  contacts {n}, step displacement err {e_q:.2e}, multiplier err {e_l:.2e}", flush=True)
    assert e_q <= 1e-7
    assert e_l <= 1e-6


def test_mismatched_smoothing_parity_and_regime_contrast():
    torch_cuda()
    dmu = {}
    for side in ("stick", "slip"):
        spec, disc, qbar, vbar, warm = _oracle_run(side, 1e-12, 30)
        q, v, rec, _ = solve_step(disc, qbar, vbar, np.zeros_like(qbar), spec.gravity, spec.mu, spec.eps,
                                  spec.planes, margin=spec.contact_margin, warm=warm)
        rng = np.random.default_rng(41)
        gq, gv = spec.loss_dir, 1e-3 * rng.standard_normal(q.shape)
        for k in (1.0, 1000.0):
            spec_b = dataclasses.replace(spec, eps=k * spec.eps)
            ref = adj.adjoint_step(disc, q, rec, gq, gv, spec_b.eps, spec.E, spec.nu)
            scene = make_scene(spec_b, max_contacts=64)
            # the contact rows' stiffness (~1/eps^2) puts the FP64 floor of the
            # relative residual near 3e-11 (sticking) and 2e-9 (sliding); z is
            # accurate well below that
            out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-10, maxit=1000, raise_noconv=False)
            info = out["info"]
            errs = {key: rel(out[key], getattr(ref, key)) for key in ("z", "dqbar", "dvbar", "dfext")}
            e_mu = abs(out["grad3"][2] - ref.dmu_fric) / abs(ref.dmu_fric)
            print(f"{side}, eps_b = {k:g} eps_f: iters {info.iters}, relres {info.relres:.2e}, "
                  f"errs {', '.join(f'{a} {b:.1e}' for a, b in errs.items())}, dL/dmu {out['grad3'][2]:.6e} "
                  f"(oracle {ref.dmu_fric:.6e})", flush=True)
            assert info.relres <= 1e-8
            for key, e in errs.items():
                assert e <= TOL_FP64, key
            assert e_mu <= TOL_FP64
            dmu[side, k] = out["grad3"][2]
            scene.close()
    assert abs(dmu["stick", 1.0]) < 0.05 * abs(dmu["slip", 1.0])
    assert abs(dmu["stick", 1000.0]) > 0.5 * abs(dmu["slip", 1000.0])


def test_one_second_sweep_on_gpu_forward():
    torch = torch_cuda()
    from paper_2603_16478_amd.rollout import GpuSim
    ratio = {}
    for two_eps2 in (1e-12, 1e-6):
        disp = {}
        for side in ("slip", "stick"):
            spec = slope_scene(side, two_eps2)
            sim = GpuSim(spec, max_contacts=64)
            q = torch.tensor(spec.q0, device="cuda")
            v = torch.tensor(spec.v0, device="cuda")
            f = torch.zeros_like(q)
            steps = int(round(1.0 / spec.h))
            print(f"sweep {side} 2eps^2 {two_eps2:g}: {steps} steps", flush=True)
            for _ in range(steps):
                q, v, _ = sim.step(q, v, f, spec.mu)
            disp[side] = float((q[:, 0] - torch.tensor(spec.q0[:, 0], device="cuda")).mean())
        ratio[two_eps2] = disp["slip"] / disp["stick"]
        print(f"2eps^2 {two_eps2:g}: slip {disp['slip']:.4e} m, stick {disp['stick']:.4e} m, "
              f"ratio {ratio[two_eps2]:.2f}", flush=True)
    assert ratio[1e-12] > 10.0
    assert ratio[1e-6] < 1.5
