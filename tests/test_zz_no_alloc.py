"""The allocation-free gradient contraction (vjp_params_noalloc) through the
C ABI against vjp_params, bit for bit, on two calls in a row on two scenes,
the second smaller: the beam with its ground contacts, then the tiny cube."""

import numpy as np
import pytest

from gpu_helpers import contact_tensors, make_scene, torch_cuda

pytestmark = pytest.mark.gpu


def _beam():
    import os
    from conftest import ROOT
    from oracle.contact import ContactSet
    from oracle.forward import StepRecord
    from synth import beam_scene
    d = np.load(os.path.join(ROOT, "tests", "golden", "beam_states_mu0.4.npz"))
    t = 3
    cs = ContactSet(d[f"vid{t}"], d[f"collider{t}"], d[f"frame{t}"], d[f"d_n{t}"], d[f"d_f{t}"],
                    d[f"fric{t}"].astype(bool))
    return beam_scene(mu=0.4), d[f"q{t}"], StepRecord(cs, d[f"delta{t}"], d[f"lam{t}"], 0.4)


def _tiny():
    from oracle.rollout import run_forward
    from synth import tiny_scene
    spec = tiny_scene("impact")
    ro = run_forward(spec, steps=12)
    return spec, ro.qs[12], ro.records[11]


def _both(spec, q, rec):
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    scene = make_scene(spec, max_contacts=max(1, rec.contacts.n))
    tens = contact_tensors(rec)
    cs = native.make_contact_state(rec.contacts.n, tens["vid"], tens["fric"], tens["frame"], tens["delta"],
                                   tens["lam"], rec.mu)
    qd = torch.tensor(q, device="cuda")
    rng = np.random.default_rng(11)
    gq = torch.tensor(rng.standard_normal(q.shape), device="cuda")
    gv = torch.tensor(1e-3 * rng.standard_normal(q.shape), device="cuda")
    z = torch.zeros_like(qd)
    opts = native.solve_opts(rtol=1e-10, maxit=2000)
    native.adjoint_setup(scene, cs, qd, opts)
    native.adjoint_solve(scene, gq, gv, z, opts)
    outs = []
    for fn in (native.vjp_params, native.vjp_params_noalloc):
        o = {k: torch.full_like(qd, np.nan) for k in ("dqbar", "dvbar", "dfext")}
        o["grad3"] = torch.zeros(3, dtype=torch.float64, device="cuda")
        o["dE"] = torch.zeros(spec.n_tets, dtype=torch.float64, device="cuda")
        o["dnu"] = torch.zeros(spec.n_tets, dtype=torch.float64, device="cuda")
        fn(scene, z, gv, o["dqbar"], o["dvbar"], o["dfext"], o["grad3"], o["dE"], o["dnu"])
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in o.items()})
    scene.close()
    return outs


def test_noalloc_vjp_equals_vjp_params_on_two_calls():
    for spec, q, rec in (_beam(), _tiny()):
        ref, got = _both(spec, q, rec)
        print(f"{spec.name}: {spec.n_tets} tets, {rec.contacts.n} contacts, grad3 {got['grad3']}", flush=True)
        assert np.all(np.isfinite(got["grad3"])) and np.any(got["grad3"] != 0.0)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
