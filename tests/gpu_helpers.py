"""Helpers for the GPU parity tests: move oracle inputs to the device and run
the C-ABI adjoint.  Inputs come from the oracle or from synth; nothing here
computes the method."""

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no HIP device")
    return torch


def make_scene(spec, max_contacts):
    from paper_2603_16478_amd import native
    return native.Scene(spec.mesh.rest, spec.mesh.tets, spec.density, spec.h, spec.eps, spec.E, spec.nu,
                        spec.gravity, spec.planes, spec.contact_margin, max_contacts,
                        material=native.MATERIAL_CODES[spec.material])


def contact_tensors(record, device="cuda"):
    torch = torch_cuda()
    cs = record.contacts
    n = cs.n
    dev = dict(device=device)
    t = {
        "vid": torch.tensor(cs.vid.astype(np.int32), dtype=torch.int32, **dev),
        "fric": torch.tensor(cs.fric.astype(np.int32), dtype=torch.int32, **dev),
        "frame": torch.tensor(cs.frame.reshape(n, 9), dtype=torch.float64, **dev),
        "delta": torch.tensor(record.delta.reshape(n, 3), dtype=torch.float64, **dev),
        "lam": torch.tensor(record.lam.reshape(n, 3), dtype=torch.float64, **dev),
    }
    if n == 0:
        t = {k: torch.zeros(1, dtype=v.dtype, **dev) for k, v in t.items()}
    return t


def run_adjoint(scene, record, q, gq, gv, rtol=1e-13, maxit=3000, restart=64, want_tet=False,
                raise_noconv=True, method=0, prec=0, precond=0, check=True):
    """setup + solve + vjp on the GPU; returns a dict of numpy results."""
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    dev = "cuda"
    tens = contact_tensors(record)
    cs = native.make_contact_state(record.contacts.n, tens["vid"], tens["fric"], tens["frame"],
                                   tens["delta"], tens["lam"], record.mu)
    qd = torch.tensor(np.ascontiguousarray(q), dtype=torch.float64, device=dev)
    gqd = torch.tensor(np.ascontiguousarray(gq), dtype=torch.float64, device=dev)
    gvd = torch.tensor(np.ascontiguousarray(gv), dtype=torch.float64, device=dev)
    z = torch.zeros_like(qd)
    opts = native.solve_opts(rtol=rtol, maxit=maxit, restart=restart, method=method, prec=prec, precond=precond)
    native.adjoint_setup(scene, cs, qd, opts)
    if check:
        native.check_status(scene)
    info = native.adjoint_solve(scene, gqd, gvd, z, opts, raise_noconv=raise_noconv)
    dqbar, dvbar, dfext = torch.empty_like(qd), torch.empty_like(qd), torch.empty_like(qd)
    grad3 = torch.zeros(3, dtype=torch.float64, device=dev)
    nt = scene.n_tets
    dE = torch.zeros(nt, dtype=torch.float64, device=dev) if want_tet else None
    dnu = torch.zeros(nt, dtype=torch.float64, device=dev) if want_tet else None
    native.vjp_params(scene, z, gvd, dqbar, dvbar, dfext, grad3, dE, dnu)
    torch.cuda.synchronize()
    out = {"z": z.cpu().numpy(), "dqbar": dqbar.cpu().numpy(), "dvbar": dvbar.cpu().numpy(),
           "dfext": dfext.cpu().numpy(), "grad3": grad3.cpu().numpy(), "info": info}
    if want_tet:
        out["dE_tet"] = dE.cpu().numpy()
        out["dnu_tet"] = dnu.cpu().numpy()
    out["_keep"] = (tens, cs, qd)
    return out


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel_entries(a, b, floor=1e-3):
    """Largest per-entry relative error |a_i - b_i| / |b_i|, each entry's
    scale floored at `floor` times the largest |b|: small entries are held to
    their own size down to that floor, not to the largest entry's."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    scale = np.maximum(np.abs(b), floor * max(np.max(np.abs(b)), 1e-300))
    return float(np.max(np.abs(a - b) / scale))
