"""Status codes of the C ABI on its error paths (inputs the host or the
kernels' own checks turn into errors; every kernel still exits normally):
an iteration cap too small to converge, an inverted element in the
linearisation state, a non-finite right-hand side, and the clearing of the
device error flag by the next setup."""

import functools

import numpy as np
import pytest

from gpu_helpers import contact_tensors, make_scene, rel, run_adjoint, torch_cuda
from oracle import adjoint as adj
from oracle.rollout import run_forward
from synth import tiny_scene

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _impact():
    spec = tiny_scene("impact")
    ro = run_forward(spec, steps=12)
    return spec, ro


def _rhs(q, seed=3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(q.shape), 1e-3 * rng.standard_normal(q.shape)


def _flipped(spec, q):
    """q with the last vertex of tet 0 reflected through the plane of the
    other three: that tet has det F < 0."""
    a, b, c, d = spec.mesh.tets[0]
    q = q.copy()
    n = np.cross(q[b] - q[a], q[c] - q[a])
    n /= np.linalg.norm(n)
    q[d] = q[d] - 2.0 * np.dot(q[d] - q[a], n) * n
    return q


def _status_of(fn):
    from paper_2603_16478_amd import native
    try:
        fn()
    except native.AdjError as e:
        return native.STATUS[e.status]
    return "ADJ_OK"


def test_iteration_cap_reports_noconv():
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _impact()
    rec, q = ro.records[10], ro.qs[11]
    gq, gv = _rhs(q)
    scene = make_scene(spec, max_contacts=64)
    st = _status_of(lambda: run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, maxit=1))
    assert st == "ADJ_E_NOCONV"
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, maxit=1, raise_noconv=False)
    assert out["info"].relres > 1e-13 and np.all(np.isfinite(out["z"]))
    # the scene stays usable: the same step converges with the default cap
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    assert rel(run_adjoint(scene, rec, q, gq, gv)["z"], ref.z) <= 1e-9
    assert native.STATUS[native.load().adj_check_status(scene.handle, None)] == "ADJ_OK"
    scene.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_inverted_element_is_reported_and_cleared_by_the_next_setup(prec):
    torch_cuda()
    spec, ro = _impact()
    rec, q = ro.records[10], ro.qs[11]
    gq, gv = _rhs(q)
    scene = make_scene(spec, max_contacts=64)
    bad = _flipped(spec, q)
    st = _status_of(lambda: run_adjoint(scene, rec, bad, gq, gv, rtol=1e-8, prec=prec, check=False))
    assert st == "ADJ_E_INVERTED"
    # a setup at a valid state clears the flag: the solve succeeds and agrees with the oracle
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13 if prec == 0 else 1e-10, prec=prec)
    assert rel(out["z"], ref.z) <= (1e-9 if prec == 0 else 1e-4)
    scene.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_non_finite_right_hand_side_is_an_argument_error(prec):
    torch_cuda()
    spec, ro = _impact()
    rec, q = ro.records[10], ro.qs[11]
    gq, gv = _rhs(q)
    gq[7, 1] = np.nan
    scene = make_scene(spec, max_contacts=64)
    st = _status_of(lambda: run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, prec=prec, check=False))
    assert st == "ADJ_E_ARG"
    scene.close()


def test_batch_inverted_scene_is_reported_and_cleared():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _impact()
    recs = [ro.records[9], ro.records[10]]
    qs = [ro.qs[10], ro.qs[11]]
    batch = native.Batch([(spec.mesh.rest, spec.mesh.tets, spec.E, spec.nu)] * 2, spec.density, spec.h, spec.eps,
                         spec.gravity, spec.planes, spec.contact_margin, [64, 64])
    dev = "cuda"
    opts = native.solve_opts(rtol=1e-12, maxit=2000)

    def run(qs_):
        tens = [contact_tensors(r) for r in recs]
        cst = [native.make_contact_state(r.contacts.n, t["vid"], t["fric"], t["frame"], t["delta"], t["lam"],
                                         r.mu) for r, t in zip(recs, tens)]
        qd = torch.tensor(np.concatenate(qs_), device=dev)
        gq = torch.tensor(np.concatenate([_rhs(x)[0] for x in qs_]), device=dev)
        gv = torch.zeros_like(gq)
        z = torch.zeros_like(gq)
        native.batch_setup(batch, cst, qd, opts)
        native.batch_solve(batch, gq, gv, z, opts)
        torch.cuda.synchronize()
        return z.cpu().numpy(), (tens, cst, qd)

    st = _status_of(lambda: run([qs[0], _flipped(spec, qs[1])]))
    assert st == "ADJ_E_INVERTED"
    z, _ = run(qs)
    n = spec.n_verts
    for k in range(2):
        ref = adj.adjoint_step(ro.disc, qs[k], recs[k], _rhs(qs[k])[0], np.zeros_like(qs[k]), spec.eps, spec.E,
                               spec.nu)
        assert rel(z[k * n:(k + 1) * n], ref.z) <= 1e-9
    batch.close()
