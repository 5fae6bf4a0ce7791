"""The backward-solver comparison of Sec. 6.2: the Krylov solve with the
sparse inverse alone (S^T S, contact blocks left to the Krylov method), block
Jacobi (3x3 diagonal blocks of Acal^T) or point Jacobi as the
preconditioner must reach the oracle's adjoint on contact-free (PCG and
GMRES) and frictionless (PCG) steps of the tiny impact scene; on a
frictional beam state the Woodbury preconditioner needs the fewest
iterations.  The semi-implicit fixed-point iteration converges to the
oracle's adjoint without contact and diverges with frictional contact.  A
batch refuses the comparison preconditioners."""

import dataclasses
import functools
import os

import numpy as np
import pytest

from gpu_helpers import make_scene, rel, run_adjoint, torch_cuda
from oracle import adjoint as adj
from oracle.rollout import run_forward, scene_disc
from synth import beam_scene, tiny_scene

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


@functools.lru_cache(maxsize=None)
def _beam(mu=0.4, t=3):
    from conftest import ROOT
    from oracle.contact import ContactSet
    from oracle.forward import StepRecord
    path = os.path.join(ROOT, "tests", "golden", f"beam_states_mu{mu}.npz")
    if not os.path.exists(path):
        pytest.skip(f"missing fixture {path}")
    d = np.load(path)
    cs = ContactSet(d[f"vid{t}"], d[f"collider{t}"], d[f"frame{t}"], d[f"d_n{t}"], d[f"d_f{t}"],
                    d[f"fric{t}"].astype(bool))
    spec = beam_scene(mu=mu)
    return spec, scene_disc(spec), d[f"q{t}"], StepRecord(cs, d[f"delta{t}"], d[f"lam{t}"], mu)


@pytest.mark.parametrize("precond", [1, 2, 3])
def test_woodbury_beats_comparison_preconditioners_on_beam(precond):
    """Frictional beam state: the Woodbury preconditioner needs fewer GMRES
    iterations than each comparison preconditioner (with the sparse inverse
    alone the stiff contact directions are outlier eigenvalues and GMRES(64)
    stalls within the budget)."""
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, disc, q, rec = _beam()
    rng = np.random.default_rng(500 + precond)
    gq, gv = spec.loss_dir, 1e-3 * rng.standard_normal(q.shape)
    scene = make_scene(spec, max_contacts=rec.contacts.n)
    print(f"beam, precond {precond}", flush=True)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, maxit=2000, precond=precond, raise_noconv=False)
    wb = run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, maxit=2000, precond=native.PRECOND_WOODBURY)
    print(f"beam precond {precond}: iters {out['info'].iters} relres {out['info'].relres:.2e}; Woodbury iters "
          f"{wb['info'].iters} relres {wb['info'].relres:.2e}", flush=True)
    assert wb["info"].relres <= 1e-8
    assert wb["info"].iters < out["info"].iters


def _contact_free():
    spec = tiny_scene("impact")
    return spec, run_forward(spec, steps=5)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precond", [1, 2, 3])
def test_comparison_preconditioners_contact_free(precond, method):
    """Contact-free tiny step: PCG (chosen automatically) and GMRES (forced)
    with either comparison preconditioner reach the oracle's adjoint."""
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _contact_free()
    rec, q = ro.records[3], ro.qs[4]
    assert rec.contacts.n == 0
    rng = np.random.default_rng(700 + precond)
    gq, gv = rng.standard_normal(q.shape), 1e-3 * rng.standard_normal(q.shape)
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=64)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, maxit=5000, precond=precond, method=method)
    info = out["info"]
    print(f"contact-free precond {precond} method {info.method}: iters {info.iters}, "
          f"z err {rel(out['z'], ref.z):.2e}", flush=True)
    assert info.method == (native.ADJ_PCG if method == 0 else native.ADJ_GMRES)
    for k in ("z", "dqbar", "dvbar", "dfext"):
        assert rel(out[k], getattr(ref, k)) <= TOL_FP64, k


@functools.lru_cache(maxsize=None)
def _frictionless():
    spec = dataclasses.replace(tiny_scene("impact"), mu=0.0)
    return spec, run_forward(spec, steps=14)


@pytest.mark.parametrize("precond", [1, 2, 3])
def test_comparison_preconditioners_tiny_pcg(precond):
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _frictionless()
    rec, q = ro.records[13], ro.qs[14]
    rng = np.random.default_rng(600 + precond)
    gq, gv = rng.standard_normal(q.shape), 1e-3 * rng.standard_normal(q.shape)
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=64)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, maxit=20000, precond=precond)
    info = out["info"]
    print(f"tiny precond {precond}: contacts {rec.contacts.n}, method {info.method}, iters {info.iters}, "
          f"z err {rel(out['z'], ref.z):.2e}", flush=True)
    assert info.method == native.ADJ_PCG
    for k in ("z", "dqbar", "dvbar", "dfext"):
        assert rel(out[k], getattr(ref, k)) <= TOL_FP64, k


def test_semi_implicit_contact_free_matches_oracle():
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, ro = _contact_free()
    rec, q = ro.records[3], ro.qs[4]
    rng = np.random.default_rng(800)
    gq, gv = rng.standard_normal(q.shape), 1e-3 * rng.standard_normal(q.shape)
    ref = adj.adjoint_step(ro.disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=64)
    out = run_adjoint(scene, rec, q, gq, gv, rtol=1e-13, maxit=5000, precond=native.PRECOND_SPARSE_INVERSE,
                      method=native.ADJ_SEMI_IMPLICIT)
    info = out["info"]
    print(f"semi-implicit contact-free: iters {info.iters}, relres {info.relres:.2e}, "
          f"z err {rel(out['z'], ref.z):.2e}", flush=True)
    assert info.method == native.ADJ_SEMI_IMPLICIT
    for k in ("z", "dqbar", "dvbar", "dfext"):
        assert rel(out[k], getattr(ref, k)) <= TOL_FP64, k


def test_semi_implicit_diverges_with_frictional_contact():
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, disc, q, rec = _beam()
    scene = make_scene(spec, max_contacts=rec.contacts.n)
    out = run_adjoint(scene, rec, q, spec.loss_dir, np.zeros_like(q), rtol=1e-8, maxit=2000,
                      precond=native.PRECOND_SPARSE_INVERSE, method=native.ADJ_SEMI_IMPLICIT, raise_noconv=False)
    info = out["info"]
    print(f"semi-implicit beam: iters {info.iters}, relres {info.relres:.2e}", flush=True)
    assert info.relres > 1.0


def test_batch_refuses_comparison_preconditioners():
    torch = torch_cuda()
    from gpu_helpers import contact_tensors
    from paper_2603_16478_amd import native
    spec, disc, q, rec = _beam()
    b = native.Batch([(spec.mesh.rest, spec.mesh.tets, spec.E, spec.nu)], spec.density, spec.h, spec.eps,
                     spec.gravity, spec.planes, spec.contact_margin, [rec.contacts.n])
    tens = contact_tensors(rec)
    cs = native.make_contact_state(rec.contacts.n, tens["vid"], tens["fric"], tens["frame"], tens["delta"],
                                   tens["lam"], rec.mu)
    qd = torch.tensor(q, device="cuda")
    native.batch_setup(b, [cs], qd, native.solve_opts())
    z = torch.zeros_like(qd)
    with pytest.raises(native.AdjError, match="NOTIMPL"):
        native.batch_solve(b, qd, torch.zeros_like(qd), z, native.solve_opts(precond=native.PRECOND_JACOBI))
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_woodbury_without_z_matches_oracle_on_beam(prec):
    """The Woodbury preconditioner with its correction applied through
    Y = S E (no cached Z; the form large scenes use) reaches the oracle's
    adjoint on a frictional beam state, in about as many iterations as with
    Z."""
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, disc, q, rec = _beam()
    rng = np.random.default_rng(900 + prec)
    gq, gv = spec.loss_dir, 1e-3 * rng.standard_normal(q.shape)
    ref = adj.adjoint_step(disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=rec.contacts.n)
    tol = TOL_FP64 if prec == 0 else 1e-4
    rtol = 1e-13 if prec == 0 else 1e-8
    noz = run_adjoint(scene, rec, q, gq, gv, rtol=rtol, maxit=3000, prec=prec,
                      precond=native.PRECOND_WOODBURY_NO_Z, raise_noconv=False)
    errs = {k: rel(noz[k], getattr(ref, k)) for k in ("z", "dqbar", "dvbar", "dfext")}
    # the iteration counts of the two forms (the same preconditioner up to
    # rounding) compared at the throughput tolerance, away from the FP64 floor
    n8 = run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, maxit=3000, prec=prec, precond=native.PRECOND_WOODBURY_NO_Z)
    w8 = run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, maxit=3000, prec=prec)
    print(f"beam Woodbury without Z (prec {prec}): iters {noz['info'].iters}, relres {noz['info'].relres:.2e}, "
          + ", ".join(f"{k} {e:.1e}" for k, e in errs.items())
          + f"; at 1e-8: {n8['info'].iters} iterations (with Z {w8['info'].iters})", flush=True)
    assert noz["info"].relres <= (1e-11 if prec == 0 else 1e-8)
    assert abs(n8["info"].iters - w8["info"].iters) <= 2
    for k, e in errs.items():
        assert e <= tol, k


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("precond", ["woodbury", "no_z"])
def test_level_sweeps_match_products_and_oracle(prec, precond):
    """A^{-1} through the level-scheduled sweeps with L (tuning a_inv = 2)
    instead of the sparse-inverse products (a_inv = 1), in the Woodbury
    preconditioner with and without Z: the same adjoint as the oracle on a
    frictional beam state, FP64 and mixed, in about as many iterations."""
    torch_cuda()
    from paper_2603_16478_amd import native
    spec, disc, q, rec = _beam()
    rng = np.random.default_rng(910 + prec)
    gq, gv = spec.loss_dir, 1e-3 * rng.standard_normal(q.shape)
    ref = adj.adjoint_step(disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
    scene = make_scene(spec, max_contacts=rec.contacts.n)
    pc = native.PRECOND_WOODBURY if precond == "woodbury" else native.PRECOND_WOODBURY_NO_Z
    tol = TOL_FP64 if prec == 0 else 1e-4
    rtol = 1e-13 if prec == 0 else 1e-8
    out = {}
    for a_inv in (1, 2):
        native.set_tuning(scene, a_inv=a_inv)
        par = run_adjoint(scene, rec, q, gq, gv, rtol=rtol, maxit=3000, prec=prec, precond=pc, raise_noconv=False)
        thr = run_adjoint(scene, rec, q, gq, gv, rtol=1e-8, maxit=3000, prec=prec, precond=pc)
        out[a_inv] = (par, thr)
    par, thr = out[2]
    errs = {k: rel(par[k], getattr(ref, k)) for k in ("z", "dqbar", "dvbar", "dfext")}
    print(f"beam sweeps ({precond}, prec {prec}): relres {par['info'].relres:.2e}, "
          + ", ".join(f"{k} {e:.1e}" for k, e in errs.items())
          + f"; at 1e-8 {thr['info'].iters} iterations (products {out[1][1]['info'].iters})", flush=True)
    assert par["info"].relres <= (1e-11 if prec == 0 else 1e-8)
    for k, e in errs.items():
        assert e <= tol, k
    assert abs(thr["info"].iters - out[1][1]["info"].iters) <= 2
    scene.close()
