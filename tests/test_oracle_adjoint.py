"""Pins for the adjoint oracle: matrix structure, per-step gradients against
central finite differences through the converged forward step, the Woodbury
identity, and a full tiny rollout (Sec. 5.1, 5.4; App. B.3)."""

import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import adjoint as adj
from oracle import woodbury
from oracle.forward import solve_step
from oracle.rollout import backward, linear_loss, run_forward, scene_disc
from synth import tiny_scene


@functools.lru_cache(maxsize=None)
def _tiny_rollout(steps):
    spec = tiny_scene("impact")
    return spec, run_forward(spec, steps=steps)


def _step_loss(spec, disc, qbar, vbar, f, mu, g, gv, warm):
    q, v, rec, _ = solve_step(disc, qbar, vbar, f, spec.gravity, mu, spec.eps, spec.planes,
                              margin=spec.contact_margin, warm=warm)
    return float(np.sum(g * q) + np.sum(gv * v)), rec


def _warm(rec):
    return {(int(rec.contacts.vid[c]), int(rec.contacts.collider[c])):
            (rec.lam[c, 0], float(np.hypot(rec.lam[c, 1], rec.lam[c, 2]))) for c in range(rec.contacts.n)}


def test_contact_free_matrix_spd_above_mass():
    """Contact-free Acal = M + h^2 sum w G^T (I - J) G is SPD with
    lambda_min >= min(M) (Sec. 5.4 contact-free)."""
    spec, ro = _tiny_rollout(3)
    rec = ro.records[-1]
    assert rec.contacts.n == 0
    sysm = adj.assemble(ro.disc, ro.qs[-1], rec, spec.eps)
    A = sysm.Acal.toarray()
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    lmin = np.linalg.eigvalsh(A).min()
    assert lmin >= ro.disc.mass.min() * (1 - 1e-9)


@pytest.mark.slow
@pytest.mark.parametrize("step", [9, 13])
def test_step_gradients_match_fd(step):
    """z^T Kcal_x equals the derivative of g.q + gv.v through one converged
    forward step, for x = E, nu, mu, qbar, vbar, f_ext (eq:compute_gradient)."""
    spec, ro = _tiny_rollout(step)
    disc = ro.disc
    qbar, vbar = ro.qs[-1], ro.vs[-1]
    warm = _warm(ro.records[-1]) if step > 0 else None
    rng = np.random.default_rng(step)
    g = rng.standard_normal(qbar.shape)
    gv = 1e-3 * rng.standard_normal(qbar.shape)
    f = spec.force(step)
    q, v, rec, _ = solve_step(disc, qbar, vbar, f, spec.gravity, spec.mu, spec.eps, spec.planes,
                              margin=spec.contact_margin, warm=warm)
    assert rec.residual < 1e-9
    grads = adj.adjoint_step(disc, q, rec, g, gv, spec.eps, spec.E, spec.nu)

    def fd(fun, eta):
        """Central difference; the step shrinks until neither side changes the
        discrete contact state (candidate set, friction rows), across which
        the step map is not differentiable."""
        for _ in range(6):
            (lp, rp), (lm, rm) = fun(eta), fun(-eta)
            same = all(np.array_equal(r.contacts.vid, rec.contacts.vid)
                       and np.array_equal(r.contacts.fric, rec.contacts.fric) for r in (rp, rm))
            if same:
                return (lp - lm) / (2 * eta)
            eta /= 10.0
        raise AssertionError("contact state changes under every probe step")

    dE = fd(lambda e: _step_loss(spec, scene_disc(spec, E=spec.E + e), qbar, vbar, f, spec.mu, g, gv, warm), 1e-5 * spec.E)
    dnu = fd(lambda e: _step_loss(spec, scene_disc(spec, nu=spec.nu + e), qbar, vbar, f, spec.mu, g, gv, warm), 1e-6)
    dq = rng.standard_normal(qbar.shape)
    dv = rng.standard_normal(qbar.shape)
    df = rng.standard_normal(qbar.shape)
    dqb = fd(lambda e: _step_loss(spec, disc, qbar + e * dq, vbar, f, spec.mu, g, gv, warm), 1e-9)
    dvb = fd(lambda e: _step_loss(spec, disc, qbar, vbar + e * dv, f, spec.mu, g, gv, warm), 1e-6)
    dfx = fd(lambda e: _step_loss(spec, disc, qbar, vbar, f + e * df, spec.mu, g, gv, warm), 1e-6)
    assert abs(grads.dE - dE) <= 1e-5 * abs(dE) + 1e-14
    assert abs(grads.dnu - dnu) <= 1e-5 * abs(dnu) + 1e-12
    assert abs(np.sum(grads.dqbar * dq) - dqb) <= 1e-4 * abs(dqb) + 1e-9
    assert abs(np.sum(grads.dvbar * dv) - dvb) <= 2e-4 * abs(dvb) + 1e-12
    assert abs(np.sum(grads.dfext * df) - dfx) <= 2e-4 * abs(dfx) + 1e-12
    if rec.contacts.fric.any():
        dmu = fd(lambda e: _step_loss(spec, disc, qbar, vbar, f, spec.mu + e, g, gv, warm), 1e-5)
        assert abs(grads.dmu_fric - dmu) <= 1e-3 * abs(dmu) + 1e-9


def test_woodbury_identity_dense():
    """(A + h^2 H^T K^T H)^{-1} via the Woodbury identity equals the explicit
    inverse (eq:woodbury_formula), on a contact state of the tiny cube."""
    spec, ro = _tiny_rollout(12)
    disc = ro.disc
    rec = ro.records[-1]
    blocks = adj.assemble(disc, ro.qs[-1], rec, spec.eps).blocks
    H, K = woodbury.contact_rows(disc.n_verts, rec.contacts, blocks)
    A = disc.A.toarray()
    P = woodbury.preconditioner_T(A, H, K, disc.h)
    explicit = np.linalg.inv(A + disc.h ** 2 * H.T @ K.T @ H)
    assert np.abs(P - explicit).max() <= 1e-6 * np.abs(explicit).max()
    # the contact part of Acal is exactly h^2 H^T K H
    from oracle.forward import contact_matrix
    Kc = contact_matrix(disc.n_verts, rec.contacts, blocks.K, disc.h).toarray()
    np.testing.assert_allclose(Kc, disc.h ** 2 * H.T @ K @ H, atol=1e-9 * np.abs(Kc).max())


def test_woodbury_exact_without_dA_gives_one_step():
    """With dA switched off the preconditioner is the exact inverse, so a
    preconditioned Krylov solve converges in one iteration."""
    spec, ro = _tiny_rollout(12)
    disc = ro.disc
    rec = ro.records[-1]
    blocks = adj.assemble(disc, ro.qs[-1], rec, spec.eps).blocks
    H, K = woodbury.contact_rows(disc.n_verts, rec.contacts, blocks)
    A = disc.A.toarray()
    AT = (A + disc.h ** 2 * H.T @ K @ H).T
    P = woodbury.preconditioner_T(A, H, K, disc.h)
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    its = []
    spla.gmres(AT @ P, b, rtol=1e-10, restart=20, maxiter=20, callback=lambda r: its.append(r),
               callback_type="pr_norm")
    assert len(its) <= 2


@pytest.mark.slow
def test_rollout_gradient_matches_fd():
    """Full 20-step tiny-impact rollout: backward recursion vs central FD in
    E, nu and along a random initial-velocity direction (Sec. 6.1 protocol)."""
    spec, ro = _tiny_rollout(20)
    g = backward(spec, ro, spec.loss_dir)
    L = lambda **kw: linear_loss(spec, run_forward(spec, **kw))  # noqa: E731
    dE = (L(E=spec.E * (1 + 1e-6)) - L(E=spec.E * (1 - 1e-6))) / (2e-6 * spec.E)
    dnu = (L(nu=spec.nu + 1e-7) - L(nu=spec.nu - 1e-7)) / 2e-7
    rng = np.random.default_rng(5)
    dv = rng.standard_normal(spec.v0.shape)
    dv[:, 2] = 0.0  # tangential: a normal perturbation shifts the touchdown step
    e = 1e-7
    dv0 = (L(v0=spec.v0 + e * dv) - L(v0=spec.v0 - e * dv)) / (2 * e)
    assert abs(g.dE - dE) <= 1e-5 * abs(dE)
    assert abs(g.dnu - dnu) <= 1e-5 * abs(dnu)
    assert abs(np.sum(g.dv0 * dv) - dv0) <= 1e-4 * abs(dv0)


def test_stored_slip_onset_solutions_solve_the_oracle_system():
    """The stored oracle z of the beam's slip-onset steps (the fixture the
    GPU parity and the benchmark compare with) solves Acal^T z = r for the
    oracle's own assembly of the stored states, one step per friction
    coefficient, and the stored states really cross the onset: the number
    of contacts at the friction bound grows over the stored steps."""
    import os
    from conftest import ROOT
    from oracle.contact import ContactSet
    from oracle.forward import StepRecord
    from synth import beam_scene
    zd = np.load(os.path.join(ROOT, "tests", "golden", "beam_onset_z.npz"))
    for mu, k in ((0.1, 2), (0.4, 2)):
        d = np.load(os.path.join(ROOT, "tests", "golden", f"beam_onset_mu{mu}.npz"))
        at_bound = []
        for j in range(int(d["steps"])):
            lam = d[f"lam{j}"]
            at_bound.append(int(np.sum(np.hypot(lam[:, 1], lam[:, 2]) > 0.99 * mu * lam[:, 0])))
        if mu == 0.1:
            assert at_bound[-2] > at_bound[0] + 40
        cs = ContactSet(d[f"vid{k}"], d[f"collider{k}"], d[f"frame{k}"], d[f"d_n{k}"], d[f"d_f{k}"],
                        d[f"fric{k}"].astype(bool))
        rec = StepRecord(cs, d[f"delta{k}"], d[f"lam{k}"], mu)
        spec = beam_scene(mu=mu)
        i = [n for n in range(zd["z"].shape[0]) if zd["mu"][n] == mu and zd["t"][n] == int(d[f"t{k}"])]
        assert len(i) == 1
        sysm = adj.assemble(scene_disc(spec), d[f"q{k}"], rec, spec.eps)
        b = spec.loss_dir.reshape(-1)
        r = sysm.Acal.T @ zd["z"][i[0]].reshape(-1) - b
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)
