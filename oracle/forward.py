"""Converged forward step of the coupled residual (Sec. 3.3, eq:dynamics).
Test infrastructure only.

The paper takes the forward solver from prior work and does not restate it;
the adjoint only needs its converged fixed point.  This module solves the same
residual with a damped Newton method (a reading of our own, since the paper
does not give one):

  unknowns   q (3 n_v), lambda_n per contact, s per frictional contact, where
             the friction force is lambda_f = -s delta_f/|delta_f| (its
             direction is slaved to the tangential slip, which the third row
             of eq:contact enforces at a solution)
  rows       r_q   = M (q - qtilde) + h^2 sum_i w_i G_i^T (G_i q - p_i(q))
                     - h^2 sum_c H_c^T lambda_c
             phi_n = phi_eps(delta_n, lambda_n)
             phi_f = phi_eps(|delta_f|, mu lambda_n - s)
  Newton     eliminating (d lambda_n, d s) from the linearised contact rows
             leaves  Acal dq = -r_q + h^2 sum_c H_c^T R^T e_c  where Acal is
             the adjoint matrix A - dA + h^2 H^T K H (Sec. 5.1) evaluated at
             the iterate, and e_c = [-phi_n/beta_n, mu phi_n/beta_n - phi_f/beta_f, 0]
             with beta = d phi / d y.
  scaling    the Newton iteration evaluates each contact row as
             phi_{eps sqrt(k)}(k delta, lambda) with k = A_vv / h^2 (the
             vertex's inertial-plus-elastic stiffness): its zero set is the
             same branch delta lambda = eps^2, so the converged state is the
             paper's, but both arguments are forces, which keeps Newton steps
             on lambda bounded far from the solution.
  globalise  backtracking on 1/2 (|r_q/h^2|^2 + |phi|^2), no inverted tets,
             and no step may shrink |delta_f| of a frictional contact below
             1% of its value (its direction is undefined at 0, so iterates must
             not jump across the origin).

A frictional contact whose converged s is negative (it separated inside the
step) has no solution of the paper's friction rows; it is demoted to
normal-only and the step is solved again.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import contact as ct
from . import fb
from .elastic import ProjectionRecord, vec
from .fem import Discretisation, deformation_gradient


@dataclasses.dataclass
class StepRecord:
    """Everything the adjoint of one step needs besides (q, qbar)."""
    contacts: ct.ContactSet
    delta: np.ndarray  # (n_c, 3) frame coordinates
    lam: np.ndarray  # (n_c, 3) frame coordinates: lambda_n, lambda_f
    mu: float
    newton_iters: int = 0
    residual: float = 0.0
    targets: np.ndarray | None = None  # (n_b, 3) binding targets d_b of the step


def elastic_force_terms(disc: Discretisation, q: np.ndarray):
    F = deformation_gradient(q, disc.tets, disc.Bm)
    rec = ProjectionRecord(F, disc.mu, disc.lam, disc.model)
    Gq = vec(F).reshape(-1)
    return rec, Gq


def _contact_state(cs, u, g0, lam_n, s):
    delta = ct.displacement_from_step(cs, u, g0)
    nc = cs.n
    x = np.hypot(delta[:, 1], delta[:, 2])
    dhat = np.zeros((nc, 2))
    nz = x > 0
    dhat[nz] = delta[nz, 1:] / x[nz, None]
    dhat[~nz, 0] = 1.0
    lam = np.zeros((nc, 3))
    lam[:, 0] = lam_n
    fr = cs.fric
    lam[fr, 1:] = -s[fr, None] * dhat[fr]
    return delta, x, dhat, lam


def _residuals(disc, u, utilde, cs, qbar, g0, lam_n, s, mu, eps, k, targets=None):
    """Rows at the step displacement u = q - qbar (utilde = qtilde - qbar)."""
    h = disc.h
    rec, Gq = elastic_force_terms(disc, qbar + u)
    Pv = vec(rec.P).reshape(-1)
    wv = np.repeat(disc.w, 9)
    r = np.repeat(disc.mass, 3) * (u - utilde).reshape(-1) + h * h * (disc.G.T @ (wv * (Gq - Pv)))
    b = disc.bindings
    if b is not None and len(b.vid):
        # -h^2 J_b^T lambda_b with lambda_b = -(q_b - d_b) / E_b (eq:binding)
        qb = (qbar + u)[b.vid]
        np.add.at(r.reshape(-1, 3), b.vid, h * h * (qb - targets) / b.E[:, None])
    delta, x, dhat, lam = _contact_state(cs, u, g0, lam_n, s)
    if cs.n:
        fw = np.einsum("cki,ck->ci", cs.frame, lam)  # world-frame contact force per contact
        np.add.at(r.reshape(-1, 3), cs.vid, -h * h * fw)
    es = eps * np.sqrt(k)
    phin = fb.phi_eps(k * delta[:, 0], lam_n, es)
    phif = np.where(cs.fric, fb.phi_eps(k * x, mu * lam_n - s, es), 0.0)
    return rec, r, phin, phif, delta, x, dhat, lam


def _merit(r, phin, phif, h):
    return 0.5 * (np.sum((r / (h * h)) ** 2) + np.sum(phin ** 2) + np.sum(phif ** 2))


def elastic_tangent(disc: Discretisation, rec: ProjectionRecord) -> sp.csr_matrix:
    """A - dA = M + h^2 sum_i w_i G_i^T (I - J_i) G_i (Sec. 5.4 contact-free),
    plus h^2 J_b^T E_b^{-1} J_b when the scene has bindings (eq:differential_2)."""
    h = disc.h
    n_t = disc.tets.shape[0]
    J = rec.jacobian()  # (n_t, 9, 9)
    IJ = np.eye(9)[None] - J
    IJ *= disc.w[:, None, None]
    rows = (9 * np.arange(n_t))[:, None, None] + np.arange(9)[None, :, None] + 0 * np.arange(9)[None, None, :]
    cols = (9 * np.arange(n_t))[:, None, None] + 0 * np.arange(9)[None, :, None] + np.arange(9)[None, None, :]
    Bd = sp.csr_matrix((IJ.reshape(-1), (rows.reshape(-1), cols.reshape(-1))), shape=(9 * n_t, 9 * n_t))
    T = disc.M + h * h * (disc.G.T @ Bd @ disc.G)
    if disc.bindings is not None and len(disc.bindings.vid):
        T = T + disc.bindings.matrix(disc.n_verts, h)
    return T.tocsr()


def contact_matrix(n_verts: int, cs: ct.ContactSet, K: np.ndarray, h: float) -> sp.csr_matrix:
    """h^2 sum_c H_c^T K_c H_c with H_c = frame_c applied to vertex v_c."""
    if cs.n == 0:
        return sp.csr_matrix((3 * n_verts, 3 * n_verts))
    Kw = np.swapaxes(cs.frame, 1, 2) @ K @ cs.frame  # world 3x3 per contact
    rows = (3 * cs.vid)[:, None, None] + np.arange(3)[None, :, None] + 0 * np.arange(3)[None, None, :]
    cols = (3 * cs.vid)[:, None, None] + 0 * np.arange(3)[None, :, None] + np.arange(3)[None, None, :]
    return sp.csr_matrix(((h * h * Kw).reshape(-1), (rows.reshape(-1), cols.reshape(-1))),
                         shape=(3 * n_verts, 3 * n_verts))


def _newton_K(cs, delta, x, dhat, lam_n, s, mu, eps, k):
    """Linearisation of the (scaled) contact rows at the iterate: K_c, R, e-coefficients."""
    nc = cs.n
    es = eps * np.sqrt(k)
    a = k * fb.ratio(k * delta[:, 0], lam_n, es)
    _, beta_n = fb.partials(k * delta[:, 0], lam_n, es)
    yf = mu * lam_n - s
    b = np.where(cs.fric, k * fb.ratio(k * x, yf, es), 0.0)
    _, beta_f = fb.partials(k * x, yf, es)
    c = np.where((x > 0) & cs.fric, s / np.where(x > 0, x, 1.0), 0.0)
    R = np.tile(np.eye(3), (nc, 1, 1))
    R[:, 1, 1:] = dhat
    R[:, 2, 1] = -dhat[:, 1]
    R[:, 2, 2] = dhat[:, 0]
    Kh = np.zeros((nc, 3, 3))
    Kh[:, 0, 0] = a
    fr = cs.fric
    Kh[fr, 1, 0] = -mu * a[fr]
    Kh[fr, 1, 1] = b[fr]
    Kh[fr, 2, 2] = c[fr]
    K = np.swapaxes(R, 1, 2) @ Kh @ R
    return a, b, beta_n, beta_f, R, K


def _newton(disc, utilde, qbar, g0, cs, q, lam_n, s, mu, eps, k, maxit, tol_force, tol_phi, targets=None):
    """Damped Newton on (q, lambda_n, s) for the rows smoothed with eps (per
    contact, eps may be an array).  Returns (q, lam_n, s, state, iters, ok)."""
    h = disc.h
    n_v = disc.n_verts
    nc = cs.n
    state = _residuals(disc, q, utilde, cs, qbar, g0, lam_n, s, mu, eps, k, targets)
    merit = _merit(state[1], state[2], state[3], h)
    it = 0
    ok = False
    for it in range(1, maxit + 1):
        rec, r, phin, phif, delta, x, dhat, lam = state
        a, b, beta_n, beta_f, R, K = _newton_K(cs, delta, x, dhat, lam_n, s, mu, eps, k)
        Acal = elastic_tangent(disc, rec) + contact_matrix(n_v, cs, K, h)
        rhs = -r.copy()
        if nc:
            e = np.zeros((nc, 3))
            e[:, 0] = -phin / beta_n
            fr = cs.fric
            e[fr, 1] = mu * phin[fr] / beta_n[fr] - phif[fr] / beta_f[fr]
            ew = np.einsum("cki,ck->ci", cs.frame, np.einsum("cki,ck->ci", R, e))
            np.add.at(rhs.reshape(-1, 3), cs.vid, h * h * ew)
        dq = spla.spsolve(Acal.tocsc(), rhs, permc_spec="MMD_AT_PLUS_A").reshape(n_v, 3)
        if nc:
            ddelta = np.einsum("cak,ck->ca", cs.frame, dq[cs.vid])
            dlam_n = -a * ddelta[:, 0] - phin / beta_n
            dx = np.einsum("ca,ca->c", dhat, ddelta[:, 1:])
            ds = np.where(cs.fric, mu * dlam_n + b * dx + phif / np.where(cs.fric, beta_f, 1.0), 0.0)
        else:
            dlam_n = np.zeros(0)
            ds = np.zeros(0)
        alpha = 1.0
        if nc:
            fr = cs.fric & (x > 0)
            ddf = ddelta[:, 1:]
            for _ in range(60):
                xn = np.hypot(*(delta[:, 1:] + alpha * ddf).T)
                if not np.any(fr & (xn < 0.01 * x)):
                    break
                alpha *= 0.5
        accepted = False
        for _ in range(40):
            qn = q + alpha * dq
            try:
                st = _residuals(disc, qn, utilde, cs, qbar, g0, lam_n + alpha * dlam_n, s + alpha * ds, mu, eps, k,
                                targets)
            except ValueError:  # inverted element
                alpha *= 0.5
                continue
            mn = _merit(st[1], st[2], st[3], h)
            if mn <= (1.0 - 1e-4 * alpha) * merit or mn == 0.0:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            break  # stagnated
        q = qn
        lam_n = lam_n + alpha * dlam_n
        s = s + alpha * ds
        prev = merit
        state, merit = st, mn
        fmax = np.max(np.abs(state[1])) / (h * h)
        pmax = max(np.max(np.abs(state[2]), initial=0.0), np.max(np.abs(state[3]), initial=0.0))
        small = np.max(np.abs(alpha * dq)) <= 4e-16 * max(1.0, np.max(np.abs(q)))
        if alpha == 1.0 and ((fmax <= tol_force and pmax <= tol_phi) or small):
            ok = fmax <= 1e3 * tol_force and pmax <= 1e3 * tol_phi
            break
        # rounding floor: within 1e3 of the tolerances and the step no longer
        # halves the residual (merit is its square)
        if fmax <= 1e3 * tol_force and pmax <= 1e3 * tol_phi and merit > 0.25 * prev:
            ok = True
            break
    else:
        fmax = np.max(np.abs(state[1])) / (h * h)
        pmax = max(np.max(np.abs(state[2]), initial=0.0), np.max(np.abs(state[3]), initial=0.0))
    if not ok:
        fmax = np.max(np.abs(state[1])) / (h * h)
        pmax = max(np.max(np.abs(state[2]), initial=0.0), np.max(np.abs(state[3]), initial=0.0))
        ok = fmax <= 1e3 * tol_force and pmax <= 1e3 * tol_phi
    return q, lam_n, s, state, it, ok


def solve_step(disc: Discretisation, qbar, vbar, f_ext, gravity, mu, eps, planes,
               spheres_old=np.zeros((0, 4)), spheres_new=np.zeros((0, 4)), margin=2e-3,
               warm=None, maxit=60, tol_force=1e-11, tol_phi=1e-13, demote=(), targets=None):
    """One implicit step; returns (q, v, StepRecord, warm-start dict).

    A direct Newton solve is tried first; if it stalls, the step is re-solved
    by continuation: the rows are smoothed with eps_j^2 = eps^2 * gamma_j for
    a decreasing sequence gamma_j -> 1, each stage warm-started from the
    last.  Only the final stage (gamma = 1) defines the returned state.
    """
    h = disc.h
    acc = gravity[None, :] + f_ext / disc.mass[:, None]
    qtilde = ct.predict(qbar, vbar, acc, h)
    cs = ct.detect(qbar, qtilde, planes, spheres_old, spheres_new, margin)
    for (v, col) in demote:
        sel = (cs.vid == v) & (cs.collider == col)
        cs.fric[sel] = False
    nc = cs.n
    lam0 = np.zeros(nc)
    s0 = np.zeros(nc)
    if warm:
        for c in range(nc):
            key = (int(cs.vid[c]), int(cs.collider[c]))
            if key in warm:
                lam0[c], s0[c] = warm[key]
    s0[~cs.fric] = 0.0
    adiag = disc.A.diagonal()
    if disc.bindings is not None and len(disc.bindings.vid):
        adiag = adiag - disc.bindings.matrix(disc.n_verts, h).diagonal()  # contact scale from M + elastic
    k = adiag[3 * cs.vid] / (h * h)
    utilde = h * vbar + (h * h) * acc
    g0 = ct.gap_at(cs, qbar)
    u, lam_n, s = utilde.copy(), lam0.copy(), s0.copy()
    total = 0
    while True:
        start = (u.copy(), lam_n.copy(), s.copy())
        u, lam_n, s, state, its, ok = _newton(disc, utilde, qbar, g0, cs, u, lam_n, s, mu, eps, k,
                                              maxit, tol_force, tol_phi, targets)
        total += its
        if not ok:
            u, lam_n, s = start
            gamma = 1e6
            while True:
                last = gamma <= 1.0
                e_j = eps * np.sqrt(max(gamma, 1.0))
                tf = tol_force if last else 1e-7
                tp = tol_phi if last else 1e-7
                u, lam_n, s, state, its, ok = _newton(disc, utilde, qbar, g0, cs, u, lam_n, s, mu, e_j,
                                                      k, maxit, tf, tp, targets)
                total += its
                if last:
                    break
                gamma /= 30.0
        bad = cs.fric & (s < 0.0)
        if not np.any(bad):
            break
        # converged with a negative friction magnitude: the contact separated
        # inside the step and the friction rows have no solution; demote it
        cs.fric[bad] = False
        s[bad] = 0.0
    rec, r, phin, phif, delta, x, dhat, lam = state
    q = qbar + u
    v = u / h
    # report the paper's (unscaled) rows
    pn = fb.phi_eps(delta[:, 0], lam[:, 0], eps)
    pf = np.where(cs.fric, fb.phi_eps(x, mu * lam[:, 0] - s, eps), 0.0)
    resid = max(np.max(np.abs(r)) / (h * h), np.max(np.abs(pn), initial=0.0),
                np.max(np.abs(pf), initial=0.0))
    record = StepRecord(cs, delta, lam, mu, total, resid,
                        None if targets is None else np.array(targets, dtype=np.float64))
    new_warm = {(int(cs.vid[c]), int(cs.collider[c])): (lam_n[c], s[c]) for c in range(nc)}
    return q, v, record, new_warm
