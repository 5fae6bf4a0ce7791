"""Contact candidates, frames and contact Jacobian blocks.  Test
infrastructure only.

Constraint displacement in the contact frame (Sec. 3.2, eq:contact):
    delta_n = n . x_v - d_n,   delta_f = T (x_v - xbar_v) - d_f,  T = [t1; t2]
with the frame held fixed within the step (Sec. 5.2, eq:diff_contact).

The paper does not describe contact detection; the reading used here:
  * colliders are half-spaces (n . x >= d) and kinematic spheres;
  * a vertex is a candidate when its gap at the inertial prediction
    qtilde = (qbar + h vbar) + (h*h) (g + f/m) is <= margin (sphere: the gap
    to the tangent plane at the frozen normal, with the sphere's new centre);
  * the frame: n = plane normal, or for a sphere (xbar - c_old)/|xbar - c_old|;
    t1 = normalise(n x e_k) with e_k the axis of smallest |n_k| (lowest k on
    ties), t2 = n x t1;
  * d_n = plane offset, or n . c_new + radius; d_f = T (c_new - c_old) for a
    sphere, 0 for a plane;
  * candidates whose predicted gap is > 0 are normal-only for the step (no
    friction rows): with the smoothed friction row a separated contact would
    need |delta_f| >= delta_n / mu, which a resting vertex cannot meet;
  * the list is sorted by vertex id, then collider (planes, then spheres).

Contact Jacobian (Sec. 5.2, eq:partial_contact, eq:final_diff_contact):
    d lambda_c / d delta_c = -K_c = -R^T Khat R,
    Khat = [[a, 0, 0], [-mu a, b, 0], [0, 0, c]],
    a = phi ratio at (delta_n, lambda_n), b = ratio at (|delta_f|, mu lambda_n - |lambda_f|),
    c = |lambda_f| / |delta_f|,   k_mu = R^T [0, lambda_n, 0]
R (App. A.1): rows [n-axis; tangential main direction; its perpendicular],
taken from lambda_f if |lambda_f| >= TAU_LAMBDA, else from delta_f if
|delta_f| >= TAU_DELTA, else the identity.  Normal-only contacts use the 1x1
block [a] on the normal axis.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import fb

TAU_LAMBDA = 1e-10  # N
TAU_DELTA = 1e-12  # m


@dataclasses.dataclass
class ContactSet:
    vid: np.ndarray  # (n_c,) int32, sorted
    collider: np.ndarray  # (n_c,) int32: plane index, or n_planes + sphere index
    frame: np.ndarray  # (n_c, 3, 3) rows n, t1, t2
    d_n: np.ndarray  # (n_c,)
    d_f: np.ndarray  # (n_c, 2)
    fric: np.ndarray  # (n_c,) bool

    @property
    def n(self) -> int:
        return int(self.vid.shape[0])

    @staticmethod
    def empty():
        return ContactSet(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 3, 3)),
                          np.zeros(0), np.zeros((0, 2)), np.zeros(0, bool))


def tangent_frame(n: np.ndarray) -> np.ndarray:
    """Rows n, t1, t2 for a unit normal n (3,)."""
    k = int(np.argmin(np.abs(n)))  # argmin returns the lowest index on ties
    e = np.zeros(3)
    e[k] = 1.0
    c = np.array([n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2], n[0] * e[1] - n[1] * e[0]])
    t1 = c / np.sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2])
    t2 = np.array([n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]])
    return np.stack([n, t1, t2])


def predict(qbar, vbar, acc, h):
    """qtilde = (qbar + h vbar) + (h*h) acc, evaluated left to right."""
    return (qbar + h * vbar) + (h * h) * acc


def detect(qbar, qtilde, planes, spheres_old, spheres_new, margin) -> ContactSet:
    planes = np.asarray(planes, dtype=np.float64).reshape(-1, 4)
    spheres_old = np.asarray(spheres_old, dtype=np.float64).reshape(-1, 4)
    spheres_new = np.asarray(spheres_new, dtype=np.float64).reshape(-1, 4)
    n_p = planes.shape[0]
    out = []
    for v in range(qbar.shape[0]):
        for p in range(n_p):
            n = planes[p, :3]
            x = qtilde[v]
            gap = ((n[0] * x[0] + n[1] * x[1]) + n[2] * x[2]) - planes[p, 3]
            if gap <= margin:
                out.append((v, p, tangent_frame(n), planes[p, 3], np.zeros(2), gap <= 0.0))
        for s in range(spheres_old.shape[0]):
            c0 = spheres_old[s, :3]
            c1 = spheres_new[s, :3]
            R = spheres_new[s, 3]
            dv = qbar[v] - c0
            nrm = np.sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2])
            if nrm == 0.0:
                continue
            n = dv / nrm
            fr = tangent_frame(n)
            d_n = ((n[0] * c1[0] + n[1] * c1[1]) + n[2] * c1[2]) + R
            x = qtilde[v]
            gap = ((n[0] * x[0] + n[1] * x[1]) + n[2] * x[2]) - d_n
            if gap <= margin:
                dc = c1 - c0
                d_f = fr[1:] @ dc
                out.append((v, n_p + s, fr, d_n, d_f, gap <= 0.0))
    if not out:
        return ContactSet.empty()
    return ContactSet(
        vid=np.array([o[0] for o in out], np.int32),
        collider=np.array([o[1] for o in out], np.int32),
        frame=np.array([o[2] for o in out]),
        d_n=np.array([o[3] for o in out], dtype=np.float64),
        d_f=np.array([o[4] for o in out], dtype=np.float64),
        fric=np.array([o[5] for o in out], dtype=bool),
    )


def displacement(cs: ContactSet, q, qbar) -> np.ndarray:
    """delta_c in frame coordinates, (n_c, 3)."""
    x = q[cs.vid]
    xb = qbar[cs.vid]
    dn = np.einsum("ck,ck->c", cs.frame[:, 0], x) - cs.d_n
    df = np.einsum("cak,ck->ca", cs.frame[:, 1:], x - xb) - cs.d_f
    return np.concatenate([dn[:, None], df], axis=1)


def gap_at(cs: ContactSet, qbar) -> np.ndarray:
    """Normal gap at the start of the step, n . xbar_v - d_n."""
    return np.einsum("ck,ck->c", cs.frame[:, 0], qbar[cs.vid]) - cs.d_n


def displacement_from_step(cs: ContactSet, u, g0) -> np.ndarray:
    """delta_c from the step displacement u = q - qbar:
    delta_n = g0 + n . u_v,  delta_f = T u_v - d_f (no cancellation of positions)."""
    uv = u[cs.vid]
    dn = g0 + np.einsum("ck,ck->c", cs.frame[:, 0], uv)
    df = np.einsum("cak,ck->ca", cs.frame[:, 1:], uv) - cs.d_f
    return np.concatenate([dn[:, None], df], axis=1)


def rotation_from(v2: np.ndarray, use_lambda: bool) -> np.ndarray:
    """App. A.1: rows [e_n; dir; perp] built from a tangential 2-vector."""
    nv = np.hypot(v2[0], v2[1])
    R = np.eye(3)
    if use_lambda:
        d1, d2 = -v2[0] / nv, -v2[1] / nv
    else:
        d1, d2 = v2[0] / nv, v2[1] / nv
    R[1, 1:] = [d1, d2]
    R[2, 1:] = [-d2, d1]
    return R


@dataclasses.dataclass
class ContactBlocks:
    R: np.ndarray  # (n_c,3,3)
    Khat: np.ndarray  # (n_c,3,3)
    K: np.ndarray  # (n_c,3,3)  K_c = R^T Khat R, frame coordinates
    kmu: np.ndarray  # (n_c,3)


def contact_blocks(cs: ContactSet, delta: np.ndarray, lam: np.ndarray, mu: float, eps: float) -> ContactBlocks:
    """K_c, k_mu per contact from the converged (delta_c, lambda_c) (eq:final_diff_contact)."""
    nc = cs.n
    Rs = np.zeros((nc, 3, 3))
    Kh = np.zeros((nc, 3, 3))
    for c in range(nc):
        dn, ln = delta[c, 0], lam[c, 0]
        a = float(fb.ratio(dn, ln, eps))
        if not cs.fric[c]:
            Rs[c] = np.eye(3)
            Kh[c, 0, 0] = a
            continue
        df = delta[c, 1:]
        lf = lam[c, 1:]
        ndf = np.hypot(df[0], df[1])
        nlf = np.hypot(lf[0], lf[1])
        if nlf >= TAU_LAMBDA:
            R = rotation_from(lf, True)
        elif ndf >= TAU_DELTA:
            R = rotation_from(df, False)
        else:
            R = np.eye(3)
        b = float(fb.ratio(ndf, mu * ln - nlf, eps))
        cc = nlf / ndf if ndf > 0 else 0.0
        Rs[c] = R
        Kh[c] = [[a, 0.0, 0.0], [-mu * a, b, 0.0], [0.0, 0.0, cc]]
    K = np.swapaxes(Rs, 1, 2) @ Kh @ Rs
    kmu = np.zeros((nc, 3))
    for c in range(nc):
        if cs.fric[c]:
            kmu[c] = Rs[c].T @ np.array([0.0, lam[c, 0], 0.0])
    return ContactBlocks(Rs, Kh, K, kmu)
