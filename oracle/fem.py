"""Discretisation of the tet mesh (Sec. 3.1 eq:implicit, Sec. 3.3 eq:internal,
eq:dynamics).  Test infrastructure only.

Conventions (column-major vec, App. B.0):
  D_m = [X_b - X_a, X_c - X_a, X_d - X_a],  B_m = D_m^{-1},  V_i = det(D_m)/6
  F   = D_s B_m = sum_k x_k Bt_k^T  with  Bt = [-1^T B_m ; B_m]  (4x3)
  vec F = G_i q,  G_i = Bt^T (x) I_3   (9 x 12 on the element's 12 DOFs)
  lumped mass: each tet gives rho V_i / 4 to each of its vertices
  w_i = 2 mu_i V_i (the paper's w = 2 mu per unit volume, App. B.2)
  A = M + h^2 sum_i w_i G_i^T G_i                       (eq:dynamics)
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


def lame(E, nu):
    """Shear modulus and Lame's first parameter (App. B.3)."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def rest_operators(rest: np.ndarray, tets: np.ndarray):
    """Per-tet B_m (n_t,3,3), volume (n_t,), Bt (n_t,4,3)."""
    X = rest[tets]  # (n_t, 4, 3)
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(Dm)
    if np.any(det <= 0):
        raise ValueError("rest tet with non-positive orientation")
    Bm = np.linalg.inv(Dm)
    vol = det / 6.0
    Bt = np.concatenate([-Bm.sum(axis=1, keepdims=True), Bm], axis=1)
    return Bm, vol, Bt


def deformation_gradient(q: np.ndarray, tets: np.ndarray, Bm: np.ndarray) -> np.ndarray:
    """F = D_s B_m per tet, (n_t, 3, 3)."""
    x = q[tets]
    Ds = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    return Ds @ Bm


def lumped_mass(n_verts: int, tets: np.ndarray, vol: np.ndarray, density: float) -> np.ndarray:
    m = np.zeros(n_verts)
    np.add.at(m, tets.reshape(-1), np.repeat(density * vol / 4.0, 4))
    return m


def global_G(n_verts: int, tets: np.ndarray, Bt: np.ndarray) -> sp.csr_matrix:
    """Stacked G: rows (tet i, 3c + r) -> d(vec F_i)_{r+3c} / d q_{k,s} = delta_rs Bt_{k,c}."""
    n_t = tets.shape[0]
    rows, cols, vals = [], [], []
    ti = np.arange(n_t)
    for c in range(3):
        for r in range(3):
            for k in range(4):
                rows.append(9 * ti + 3 * c + r)
                cols.append(3 * tets[:, k] + r)
                vals.append(Bt[:, k, c])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(9 * n_t, 3 * n_verts))


@dataclasses.dataclass
class Bindings:
    """Bilateral bindings (Sec. 3.2, eq:binding): vertex vid[b] is held to a
    target d_b (given per step) by a linear spring of compliance E[b]:
    phi_b = (q_vid - d_b) + E_b lambda_b = 0, so the binding force on the
    vertex is lambda_b = -(q_vid - d_b) / E_b."""
    vid: np.ndarray  # (n_b,) int, distinct vertices
    E: np.ndarray  # (n_b,) > 0

    def matrix(self, n_verts: int, h: float) -> sp.csr_matrix:
        """h^2 J_b^T E_b^{-1} J_b (the binding term of the system matrix)."""
        d = np.zeros(3 * n_verts)
        for v, e in zip(self.vid, self.E):
            d[3 * v:3 * v + 3] += h * h / e
        return sp.diags(d).tocsr()


@dataclasses.dataclass
class Discretisation:
    n_verts: int
    tets: np.ndarray
    Bm: np.ndarray
    vol: np.ndarray
    Bt: np.ndarray
    mass: np.ndarray  # per vertex (n_v,)
    G: sp.csr_matrix  # (9 n_t, 3 n_v)
    mu: np.ndarray  # per tet
    lam: np.ndarray  # per tet
    w: np.ndarray  # per tet, 2 mu V
    h: float
    A: sp.csr_matrix  # (3 n_v, 3 n_v), binding term included
    bindings: Bindings | None = None
    model: str = "nh"  # local projection: "nh", "arap" or "corot" (App. B.2)

    @property
    def M(self) -> sp.dia_matrix:
        return sp.diags(np.repeat(self.mass, 3))


def discretise(rest, tets, density, E, nu, h, bindings: Bindings | None = None, model: str = "nh") -> Discretisation:
    n_v = rest.shape[0]
    Bm, vol, Bt = rest_operators(rest, tets)
    mass = lumped_mass(n_v, tets, vol, density)
    G = global_G(n_v, tets, Bt)
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), vol.shape)
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), vol.shape)
    mu, lam = lame(E, nu)
    w = 2.0 * mu * vol
    Wd = sp.diags(np.repeat(w, 9))
    A = (sp.diags(np.repeat(mass, 3)) + h * h * (G.T @ Wd @ G)).tocsr()
    if bindings is not None and len(bindings.vid):
        A = (A + bindings.matrix(n_v, h)).tocsr()
    return Discretisation(n_v, tets, Bm, vol, Bt, mass, G, mu.copy(), lam.copy(), w, h, A, bindings, model)
