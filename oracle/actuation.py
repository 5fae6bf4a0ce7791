"""Per-tet active stress of the actuated workload (the quadruped), test
infrastructure only.  Tet t of group g carries the active first Piola
stress P_a = a_g d_t d_t^T with its fibre direction d_t; its virtual work
V_t P_a : F_t gives the nodal forces f_v = -V_t P_a grad N_v, so the external
force of a step is linear in the group parameters, f = Phi a, and the
gradient of a loss through the step's external force is dL/da = Phi^T dL/df.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import Discretisation


def force_matrix(disc: Discretisation, group: np.ndarray, fibre: np.ndarray, n_groups: int) -> sp.csr_matrix:
    """Phi (3 n_v x n_groups): column g is the nodal force of a unit
    parameter of group g."""
    rows, cols, vals = [], [], []
    for t in range(disc.tets.shape[0]):
        d = fibre[t]
        Pa = np.outer(d, d)
        for k in range(4):
            f = -disc.vol[t] * (Pa @ disc.Bt[t, k])
            v = disc.tets[t, k]
            rows += [3 * v, 3 * v + 1, 3 * v + 2]
            cols += [group[t]] * 3
            vals += list(f)
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * disc.n_verts, n_groups))


def active_energy(disc: Discretisation, group: np.ndarray, fibre: np.ndarray, a: np.ndarray, q: np.ndarray) -> float:
    """W(q) = sum_t V_t a_g(t) d_t^T F_t(q) d_t, whose negative gradient is the
    active force."""
    x = q[disc.tets]  # (n_t, 4, 3)
    Ds = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    F = Ds @ disc.Bm
    return float(np.sum(disc.vol * a[group] * np.einsum("ti,tij,tj->t", fibre, F, fibre)))
