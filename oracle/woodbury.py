"""Dense Woodbury preconditioner for the transposed adjoint system (Sec. 5.4,
eq:woodbury_formula).  Test infrastructure only; meant for small meshes.

For the contact part Kcal = h^2 H^T K H, the identity reads
    (A + h^2 H^T K H)^{-1} = A^{-1} - h^2 A^{-1} H^T (K^{-1} + h^2 H A^{-1} H^T)^{-1} H A^{-1}
and the preconditioner for Acal^T = (A - dA + Kcal)^T drops -dA (the paper
builds it from A + Kcal) and uses K^T, i.e.
    P = A^{-1} - h^2 A^{-1} H^T (K^{-T} + h^2 H A^{-1} H^T)^{-1} H A^{-1}.
Rows whose K block is singular (a zero c = |lambda_f|/|delta_f|) are dropped
from H: their contribution to Kcal is zero.
"""

from __future__ import annotations

import numpy as np

from .contact import ContactBlocks, ContactSet


def contact_rows(n_verts: int, cs: ContactSet, blocks: ContactBlocks):
    """H in the rotated contact basis (rows R_c frame_c on vertex v_c) and the
    block-diagonal Khat, restricted to the rows that Kcal actually uses."""
    rows = []
    kblocks = []
    for c in range(cs.n):
        Q = blocks.R[c] @ cs.frame[c]  # rows: normal, slip direction, perpendicular
        Kh = blocks.Khat[c]
        keep = [0] if not cs.fric[c] else [i for i in range(3) if i < 2 or Kh[2, 2] != 0.0]
        for i in keep:
            r = np.zeros(3 * n_verts)
            r[3 * cs.vid[c]:3 * cs.vid[c] + 3] = Q[i]
            rows.append(r)
        kblocks.append(Kh[np.ix_(keep, keep)])
    if not rows:
        return np.zeros((0, 3 * n_verts)), np.zeros((0, 0))
    H = np.array(rows)
    m = H.shape[0]
    K = np.zeros((m, m))
    o = 0
    for kb in kblocks:
        n = kb.shape[0]
        K[o:o + n, o:o + n] = kb
        o += n
    return H, K


def preconditioner_T(A: np.ndarray, H: np.ndarray, K: np.ndarray, h: float) -> np.ndarray:
    """Dense P = (A + h^2 H^T K^T H)^{-1} through the Woodbury identity."""
    Ainv = np.linalg.inv(A)
    if H.shape[0] == 0:
        return Ainv
    C = np.linalg.inv(K).T + h * h * (H @ Ainv @ H.T)
    return Ainv - h * h * Ainv @ H.T @ np.linalg.solve(C, H @ Ainv)


def capacitance_T(A: np.ndarray, H: np.ndarray, K: np.ndarray, h: float) -> np.ndarray:
    """C^T-system capacitance K^{-T} + h^2 H A^{-1} H^T."""
    return np.linalg.inv(K).T + h * h * (H @ np.linalg.solve(A, H.T))
