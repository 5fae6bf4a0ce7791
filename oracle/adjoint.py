"""Adjoint of one converged step (Sec. 5.1 eq:differential_2, eq:adjoint,
eq:compute_gradient; Sec. 5.2 eq:final_diff_contact; App. B.3).  Test
infrastructure only.

    Acal   = A - dA + h^2 H_c^T K_c H_c,   dA = h^2 sum_i w_i G_i^T J_i G_i
    Acal^T z = (dL/dq + dL/dv / h)^T                        (eq:adjoint)
    dL/dqbar = z^T (M + h^2 H_c^T K_c P_f H_c) - dL/dv / h
    dL/dvbar = h M z,   dL/df_ext = h^2 z
    dL/dmu_fric = -h^2 sum_c (H_c z) . k_mu,c
    dL/dmu_i  = 2 h^2 V_i (G_i z) . (mu_i dp_i/dmu + p_i - G_i q)
    dL/dlam_i = 2 h^2 V_i mu_i (G_i z) . dp_i/dlam           (App. B.3, with
                w_i = 2 mu_i V_i so the per-volume formulas gain V_i)
    dL/dE, dL/dnu by the chain rule through mu = E/(2(1+nu)),
                lam = E nu/((1+nu)(1-2nu)).
    Bindings (eq:binding; eq:differential_2 rhs_d_b and rhs_E_b), with
    lambda_b = -(q_b - d_b) / E_b:
    dL/dd_b = h^2 E_b^{-1} z_b,   dL/dE_b = -h^2 E_b^{-1} lambda_b . z_b

The solve is a direct sparse LU of Acal^T (the plain definition of z) followed
by iterative refinement whose residual is formed in extended precision
(numpy.longdouble), so the oracle's own error is far below the tolerances the
HIP path is held to.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import contact as ct
from .elastic import ProjectionRecord, vec
from .fem import Discretisation, deformation_gradient
from .forward import StepRecord, contact_matrix, elastic_tangent


@dataclasses.dataclass
class AdjointSystem:
    Acal: sp.csr_matrix
    rec: ProjectionRecord
    blocks: ct.ContactBlocks


def assemble(disc: Discretisation, q: np.ndarray, record: StepRecord, eps: float) -> AdjointSystem:
    F = deformation_gradient(q, disc.tets, disc.Bm)
    rec = ProjectionRecord(F, disc.mu, disc.lam, disc.model)
    blocks = ct.contact_blocks(record.contacts, record.delta, record.lam, record.mu, eps)
    Acal = elastic_tangent(disc, rec) + contact_matrix(disc.n_verts, record.contacts, blocks.K, disc.h)
    return AdjointSystem(Acal.tocsr(), rec, blocks)


def _matvec_ld(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = A x accumulated in numpy.longdouble."""
    data = A.data.astype(np.longdouble)
    prod = data * x.astype(np.longdouble)[A.indices]
    y = np.zeros(A.shape[0], dtype=np.longdouble)
    np.add.at(y, np.repeat(np.arange(A.shape[0]), np.diff(A.indptr)), prod)
    return y


def solve_transposed(Acal: sp.csr_matrix, rhs: np.ndarray, refine: int = 3) -> np.ndarray:
    """z = Acal^{-T} rhs by SuperLU plus refinement with a long-double residual."""
    AT = Acal.T.tocsc()
    lu = spla.splu(AT, permc_spec="COLAMD")
    z = lu.solve(rhs)
    ATr = AT.tocsr()
    b = rhs.astype(np.longdouble)
    for _ in range(refine):
        r = (b - _matvec_ld(ATr, z)).astype(np.float64)
        z = z + lu.solve(r)
    return z


@dataclasses.dataclass
class StepGradients:
    z: np.ndarray  # (n_v, 3)
    dqbar: np.ndarray  # (n_v, 3)
    dvbar: np.ndarray
    dfext: np.ndarray
    dmu_fric: float
    dmu_tet: np.ndarray  # per tet (Lame mu)
    dlam_tet: np.ndarray
    dE_tet: np.ndarray
    dnu_tet: np.ndarray
    dtarget: np.ndarray | None = None  # (n_b, 3) dL/dd_b
    dE_bind: np.ndarray | None = None  # (n_b,) dL/dE_b

    @property
    def dE(self) -> float:
        return float(self.dE_tet.sum())

    @property
    def dnu(self) -> float:
        return float(self.dnu_tet.sum())


def lame_chain(dmu, dlam, E, nu):
    """(dL/dE, dL/dnu) from (dL/dmu, dL/dlam) (App. B.3)."""
    dmu_dE = 1.0 / (2.0 * (1.0 + nu))
    dlam_dE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    dmu_dnu = -E / (2.0 * (1.0 + nu) ** 2)
    dlam_dnu = E * (1.0 + 2.0 * nu * nu) / ((1.0 + nu) ** 2 * (1.0 - 2.0 * nu) ** 2)
    return dmu * dmu_dE + dlam * dlam_dE, dmu * dmu_dnu + dlam * dlam_dnu


def vjp(disc: Discretisation, sysm: AdjointSystem, q: np.ndarray, record: StepRecord,
        z: np.ndarray, dL_dv: np.ndarray, E, nu) -> StepGradients:
    h = disc.h
    n_v = disc.n_verts
    z3 = z.reshape(n_v, 3)
    cs = record.contacts
    mass = disc.mass[:, None]
    dqbar = mass * z3 - dL_dv.reshape(n_v, 3) / h
    dmu_fric = 0.0
    if cs.n:
        Hz = np.einsum("cak,ck->ca", cs.frame, z3[cs.vid])  # frame coordinates
        Pf = np.diag([0.0, 1.0, 1.0])
        # h^2 H_c^T P_f K_c^T H_c z  (transpose of K_qbar's contact part)
        t = np.einsum("cba,cb->ca", sysm.blocks.K, Hz)  # K_c^T (H_c z)
        t = t @ Pf
        tw = np.einsum("cki,ck->ci", cs.frame, t)
        np.add.at(dqbar, cs.vid, h * h * tw)
        dmu_fric = float(-h * h * np.sum(np.einsum("ca,ca->c", Hz, sysm.blocks.kmu)))
    dvbar = h * mass * z3
    dfext = h * h * z3
    rec = sysm.rec
    Gz = (disc.G @ z).reshape(-1, 9)
    Gq = (disc.G @ q.reshape(-1)).reshape(-1, 9)
    p = vec(rec.P)
    dp_dmu = vec(rec.dP_dmu())
    dp_dlam = vec(rec.dP_dlam())
    V = disc.vol
    mu_i = disc.mu
    dmu_tet = 2 * h * h * V * np.einsum("ij,ij->i", Gz, mu_i[:, None] * dp_dmu + p - Gq)
    dlam_tet = 2 * h * h * V * mu_i * np.einsum("ij,ij->i", Gz, dp_dlam)
    E = np.broadcast_to(np.asarray(E, float), V.shape)
    nu = np.broadcast_to(np.asarray(nu, float), V.shape)
    dE_tet, dnu_tet = lame_chain(dmu_tet, dlam_tet, E, nu)
    dtarget = dE_bind = None
    b = disc.bindings
    if b is not None and len(b.vid):
        zb = z3[b.vid]
        lam_b = -(q.reshape(n_v, 3)[b.vid] - record.targets) / b.E[:, None]
        dtarget = h * h * zb / b.E[:, None]
        dE_bind = -h * h * np.einsum("bk,bk->b", lam_b, zb) / b.E
    return StepGradients(z3.copy(), dqbar, dvbar, dfext, dmu_fric, dmu_tet, dlam_tet, dE_tet, dnu_tet,
                         dtarget, dE_bind)


def adjoint_step(disc: Discretisation, q, record: StepRecord, dL_dq, dL_dv, eps, E, nu,
                 refine: int = 3) -> StepGradients:
    """Full per-step adjoint: assemble, solve Acal^T z = g_q + g_v/h, contract."""
    sysm = assemble(disc, q, record, eps)
    rhs = dL_dq.reshape(-1) + dL_dv.reshape(-1) / disc.h
    z = solve_transposed(sysm.Acal, rhs, refine)
    return vjp(disc, sysm, q, record, z, dL_dv, E, nu)
