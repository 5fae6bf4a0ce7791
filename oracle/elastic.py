"""Local elastic projection and its SVD-based Jacobian (Sec. 5.3; App. B.0-B.4).
Test infrastructure only.

The projection of element i keeps the singular vectors of F = U diag(sigma) V^T
and replaces the singular values by theta(sigma), the minimiser of
Psi = w/2 |theta - sigma|^2 + zeta(theta) with w = 2 mu (App. B.2).  For
Neo-Hookean the optimality condition is
    g(theta) = mu (3 theta - 2 sigma - 1/theta) + lam log(J) / theta = 0,
    J = theta_1 theta_2 theta_3                                  (App. B.3)
solved here by Newton's method from theta = sigma.

Jacobian (App. B.0, main text Sec. 5.3):
    dvecP/dvecF = (V (x) U) [ D W D^T + Diag(vec M) + Diag(vec N) T ] (V (x) U)^T
The printed main-text and appendix formula multiply T by Diag(vec M); the
element-wise derivation in App. B.0 (Y_ij = M_ij X_ij + N_ij X_ji) requires
Diag(vec N) there.  This module uses N (the reading that finite differences
confirm; see tests/test_oracle_elastic.py).

Divided differences: (theta_i - theta_j)/(sigma_i - sigma_j) is evaluated with
the closed form obtained by subtracting the optimality conditions g_i - g_j = 0,
    q_ij = 2 mu / (3 mu + (mu - lam log J) / (theta_i theta_j)),
which is exact for the root theta, free of cancellation, and at sigma_i =
sigma_j equals W_ii - W_ij, the degenerate limit of App. B.4.  Then
    M_ij = (q_ij + (theta_i + theta_j)/(sigma_i + sigma_j)) / 2
    N_ij = (q_ij - (theta_i + theta_j)/(sigma_i + sigma_j)) / 2   (App. B.0)
"""

from __future__ import annotations

import numpy as np

# D x = vec(Diag x), T vec X = vec X^T  (App. B.1, 3D), column-major vec
D3 = np.zeros((9, 3))
for _i in range(3):
    D3[_i + 3 * _i, _i] = 1.0
T3 = np.zeros((9, 9))
for _r in range(3):
    for _c in range(3):
        T3[_r + 3 * _c, _c + 3 * _r] = 1.0


def vec(X: np.ndarray) -> np.ndarray:
    """Column-stacking vec of (..., 3, 3) -> (..., 9)."""
    return np.swapaxes(X, -1, -2).reshape(X.shape[:-2] + (9,))


def unvec(v: np.ndarray) -> np.ndarray:
    return np.swapaxes(v.reshape(v.shape[:-1] + (3, 3)), -1, -2)


def svd3(F: np.ndarray):
    """F = U diag(s) V^T for a batch (n,3,3); requires det F > 0."""
    if np.any(np.linalg.det(F) <= 0):
        raise ValueError("inverted element: det F <= 0")
    U, s, Vh = np.linalg.svd(F)
    return U, s, np.swapaxes(Vh, -1, -2)


def _nh_g(theta, sigma, mu, lam):
    logJ = np.log(theta).sum(axis=-1, keepdims=True)
    return mu[..., None] * (3 * theta - 2 * sigma - 1 / theta) + lam[..., None] * logJ / theta


def _nh_dg_dtheta(theta, mu, lam):
    """dg/dtheta = Diag(3 mu + (mu - lam log J)/theta^2) + lam theta^{-1} theta^{-T} (App. B.2)."""
    logJ = np.log(theta).sum(axis=-1)
    inv = 1.0 / theta
    Dg = 3 * mu[..., None] + (mu - lam * logJ)[..., None] * inv * inv
    H = lam[..., None, None] * inv[..., :, None] * inv[..., None, :]
    idx = np.arange(3)
    H[..., idx, idx] += Dg
    return H


def nh_theta(sigma, mu, lam, tol=1e-15, maxit=60):
    """Newton on g(theta) = 0 from theta = sigma (App. B.3), batched."""
    sigma = np.asarray(sigma, dtype=np.float64)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), sigma.shape[:-1]).copy()
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), sigma.shape[:-1]).copy()
    theta = sigma.copy()
    for _ in range(maxit):
        g = _nh_g(theta, sigma, mu, lam)
        H = _nh_dg_dtheta(theta, mu, lam)
        d = -np.linalg.solve(H, g[..., None])[..., 0]
        step = np.ones(theta.shape[:-1])
        # keep theta > 0 (log J must stay defined)
        while True:
            bad = np.any(theta + step[..., None] * d <= 0, axis=-1)
            if not np.any(bad):
                break
            step[bad] *= 0.5
        theta = theta + step[..., None] * d
        if np.all(np.abs(step[..., None] * d) <= tol * np.abs(theta)):
            break
    # one polishing Newton step at the converged point
    g = _nh_g(theta, sigma, mu, lam)
    H = _nh_dg_dtheta(theta, mu, lam)
    theta = theta - np.linalg.solve(H, g[..., None])[..., 0]
    return theta


class ProjectionRecord:
    """Per-element SVD record: U, sigma, V, theta, W, M, N, dtheta/dmu,
    dtheta/dlam, and the projected P = U diag(theta) V^T."""

    def __init__(self, F, mu, lam, model="nh"):
        F = np.asarray(F, dtype=np.float64)
        batch = F.shape[:-2]
        mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), batch).copy()
        lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), batch).copy()
        U, s, V = svd3(F)
        self.U, self.sigma, self.V = U, s, V
        ones = np.ones_like(s)
        if model == "nh":
            th = nh_theta(s, mu, lam)
            H = _nh_dg_dtheta(th, mu, lam)
            Hinv = np.linalg.inv(H)
            W = 2 * mu[..., None, None] * Hinv  # W = -(dg/dtheta)^{-1} dg/dsigma, dg/dsigma = -2 mu I
            logJ = np.log(th).sum(axis=-1)
            self.dth_dmu = -(Hinv @ (3 * th - 2 * s - 1 / th)[..., None])[..., 0]
            self.dth_dlam = -(Hinv @ (logJ[..., None] / th)[..., None])[..., 0]
            qij = 2 * mu[..., None, None] / (
                3 * mu[..., None, None]
                + (mu - lam * logJ)[..., None, None] / (th[..., :, None] * th[..., None, :])
            )
        elif model == "arap":
            th = ones.copy()
            W = np.zeros(batch + (3, 3))
            qij = np.zeros(batch + (3, 3))
            self.dth_dmu = np.zeros_like(s)
            self.dth_dlam = np.zeros_like(s)
        elif model == "corot":
            Hc = 4 * mu[..., None, None] * np.eye(3) + lam[..., None, None] * np.ones((3, 3))
            Hinv = np.linalg.inv(Hc)
            th = 1 + (Hinv @ (2 * mu[..., None] * (s - 1))[..., None])[..., 0]
            W = 2 * mu[..., None, None] * Hinv
            qij = np.full(batch + (3, 3), 0.5)
            tr = (th - 1).sum(axis=-1, keepdims=True)
            self.dth_dmu = -(Hinv @ (2 * (2 * th - s - 1))[..., None])[..., 0]
            self.dth_dlam = -(Hinv @ (tr * ones)[..., None])[..., 0]
        else:
            raise ValueError(model)
        self.theta, self.W = th, W
        avg = (th[..., :, None] + th[..., None, :]) / (s[..., :, None] + s[..., None, :])
        M = 0.5 * (qij + avg)
        N = 0.5 * (qij - avg)
        idx = np.arange(3)
        M[..., idx, idx] = 0.0
        N[..., idx, idx] = 0.0
        self.M, self.N = M, N
        self.P = U @ (th[..., :, None] * np.swapaxes(V, -1, -2))
        self.mu, self.lam = mu, lam

    def jacobian(self) -> np.ndarray:
        """dvecP/dvecF, (..., 9, 9), literally (V(x)U)[D W D^T + Diag(vecM) + Diag(vecN) T](V(x)U)^T."""
        U, V = self.U, self.V
        K = np.einsum("...ab,...cd->...acbd", V, U).reshape(U.shape[:-2] + (9, 9))
        core = D3 @ self.W @ D3.T
        core = core + _diag_embed(vec(self.M)) + _diag_embed(vec(self.N)) @ T3
        return K @ core @ np.swapaxes(K, -1, -2)

    def dP_dmu(self) -> np.ndarray:
        """U Diag(dtheta/dmu) V^T (App. B.3)."""
        return self.U @ (self.dth_dmu[..., :, None] * np.swapaxes(self.V, -1, -2))

    def dP_dlam(self) -> np.ndarray:
        return self.U @ (self.dth_dlam[..., :, None] * np.swapaxes(self.V, -1, -2))


def _diag_embed(v):
    out = np.zeros(v.shape + (v.shape[-1],))
    idx = np.arange(v.shape[-1])
    out[..., idx, idx] = v
    return out


def project(F, mu, lam, model="nh") -> np.ndarray:
    """P(F) = U diag(theta(sigma)) V^T."""
    return ProjectionRecord(F, mu, lam, model).P
