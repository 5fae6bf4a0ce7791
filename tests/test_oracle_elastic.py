"""Pins for the SVD projection Jacobian oracle (Sec. 5.3; App. B.0-B.4)."""

import numpy as np
import pytest

from conftest import load_golden
from oracle.elastic import D3, T3, ProjectionRecord, nh_theta, project, unvec, vec

MU, LAM = 3.4e5, 3.1e6  # nu = 0.45 at E ~ 1e6


def _rand_F(rng, scale=0.3):
    while True:
        F = np.eye(3) + scale * rng.standard_normal((3, 3))
        if np.linalg.det(F) > 0.2:
            return F


def _rot(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def _fd_jacobian(F, model, eta=1e-6):
    J = np.zeros((9, 9))
    for k in range(9):
        d = np.zeros(9)
        d[k] = eta
        Pp = project(unvec(vec(F) + d)[None], MU, LAM, model)[0]
        Pm = project(unvec(vec(F) - d)[None], MU, LAM, model)[0]
        J[:, k] = (vec(Pp) - vec(Pm)) / (2 * eta)
    return J


def test_permutation_matrices_match_appendix():
    g = load_golden("permutation_matrices_appB1.txt")
    np.testing.assert_array_equal(D3, g["D3"])
    np.testing.assert_array_equal(T3, g["T3"])
    X = np.arange(9.0).reshape(3, 3)
    np.testing.assert_array_equal(D3 @ np.array([1.0, 2, 3]), vec(np.diag([1.0, 2, 3])))
    np.testing.assert_array_equal(T3 @ vec(X), vec(X.T))


@pytest.mark.parametrize("model", ["nh", "arap", "corot"])
def test_jacobian_matches_central_differences(model):
    rng = np.random.default_rng(7)
    for _ in range(4):
        F = _rand_F(rng)
        J = ProjectionRecord(F[None], MU, LAM, model).jacobian()[0]
        Jfd = _fd_jacobian(F, model)
        assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(J).max()


def test_printed_M_in_place_of_N_fails_fd():
    """The printed Diag(vec M) T term contradicts finite differences; the
    derivation's Diag(vec N) T agrees (reading of Sec. 5.3 / App. B.0)."""
    rng = np.random.default_rng(8)
    F = _rand_F(rng)
    rec = ProjectionRecord(F[None], MU, LAM)
    K = np.kron(rec.V[0], rec.U[0])
    diag = lambda v: np.diag(v)  # noqa: E731
    printed = K @ (D3 @ rec.W[0] @ D3.T + diag(vec(rec.M[0])) + diag(vec(rec.M[0])) @ T3) @ K.T
    Jfd = _fd_jacobian(F, "nh")
    assert np.abs(printed - Jfd).max() > 1e-2 * np.abs(Jfd).max()
    assert np.abs(rec.jacobian()[0] - Jfd).max() <= 1e-7 * np.abs(Jfd).max()


def test_jacobian_symmetric():
    rng = np.random.default_rng(9)
    F = _rand_F(rng, 0.5)
    J = ProjectionRecord(F[None], MU, LAM).jacobian()[0]
    np.testing.assert_allclose(J, J.T, atol=1e-14 * np.abs(J).max())


def test_rest_state_closed_forms():
    """theta(1) = 1, P(I) = I; at rest W = (I - lam/(4mu+3lam) 1 1^T)/2,
    M_ij = 3/4, N_ij = -1/4 (App. B.2, B.4)."""
    rec = ProjectionRecord(np.eye(3)[None], MU, LAM)
    np.testing.assert_allclose(rec.theta[0], 1.0, atol=1e-15)
    np.testing.assert_allclose(rec.P[0], np.eye(3), atol=1e-15)
    W = 0.5 * (np.eye(3) - LAM / (4 * MU + 3 * LAM) * np.ones((3, 3)))
    np.testing.assert_allclose(rec.W[0], W, rtol=1e-13)
    off = ~np.eye(3, dtype=bool)
    np.testing.assert_allclose(rec.M[0][off], 0.75, rtol=1e-13)
    np.testing.assert_allclose(rec.N[0][off], -0.25, rtol=1e-13)


def test_arap_equals_polar_derivative():
    """theta = 1: dP is the derivative of the polar rotation,
    U [(X_ij - X_ji)/(sigma_i + sigma_j)] V^T with X = U^T dF V."""
    rng = np.random.default_rng(10)
    F = _rand_F(rng)
    rec = ProjectionRecord(F[None], MU, LAM, "arap")
    U, s, V = rec.U[0], rec.sigma[0], rec.V[0]
    J = rec.jacobian()[0]
    for _ in range(3):
        dF = rng.standard_normal((3, 3))
        X = U.T @ dF @ V
        Y = (X - X.T) / (s[:, None] + s[None, :])
        np.testing.assert_allclose(J @ vec(dF), vec(U @ Y @ V.T), atol=1e-12)


def test_corot_W_constant():
    """Co-rotational: W = I/2 - lam/(2(4mu+3lam)) 1 1^T for any F (App. B.2)."""
    rng = np.random.default_rng(11)
    rec = ProjectionRecord(_rand_F(rng)[None], MU, LAM, "corot")
    W = 0.5 * np.eye(3) - LAM / (2 * (4 * MU + 3 * LAM)) * np.ones((3, 3))
    np.testing.assert_allclose(rec.W[0], W, rtol=1e-12)


def test_isotropy_and_gauge():
    """P(R F Q) = R P(F) Q for rotations R, Q; J transforms alike."""
    rng = np.random.default_rng(12)
    F = _rand_F(rng)
    R, Q = _rot(rng), _rot(rng)
    P = project(F[None], MU, LAM)[0]
    P2 = project((R @ F @ Q)[None], MU, LAM)[0]
    np.testing.assert_allclose(P2, R @ P @ Q, atol=1e-13)
    J = ProjectionRecord(F[None], MU, LAM).jacobian()[0]
    J2 = ProjectionRecord((R @ F @ Q)[None], MU, LAM).jacobian()[0]
    dF = rng.standard_normal((3, 3))
    np.testing.assert_allclose(unvec(J2 @ vec(R @ dF @ Q)), R @ unvec(J @ vec(dF)) @ Q, atol=1e-12)


def test_degenerate_limit_is_continuous():
    """At sigma_i = sigma_j the closed form equals the limit (App. B.4)."""
    rng = np.random.default_rng(13)
    R, Q = _rot(rng), _rot(rng)
    Fd = R @ np.diag([1.1, 1.1, 0.9]) @ Q
    J0 = ProjectionRecord(Fd[None], MU, LAM).jacobian()[0]
    Fp = R @ np.diag([1.1 + 1e-7, 1.1, 0.9]) @ Q
    J1 = ProjectionRecord(Fp[None], MU, LAM).jacobian()[0]
    assert np.abs(J0 - J1).max() <= 1e-6 * np.abs(J0).max()
    assert np.abs(J0 - _fd_jacobian(Fd, "nh")).max() <= 1e-6 * np.abs(J0).max()
    rec = ProjectionRecord(Fd[None], MU, LAM)
    W = rec.W[0]
    i, j = 0, 1
    th, sg = rec.theta[0][0], rec.sigma[0][0]
    assert abs(rec.M[0][i, j] - 0.5 * (W[i, i] - W[i, j] + th / sg)) < 1e-12
    assert abs(rec.N[0][i, j] - 0.5 * (W[i, i] - W[i, j] - th / sg)) < 1e-12


def test_W_and_parameter_derivatives_match_fd():
    """W = dtheta/dsigma (App. B.2) and dtheta/dmu, dtheta/dlam (App. B.3)."""
    s = np.array([1.2, 0.95, 0.8])  # descending, the order numpy's SVD returns
    rec = ProjectionRecord(np.diag(s)[None], MU, LAM)
    th = lambda sg, mu=MU, lam=LAM: nh_theta(sg[None], mu, lam)[0]  # noqa: E731
    for k in range(3):
        d = np.zeros(3)
        d[k] = 1e-6
        col = (th(s + d) - th(s - d)) / 2e-6
        np.testing.assert_allclose(rec.W[0][:, k], col, rtol=1e-6, atol=1e-9)
    dmu = (th(s, MU * (1 + 1e-6)) - th(s, MU * (1 - 1e-6))) / (2e-6 * MU)
    dlam = (th(s, MU, LAM * (1 + 1e-6)) - th(s, MU, LAM * (1 - 1e-6))) / (2e-6 * LAM)
    np.testing.assert_allclose(rec.dth_dmu[0], dmu, rtol=1e-5)
    np.testing.assert_allclose(rec.dth_dlam[0], dlam, rtol=1e-5)
    # the paper's Sherman-Morrison form of W
    t = rec.theta[0]
    logJ = np.log(t).sum()
    Dg = np.diag(3 * MU + (MU - LAM * logJ) / t ** 2)
    Di = np.linalg.inv(Dg)
    u = 1 / t
    W_sm = 2 * MU * Di @ (np.eye(3) - LAM * np.outer(u, u) / (1 + LAM * u @ Di @ u) @ Di.T)
    np.testing.assert_allclose(rec.W[0], W_sm, rtol=1e-12)
