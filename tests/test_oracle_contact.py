"""Pins for the contact oracle (Sec. 3.2 eq:contact, Sec. 5.2
eq:partial_contact / eq:final_diff_contact, App. A.1)."""

import numpy as np

from oracle import contact as ct

EPS = np.sqrt(0.5e-12)


def _local_law(delta, mu, eps):
    """lambda_c(delta_c) from the three contact rows on their zero set:
    lambda_n = eps^2/delta_n, |lambda_f| = mu lambda_n - eps^2/|delta_f|,
    lambda_f antiparallel to delta_f (eq:contact)."""
    dn, df = delta[0], delta[1:]
    x = np.hypot(*df)
    ln = eps * eps / dn
    s = mu * ln - eps * eps / x
    return np.concatenate([[ln], -s * df / x])


def _one(fric=True):
    return ct.ContactSet(np.array([0], np.int32), np.array([0], np.int32), np.eye(3)[None],
                         np.zeros(1), np.zeros((1, 2)), np.array([fric]))


def test_K_matches_fd_of_local_law():
    rng = np.random.default_rng(0)
    mu = 0.4
    for _ in range(20):
        dn = 10.0 ** rng.uniform(-12.5, -11)  # lambda_n ~ 0.05 .. 0.5 N
        ln = EPS * EPS / dn
        x_min = dn / mu  # s >= 0 needs |delta_f| >= delta_n/mu
        x = x_min * 10.0 ** rng.uniform(0.01, 3)
        ang = rng.uniform(0, 2 * np.pi)
        delta = np.array([dn, x * np.cos(ang), x * np.sin(ang)])
        lam = _local_law(delta, mu, EPS)
        blk = ct.contact_blocks(_one(), delta[None], lam[None], mu, EPS)
        Kfd = np.zeros((3, 3))
        for k in range(3):
            h = 1e-6 * (dn if k == 0 else x)
            d = np.zeros(3)
            d[k] = h
            Kfd[:, k] = -(_local_law(delta + d, mu, EPS) - _local_law(delta - d, mu, EPS)) / (2 * h)
        assert np.abs(blk.K[0] - Kfd).max() <= 1e-6 * np.abs(Kfd).max(), (blk.K[0], Kfd)
        # k_mu = -d lambda/d mu
        dmu = 1e-6
        kfd = -(_local_law(delta, mu + dmu, EPS) - _local_law(delta, mu - dmu, EPS)) / (2 * dmu)
        np.testing.assert_allclose(blk.kmu[0], kfd, rtol=1e-6, atol=1e-12 * ln)


def test_frictionless_block_is_diag():
    """mu = 0: R K R^T = Diag(lambda_n/delta_n, 0, 0) (Sec. 5.4 frictionless)."""
    dn = 2e-12
    ln = EPS * EPS / dn
    blk = ct.contact_blocks(_one(False), np.array([[dn, 0.0, 0.0]]), np.array([[ln, 0, 0]]), 0.0, EPS)
    np.testing.assert_allclose(blk.K[0], np.diag([ln / dn, 0, 0]), rtol=1e-14)


def test_rotation_rule():
    """App. A.1: R from lambda_f if it exceeds tau, else delta_f, else I;
    R delta = [delta_n, |delta_f|, 0] and R lambda = [lambda_n, -|lambda_f|, 0]."""
    delta = np.array([1e-12, 3e-9, -4e-9])
    lam = np.array([0.5, -0.3, 0.4])
    blk = ct.contact_blocks(_one(), delta[None], lam[None], 1.0, EPS)
    R = blk.R[0]
    np.testing.assert_allclose(R @ delta, [1e-12, 5e-9, 0.0], atol=1e-24)
    np.testing.assert_allclose(R @ lam, [0.5, -0.5, 0.0], atol=1e-15)
    blk = ct.contact_blocks(_one(), delta[None], np.array([[0.5, 0.0, 0.0]]), 1.0, EPS)
    np.testing.assert_allclose(blk.R[0] @ delta, [1e-12, 5e-9, 0.0], atol=1e-24)
    blk = ct.contact_blocks(_one(), np.array([[1e-12, 0.0, 0.0]]), np.array([[0.5, 0.0, 0.0]]), 1.0, EPS)
    np.testing.assert_array_equal(blk.R[0], np.eye(3))


def test_tangent_frame_orthonormal_right_handed():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        F = ct.tangent_frame(n)
        np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-15)
        assert np.linalg.det(F) > 0
    np.testing.assert_array_equal(ct.tangent_frame(np.array([0.0, 0.0, 1.0])),
                                  [[0, 0, 1], [0, 1, 0], [-1, 0, 0]])


def test_detection_brute_force():
    """Candidates: predicted gap <= margin; normal-only when the gap is > 0."""
    rng = np.random.default_rng(2)
    q = rng.uniform(-0.01, 0.01, size=(200, 3))
    planes = np.array([[0.0, 0.0, 1.0, 0.0]])
    cs = ct.detect(q, q, planes, np.zeros((0, 4)), np.zeros((0, 4)), 2e-3)
    expect = np.nonzero(q[:, 2] <= 2e-3)[0]
    np.testing.assert_array_equal(cs.vid, expect)
    np.testing.assert_array_equal(cs.fric, q[expect, 2] <= 0)
