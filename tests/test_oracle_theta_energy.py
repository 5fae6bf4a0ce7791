"""Pin of the Neo-Hookean prox singular values theta(sigma) against the energy
that defines them (App. B.2).

theta is the minimiser of
    Psi(theta; sigma) = w/2 |theta - sigma|^2 + zeta(theta),   w = 2 mu,
    zeta(theta) = mu/2 (I1 - log I3 - 3) + lam/8 (log I3)^2,
    I1 = sum theta_k^2,  I3 = J^2,  J = theta_1 theta_2 theta_3.
Here Psi is written from that printed energy alone and minimised in 50-digit
arithmetic by Newton's method whose gradient and Hessian are high-precision
numerical derivatives of Psi (no hand-derived optimality condition), so a
misreading of the oracle's closed-form g(theta) cannot cancel out."""

import mpmath
import numpy as np
import pytest

from oracle.elastic import nh_theta


def _psi(th, sig, mu, lam):
    I1 = sum(t * t for t in th)
    J = th[0] * th[1] * th[2]
    logI3 = mpmath.log(J * J)
    zeta = mu / 2 * (I1 - logI3 - 3) + lam / 8 * logI3 ** 2
    w = 2 * mu
    return w / 2 * sum((t - s) ** 2 for t, s in zip(th, sig)) + zeta


def _grad_hess(f, x):
    n = len(x)
    g = mpmath.matrix(n, 1)
    H = mpmath.matrix(n, n)
    for i in range(n):
        o = [0] * n
        o[i] = 1
        g[i] = mpmath.diff(f, x, tuple(o))
        for j in range(i, n):
            o2 = [0] * n
            o2[i] += 1
            o2[j] += 1
            H[i, j] = H[j, i] = mpmath.diff(f, x, tuple(o2))
    return g, H


def _minimise_psi(sigma, mu, lam):
    """Damped Newton on numerical derivatives of Psi, 50 digits."""
    with mpmath.workdps(50):
        sig = [mpmath.mpf(float(s)) for s in sigma]
        mu_, lam_ = mpmath.mpf(float(mu)), mpmath.mpf(float(lam))

        def f(*th):
            return _psi(th, sig, mu_, lam_)

        x = list(sig)
        for _ in range(60):
            g, H = _grad_hess(f, x)
            d = mpmath.lu_solve(H, -g)
            step = mpmath.mpf(1)
            while True:
                xn = [x[k] + step * d[k] for k in range(3)]
                if min(xn) > 0 and f(*xn) <= f(*x):
                    break
                step /= 2
            x = xn
            if mpmath.norm(d) * step < mpmath.mpf(10) ** -35:
                break
        g, H = _grad_hess(f, x)
        eig = mpmath.eigsy(H)[0]
        return np.array([float(t) for t in x]), float(mpmath.norm(g)), min(float(e) for e in eig)


SIGMAS = [
    (1.3, 0.8, 0.95),        # mixed stretch / compression
    (0.6, 1.4, 1.1),
    (0.7, 0.7, 0.7),         # uniform compression (triple degenerate)
    (1.25, 1.25 + 1e-9, 0.9),  # near-degenerate pair
    (0.5, 0.5, 1.9),         # exactly degenerate pair, large stretch
    (0.3, 2.5, 1.0),         # strong deformation
    (1.0, 1.0, 1.0),         # rest
]


@pytest.mark.parametrize("nu", [0.3, 0.45, 0.48])
@pytest.mark.parametrize("sigma", SIGMAS)
def test_theta_minimises_printed_energy(sigma, nu):
    E = 1e6
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    ref, gnorm, hmin = _minimise_psi(sigma, mu, lam)
    assert hmin > 0  # a strict local minimum of Psi
    th = nh_theta(np.array([sigma]), mu, lam)[0]
    err = np.max(np.abs(th - ref) / np.abs(ref))
    assert err <= 1e-12, (th, ref, err)


def test_pin_rejects_a_plausible_misreading():
    """The root of the condition with lam log J theta (in place of
    lam log J / theta) coincides at rest but misses the minimiser away from
    it: the pin above would catch that mistake."""
    sigma, mu, lam = np.array([1.3, 0.8, 0.95]), 3.4e5, 3.1e6
    ref, _, _ = _minimise_psi(sigma, mu, lam)
    th = sigma.copy()
    for _ in range(100):
        logJ = np.log(th).sum()
        g = mu * (3 * th - 2 * sigma - 1 / th) + lam * logJ * th
        Hm = np.diag(mu * (3 + 1 / th ** 2) + lam * logJ) + lam * np.outer(th, 1 / th)
        th = th - np.linalg.solve(Hm, g)
    logJ = np.log(th).sum()
    g = mu * (3 * th - 2 * sigma - 1 / th) + lam * logJ * th
    assert np.max(np.abs(g)) <= 1e-8 * mu  # th is a root of the misread condition
    assert np.max(np.abs(th - ref) / ref) > 1e-4
