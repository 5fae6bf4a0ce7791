"""Pins for the smoothed Fischer-Burmeister oracle (Sec. 5.2, App. A.2)."""

import mpmath
import numpy as np
import pytest

from oracle import fb

EPS = np.sqrt(0.5e-12)
mpmath.mp.dps = 60


def _mp_phi(x, y, eps):
    x, y, e = mpmath.mpf(x), mpmath.mpf(y), mpmath.mpf(eps)
    return x + y - mpmath.sqrt(x * x + y * y + 2 * e * e)


def _mp_ratio(x, y, eps):
    x, y, e = mpmath.mpf(x), mpmath.mpf(y), mpmath.mpf(eps)
    r = mpmath.sqrt(x * x + y * y + 2 * e * e)
    return (1 - x / r) / (1 - y / r)


def _samples(rng, n=400):
    mags = 10.0 ** rng.uniform(-14, 1, size=(n, 2))
    signs = rng.choice([-1.0, 1.0], size=(n, 2))
    return mags * signs


def test_zero_set_is_positive_branch_of_xy_eps2():
    """phi_eps(x, y) = 0 exactly on x y = eps^2 with x, y > 0 (Sec. 5.2)."""
    rng = np.random.default_rng(0)
    x = 10.0 ** rng.uniform(-13, 1, size=200)
    y = EPS * EPS / x
    for xi, yi in zip(x, y):
        assert abs(float(_mp_phi(xi, yi, EPS))) <= 1e-15 * (xi + yi)
        assert abs(fb.phi_eps(xi, yi, EPS)) <= 1e-15 * (xi + yi)
    # the negative branch x y = eps^2, x, y < 0 is not a zero: phi = 2 (x + y)
    assert np.all(fb.phi_eps(-x, -y, EPS) < 0)
    np.testing.assert_allclose(fb.phi_eps(-x, -y, EPS), 2 * (-x - y), rtol=1e-12)


def test_hard_fb_complementarity():
    """eps = 0: phi = 0 iff x >= 0, y >= 0, x y = 0 (Sec. 3.2)."""
    vals = [-1.0, -1e-3, -0.0, 0.0, 1e-3, 2.0]
    for x in vals:
        for y in vals:
            zero = fb.phi_eps_plain(x, y, 0.0) == 0.0
            comp = (x >= 0) and (y >= 0) and (x * y == 0)
            assert zero == comp, (x, y)


@pytest.mark.parametrize("seed", [1, 2])
def test_stable_forms_match_high_precision_definition(seed):
    rng = np.random.default_rng(seed)
    pts = _samples(rng)
    for x, y in pts:
        ref = float(_mp_phi(x, y, EPS))
        got = float(fb.phi_eps(x, y, EPS))
        assert abs(got - ref) <= 4e-16 * max(abs(ref), 1e-300) + 1e-300 or abs(got - ref) <= 1e-15 * abs(ref), (x, y, got, ref)
        rr = float(_mp_ratio(x, y, EPS))
        rg = float(fb.ratio(x, y, EPS))
        assert abs(rg - rr) <= 1e-14 * abs(rr), (x, y, rg, rr)


def test_partials_on_zero_set():
    """On x y = eps^2: d phi/dx = y/(x+y), d phi/dy = x/(x+y) (eq:diff_fb)
    and the ratio equals y/x (App. A.2)."""
    x = 10.0 ** np.linspace(-12, 0, 25)
    y = EPS * EPS / x
    px, py = fb.partials(x, y, EPS)
    np.testing.assert_allclose(px, y / (x + y), rtol=1e-13)
    np.testing.assert_allclose(py, x / (x + y), rtol=1e-13)
    np.testing.assert_allclose(fb.ratio(x, y, EPS), y / x, rtol=1e-13)


def test_partials_match_finite_differences():
    rng = np.random.default_rng(3)
    eps = 1e-2
    for _ in range(50):
        x, y = rng.uniform(-1, 1, 2)
        px, py = fb.partials(x, y, eps)
        d = 1e-6
        fx = (fb.phi_eps_plain(x + d, y, eps) - fb.phi_eps_plain(x - d, y, eps)) / (2 * d)
        fy = (fb.phi_eps_plain(x, y + d, eps) - fb.phi_eps_plain(x, y - d, eps)) / (2 * d)
        assert abs(px - fx) < 1e-8 and abs(py - fy) < 1e-8
