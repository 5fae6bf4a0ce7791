"""Smoothed Fischer-Burmeister function (Sec. 5.2; App. A.2).  Test
infrastructure only.

    phi_eps(x, y) = x + y - sqrt(x^2 + y^2 + 2 eps^2)
Its zero set is the positive branch of x y = eps^2.  With r = sqrt(...):
    d phi/dx = 1 - x/r = (r - x)/r,   d phi/dy = 1 - y/r = (r - y)/r
and the contact-Jacobian entries use the ratio (r - x)/(r - y), which equals
y/x on the zero set (Sec. 5.2, eq:diff_fb; App. A.2 writes the general ratio).

``phi_eps_plain`` is the definition as printed.  The other functions evaluate
the same quantities through the algebraically identical forms
    r - x = (y^2 + 2 eps^2)/(r + x)          (x > 0)
    x + y - r = 2 (x y - eps^2)/(x + y + r)  (x + y > 0)
that avoid the cancellation of two nearly equal numbers when one argument is
~1e-12 and the other ~1 (the converged contact regime); tests pin them against
a 50-digit evaluation of the definition.
"""

from __future__ import annotations

import numpy as np


def phi_eps_plain(x, y, eps):
    return x + y - np.sqrt(x * x + y * y + 2.0 * eps * eps)


def _r(x, y, eps):
    return np.sqrt(x * x + y * y + 2.0 * eps * eps)


def r_minus(x, y, eps, r=None):
    """r - x without cancellation."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if r is None:
        r = _r(x, y, eps)
    pos = x > 0
    safe = np.where(pos, (y * y + 2.0 * eps * eps) / np.where(pos, r + x, 1.0), r - x)
    return safe


def phi_eps(x, y, eps):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r = _r(x, y, eps)
    s = x + y
    pos = s > 0
    return np.where(pos, 2.0 * (x * y - eps * eps) / np.where(pos, s + r, 1.0), s - r)


def partials(x, y, eps):
    """(d phi/dx, d phi/dy) = ((r - x)/r, (r - y)/r)."""
    r = _r(np.asarray(x, float), np.asarray(y, float), eps)
    return r_minus(x, y, eps, r) / r, r_minus(y, x, eps, r) / r


def ratio(x, y, eps):
    """(d phi/dx)/(d phi/dy) = (r - x)/(r - y)  (App. A.2: omega/E)."""
    r = _r(np.asarray(x, float), np.asarray(y, float), eps)
    return r_minus(x, y, eps, r) / r_minus(y, x, eps, r)
