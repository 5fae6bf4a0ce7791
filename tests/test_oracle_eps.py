"""Pins for the smoothing parameter (Sec. 5.2 and the forward-backward
smoothing consistency analysis of the appendix), on the slope cube of the
smoothing sweep (Sec. 6, smoothing parameter sensitivity).

* Mismatched smoothing: at a point of the forward's zero set x y = eps_f^2,
  the backward ratio (d phi/dx)/(d phi/dy) evaluated with eps_b != eps_f is
  off by eps_f^2/eps_b^2 on an active row (x ~ eps_f^2, y ~ 1) and by the
  reciprocal on an inactive row (x ~ 1, y ~ eps_f^2), to leading order.
* With matched smoothing the per-step gradients dL/dmu and dL/dE equal
  central finite differences through the converged forward step on the
  sticking and on the sliding cube; with eps_b = 1000 eps_f the sticking
  cube's dL/dmu takes the sliding cube's scale.
* A sticking cube settles at 2 eps^2 = 1e-12 while a sliding one keeps
  accelerating down the slope.
"""

import functools

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import fb
from oracle.forward import solve_step
from oracle.rollout import scene_disc
from synth import slope_scene


@pytest.mark.parametrize("two_eps2_f,two_eps2_b", [(1e-12, 1e-6), (1e-12, 1e-9), (1e-9, 1e-6)])
def test_mismatched_smoothing_scales_rows(two_eps2_f, two_eps2_b):
    ef, eb = np.sqrt(0.5 * two_eps2_f), np.sqrt(0.5 * two_eps2_b)
    for y in (0.3, 1.0, 4.0):
        x = ef * ef / y  # active row on the forward's zero set
        assert abs(float(fb.phi_eps(x, y, ef))) <= 1e-15 * y
        matched = float(fb.ratio(x, y, ef))
        assert matched == pytest.approx(y / x, rel=1e-12)  # y/x on the zero set
        mism = float(fb.ratio(x, y, eb))
        assert mism / matched == pytest.approx(ef * ef / (eb * eb), rel=2e-3)
        # inactive row: roles swapped
        mism_i = float(fb.ratio(y, x, eb))
        matched_i = float(fb.ratio(y, x, ef))
        assert matched_i == pytest.approx(x / y, rel=1e-12)
        assert mism_i / matched_i == pytest.approx(eb * eb / (ef * ef), rel=2e-3)


@functools.lru_cache(maxsize=None)
def _settled(side, two_eps2, steps):
    spec = slope_scene(side, two_eps2)
    disc = scene_disc(spec)
    q, v, warm = spec.q0.copy(), spec.v0.copy(), None
    xs = []
    for _ in range(steps):
        q, v, rec, warm = solve_step(disc, q, v, np.zeros_like(q), spec.gravity, spec.mu, spec.eps, spec.planes,
                                     margin=spec.contact_margin, warm=warm)
        assert rec.residual < 1e-9
        xs.append(float(np.mean(q[:, 0] - spec.q0[:, 0])))
    return spec, disc, q, v, warm, np.array(xs)


def test_stick_settles_and_slip_accelerates():
    _, _, _, _, _, stick = _settled("stick", 1e-12, 30)
    _, _, _, _, _, slip = _settled("slip", 1e-12, 30)
    # stick: over the last ten steps the cube moves less than 1e-3 of its
    # settling shift (what remains is elastic vibration)
    assert abs(stick[-1] - stick[-11]) <= 1e-3 * abs(stick[-1])
    # slip: the down-slope speed grows
    dv = np.diff(slip)
    assert dv[-1] > dv[-11] > 0
    assert slip[-1] > 2 * stick[-1]


def _fd(fun, eta, rec):
    for _ in range(6):
        (lp, rp), (lm, rm) = fun(eta), fun(-eta)
        if all(np.array_equal(r.contacts.vid, rec.contacts.vid) and np.array_equal(r.contacts.fric, rec.contacts.fric)
               for r in (rp, rm)):
            return (lp - lm) / (2 * eta)
        eta /= 10.0
    raise AssertionError("contact state changes under every probe step")


def _step_gradients(side, eps_scale):
    """(adjoint dL/dmu, dL/dE at eps_b = eps_scale * eps_f, FD dL/dmu, FD
    dL/dE) at the step after 30 settling steps."""
    spec, disc, qbar, vbar, warm, _ = _settled(side, 1e-12, 30)
    f = np.zeros_like(qbar)
    rng = np.random.default_rng(31)
    g = spec.loss_dir
    gv = 1e-3 * rng.standard_normal(qbar.shape)

    def loss(mu, d):
        q_, v_, r_, _ = solve_step(d, qbar, vbar, f, spec.gravity, mu, spec.eps, spec.planes,
                                   margin=spec.contact_margin, warm=warm)
        return float(np.sum(g * q_) + np.sum(gv * v_)), r_

    q, v, rec, _ = solve_step(disc, qbar, vbar, f, spec.gravity, spec.mu, spec.eps, spec.planes,
                              margin=spec.contact_margin, warm=warm)
    assert rec.contacts.fric.all()
    fd_mu = _fd(lambda e: loss(spec.mu + e, disc), 1e-6, rec)
    fd_E = _fd(lambda e: loss(spec.mu, scene_disc(spec, E=spec.E + e)), 1e-5 * spec.E, rec)
    out = []
    for k in eps_scale:
        gr = adj.adjoint_step(disc, q, rec, g, gv, k * spec.eps, spec.E, spec.nu)
        out.append((gr.dmu_fric, gr.dE))
    return out, fd_mu, fd_E


@pytest.mark.slow
def test_matched_smoothing_gives_fd_gradient_and_mismatch_erases_regimes():
    """Sliding and sticking cube at 2 eps_f^2 = 1e-12.  Matched smoothing:
    dL/dmu and dL/dE equal central differences through the converged step in
    both regimes, and dL/dmu of the sticking cube is far smaller than that of
    the sliding one.  Backward smoothing 2 eps_b^2 = 1e-6: the sticking
    cube's dL/dmu moves to the sliding cube's scale (the contrast between the
    regimes is lost) and its dL/dE is wrong as well."""
    res = {}
    for side in ("stick", "slip"):
        (matched, mism), fd_mu, fd_E = _step_gradients(side, (1.0, 1000.0))
        print(f"{side}: dL/dmu FD {fd_mu:.6e} matched {matched[0]:.6e} mismatched {mism[0]:.6e}; "
              f"dL/dE FD {fd_E:.6e} matched {matched[1]:.6e} mismatched {mism[1]:.6e}")
        assert abs(matched[0] - fd_mu) <= 1e-4 * abs(fd_mu)
        assert abs(matched[1] - fd_E) <= 1e-5 * abs(fd_E)
        res[side] = (matched, mism)
    (st_m, st_x), (sl_m, sl_x) = res["stick"], res["slip"]
    assert abs(st_m[0]) < 0.05 * abs(sl_m[0])  # matched: the regimes differ by > 20x
    assert abs(st_x[0]) > 0.5 * abs(sl_x[0])  # mismatched: same scale
    assert abs(st_x[0] - st_m[0]) > 10 * abs(st_m[0])
    assert abs(st_x[1] - st_m[1]) > 0.2 * abs(st_m[1])
