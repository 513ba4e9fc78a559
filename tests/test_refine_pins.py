"""Pins of the refinement oracle (oracle/refine.py), CPU only.

* integer sample positions reduce bilinear stacking to the plain
  shift-and-stack of the search (oracle O3), PSF-weighted over the cutout;
* on linear-ramp frames bilinear sampling is exact, so SN and its gradient
  have closed forms (ramp variance (w^2 - 1)/12 per unit slope);
* central finite differences agree with the analytic gradient away from
  pixel boundaries;
* ascent from a jittered start on a noise-free mover raises SN and moves
  toward the true track;
* planted mistakes (no dt in the velocity gradient, fractional offsets
  taken from the wrong pixel) fail the pins.
"""

import math

import numpy as np
import pytest

from oracle import refine
from oracle import sst_oracle as so


def test_integer_positions_reduce_to_plain_stack():
    rng = np.random.default_rng(1)
    n, h, w = 5, 30, 40
    f = rng.normal(3, 1, size=(n, h, w)).astype(np.float32)
    t = np.arange(n, dtype=np.float64)
    x0, y0, vx, vy = 14, 11, 2, -1
    C = 7
    sn, _ = refine.objective(f, t, 0.0, [x0, y0, vx, vy], cutout=C, fwhm=2.0)
    b, s2 = so.frame_stats(f)
    S, c, _ = so.stack_velocity(f, vx * t.astype(np.int64), vy * t.astype(np.int64), offsets=b)
    wts = refine.psf_weights(C, 2.0)
    R = C // 2
    num = float((wts * S[y0 - R:y0 + R + 1, x0 - R:x0 + R + 1]).sum())
    want = num / math.sqrt(float((wts ** 2).sum()) * float(s2.sum()))
    assert sn == pytest.approx(want, rel=1e-12, abs=1e-12)


def _ramp_frames(n, h, w, a, b, c):
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    return np.stack([a[i] * xx + b[i] * yy + c[i] for i in range(n)]).astype(np.float32)


def test_linear_ramps_closed_form():
    n, h, w = 4, 40, 48
    a = np.array([0.5, -0.25, 1.0, 0.125])
    b = np.array([0.25, 0.5, -0.75, 0.0])
    c = np.array([3.0, -2.0, 0.5, 7.0])
    f = _ramp_frames(n, h, w, a, b, c)
    t = np.array([0.0, 0.35, 0.9, 1.6])
    th = np.array([20.3, 17.65, 2.4, -1.3])
    C, fwhm = 9, 2.5
    sn, g = refine.objective(f, t, 0.2, th, cutout=C, fwhm=fwhm)
    wts = refine.psf_weights(C, fwhm)
    xc, yc = (w - 1) / 2.0, (h - 1) / 2.0
    dt = t - 0.2
    var = a ** 2 * (w * w - 1) / 12.0 + b ** 2 * (h * h - 1) / 12.0
    norm = math.sqrt(float((wts ** 2).sum()) * float(var.sum()))
    W = float(wts.sum())
    num = W * float(np.sum(a * (th[0] + th[2] * dt - xc) + b * (th[1] + th[3] * dt - yc)))
    assert sn == pytest.approx(num / norm, rel=1e-12)
    want = np.array([a.sum(), b.sum(), (a * dt).sum(), (b * dt).sum()]) * W / norm
    assert np.allclose(g, want, rtol=1e-12, atol=1e-14)


def test_finite_differences_agree():
    rng = np.random.default_rng(2)
    f = rng.normal(0, 1, size=(6, 40, 50)).astype(np.float32)
    t = np.arange(6) * 0.3
    th = np.array([20.3, 17.6, 3.2, -1.7])
    sn, g, m = refine.objective(f, t, 0.0, th, cutout=9, absolute=True)
    h = 1e-6
    assert m["kink"] > 10 * h * (1 + 1.5)
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        fd = (refine.objective(f, t, 0.0, th + e, cutout=9)[0] - refine.objective(f, t, 0.0, th - e, cutout=9)[0]) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-8)


def test_ascent_on_noise_free_mover():
    n, h, w = 12, 48, 64
    t = np.linspace(0, 2.0, n)
    truth = np.array([30.2, 22.7, 4.3, -2.6])
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    s = 2.5 / (2 * math.sqrt(2 * math.log(2)))
    f = np.stack([10 * np.exp(-((xx - truth[0] - truth[2] * ti) ** 2 + (yy - truth[1] - truth[3] * ti) ** 2)
                              / (2 * s * s)) for ti in t]).astype(np.float32)
    f += np.random.default_rng(3).normal(0, 0.01, size=f.shape).astype(np.float32)
    start = truth + np.array([0.4, -0.3, 0.25, 0.2])
    th, sn, g, path = refine.ascend(f, t, 0.0, start, steps=40, lr=0.005, cutout=15)
    assert path[-1] > path[0]
    assert np.linalg.norm(th - truth) < 0.5 * np.linalg.norm(start - truth)


def test_planted_missing_dt_is_caught(monkeypatch):
    real = refine.objective

    def bad(*args, **kw):
        out = real(*args, **kw)
        g = out[1].copy()
        g[2], g[3] = g[0], g[1]
        return (out[0], g) + tuple(out[2:])
    monkeypatch.setattr(refine, "objective", bad)
    with pytest.raises(AssertionError):
        test_linear_ramps_closed_form()


def test_planted_flipped_fraction_is_caught(monkeypatch):
    real_floor = np.floor
    monkeypatch.setattr(refine.np, "floor", lambda x: real_floor(x) + 1)  # fx -> fx - 1
    # (linear ramps cannot see it: any affine combination reproduces them)
    with pytest.raises(AssertionError):
        test_integer_positions_reduce_to_plain_stack()


def pin_psf_weights():
    """The Gaussian weights against facts that fix them: the centre weight
    is 1; a FWHM of 4 px puts weight 1/2 exactly 2 px from the centre along
    either axis and 1/4 on the diagonal there (the 2-D Gaussian is the
    product of two 1-D ones); the grid is symmetric; and the sum of squared
    weights over a wide cutout is the integral pi s^2 with s = FWHM /
    (2 sqrt(2 ln 2)) (Poisson summation: the lattice sum of exp(-u^2/s^2)
    equals sqrt(pi) s up to terms of order exp(-pi^2 s^2))."""
    wts = refine.psf_weights(9, 4.0)
    R = 4
    assert wts.shape == (9, 9)
    assert wts[R, R] == 1.0
    for dy, dx in ((0, 2), (0, -2), (2, 0), (-2, 0)):
        assert wts[R + dy, R + dx] == pytest.approx(0.5, rel=1e-14)
    assert wts[R + 2, R + 2] == pytest.approx(0.25, rel=1e-14)
    assert np.array_equal(wts, wts.T) and np.array_equal(wts, wts[::-1]) and np.array_equal(wts, wts[:, ::-1])
    assert np.all(wts > 0) and np.all(wts <= 1)
    fwhm = 6.0
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    w33 = refine.psf_weights(33, fwhm)
    assert float((w33 ** 2).sum()) == pytest.approx(math.pi * s * s, rel=1e-12)


def test_psf_weights_closed_forms():
    pin_psf_weights()


def test_planted_fwhm_as_sigma_is_caught(monkeypatch):
    def bad(cutout, fwhm):
        r = cutout // 2
        u = np.arange(-r, r + 1, dtype=np.float64)
        return np.exp(-(u[None, :] ** 2 + u[:, None] ** 2) / (2.0 * fwhm * fwhm))
    monkeypatch.setattr(refine, "psf_weights", bad)
    with pytest.raises(AssertionError):
        pin_psf_weights()
