"""Sub-pixel refinement of a detection (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by tests and the benchmark, never by the
GPU library.

The paper's tracks come back with a motion and a pixel position on the trial
grid (Sec. 2.1); this step refines them continuously.  For a candidate
theta = (x0, y0, vx, vy), a C x C cutout (C odd, R = C // 2) is stacked with
bilinear sub-pixel sampling along the linear track:

  C(u, v) = sum_i  bilin(G_i; x0 + u + vx dt_i, y0 + v + vy dt_i),
            u, v in [-R, R],  dt_i = t_i - t_ref,
  G_i     = F_i - b_i inside the frame, 0 outside (out-of-frame samples add
            nothing, as in the search),
  bilin(G; X, Y) with ix = floor(X), fx = X - ix (likewise y):
            (1-fx)(1-fy) G[iy][ix] + fx(1-fy) G[iy][ix+1]
          + (1-fx) fy G[iy+1][ix] + fx fy G[iy+1][ix+1].

The objective is a PSF-weighted S/N with a parameter-free normaliser:

  SN(theta) = sum_{u,v} w(u,v) C(u,v) / sqrt( sum_{u,v} w(u,v)^2 * sum_i s2_i ),
  w(u,v) = exp(-(u^2 + v^2) / (2 s^2)),  s = FWHM / (2 sqrt(2 ln 2)).

Its gradient is exact almost everywhere (bilinear interpolation is piecewise
linear in the sample position; at integer sample positions the formula
above, with ix = floor(X), gives the derivative from the right):

  d bilin / dX = (1-fy)(G[iy][ix+1] - G[iy][ix]) + fy (G[iy+1][ix+1] - G[iy+1][ix])
  d bilin / dY = (1-fx)(G[iy+1][ix] - G[iy][ix]) + fx (G[iy+1][ix+1] - G[iy][ix+1])
  dSN/dx0 = sum w dbilin/dX / norm,   dSN/dvx = sum dt_i w dbilin/dX / norm, ...

Refinement is plain gradient ascent, theta <- theta + lr * grad SN(theta),
for a given number of steps.
"""

from __future__ import annotations

import math

import numpy as np

from .sst_oracle import frame_stats


def psf_weights(cutout: int, fwhm: float) -> np.ndarray:
    """[C][C] float64 Gaussian weights, index [v + R][u + R]."""
    r = cutout // 2
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    u = np.arange(-r, r + 1, dtype=np.float64)
    return np.exp(-(u[None, :] ** 2 + u[:, None] ** 2) / (2.0 * s * s))


def _gather(G: np.ndarray, iy: np.ndarray, ix: np.ndarray) -> np.ndarray:
    h, w = G.shape
    ok = (ix >= 0) & (ix < w) & (iy >= 0) & (iy < h)
    out = np.zeros(ix.shape, np.float64)
    out[ok] = G[iy[ok], ix[ok]]
    return out


def objective(frames: np.ndarray, t, t_ref: float, theta, cutout: int = 33, fwhm: float = 2.5,
              stats=None, absolute: bool = False):
    """SN(theta) and its gradient (4,) in float64.

    With absolute=True also returns magnitude sums (divided by the
    normaliser) used by tolerance checks: 'A' = sum of the |terms| of the
    numerator, 'Ag' = the same for the gradient (times 1 + |dt|), 'L' =
    sum of |w dbilin/dX| + |w dbilin/dY| times 1 + |dt| (how far SN can move
    per unit of parameter change), 'kink' = the smallest distance of any
    frame's fractional sample offset to a pixel boundary (0 or 1)."""
    f = np.asarray(frames, np.float64)
    n = f.shape[0]
    b, s2 = frame_stats(frames) if stats is None else stats
    x0, y0, vx, vy = (float(v) for v in theta)
    wts = psf_weights(cutout, fwhm)
    r = cutout // 2
    U, V = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1))
    norm = math.sqrt(float((wts ** 2).sum()) * float(np.sum(s2)))
    num = gx = gy = gvx = gvy = 0.0
    A = Ag = L = 0.0
    kink = 1.0
    t = np.asarray(t, np.float64)
    for i in range(n):
        dt = t[i] - t_ref
        G = f[i] - b[i]
        X = x0 + vx * dt + U
        Y = y0 + vy * dt + V
        ix = np.floor(X).astype(np.int64)
        iy = np.floor(Y).astype(np.int64)
        fx = X - ix
        fy = Y - iy
        g00 = _gather(G, iy, ix)
        g01 = _gather(G, iy, ix + 1)
        g10 = _gather(G, iy + 1, ix)
        g11 = _gather(G, iy + 1, ix + 1)
        val = (1 - fx) * (1 - fy) * g00 + fx * (1 - fy) * g01 + (1 - fx) * fy * g10 + fx * fy * g11
        dX = (1 - fy) * (g01 - g00) + fy * (g11 - g10)
        dY = (1 - fx) * (g10 - g00) + fx * (g11 - g01)
        num += float((wts * val).sum())
        tx = float((wts * dX).sum())
        ty = float((wts * dY).sum())
        gx += tx
        gy += ty
        gvx += dt * tx
        gvy += dt * ty
        if absolute:
            a00, a01, a10, a11 = np.abs(g00), np.abs(g01), np.abs(g10), np.abs(g11)
            A += float((wts * ((1 - fx) * (1 - fy) * a00 + fx * (1 - fy) * a01 + (1 - fx) * fy * a10
                               + fx * fy * a11)).sum())
            Ag += float((wts * (a00 + a01 + a10 + a11)).sum()) * (1.0 + abs(dt))
            L += float(np.abs(wts * dX).sum() + np.abs(wts * dY).sum()) * (1.0 + abs(dt))
            kink = min(kink, float(min(fx.min(), 1 - fx.max(), fy.min(), 1 - fy.max())))
    sn = num / norm
    grad = np.array([gx, gy, gvx, gvy]) / norm
    if absolute:
        return sn, grad, {"A": A / norm, "Ag": Ag / norm, "L": L / norm, "kink": kink, "norm": norm}
    return sn, grad


def ascend(frames: np.ndarray, t, t_ref: float, theta, steps: int, lr: float, cutout: int = 33,
           fwhm: float = 2.5):
    """Gradient ascent: returns (theta_final, SN(theta_final), grad(theta_final), SN path)."""
    stats = frame_stats(frames)
    th = np.asarray(theta, np.float64).copy()
    path = []
    for _ in range(steps):
        sn, g = objective(frames, t, t_ref, th, cutout, fwhm, stats)
        path.append(sn)
        th = th + lr * g
    sn, g = objective(frames, t, t_ref, th, cutout, fwhm, stats)
    path.append(sn)
    return th, sn, g, np.array(path)
