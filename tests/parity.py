"""Comparison of GPU results with the float64 oracle (test helper).

Tolerances follow from the float32 arithmetic of the GPU path, with u = 2^-24:

* stacked flux: every sample is (F - b32) rounded once (b32 = float32 of the
  background), then N such terms are summed in float32 in some order, so
      |S_gpu - S| <= (N u) A'(p) + c u max|b|  (+ second order),
  with A'(p) = sum of |F - b| over the pixel's in-frame samples.  For the
  plain stack without background subtraction this is N u A(p) <= 1e-5 A(p)
  for N <= 167, the 1e-5 relative target; A(p) makes the bound meaningful
  where the sum itself is near zero;
* S/N: the flux error divided by sqrt(V), plus a few ulp from the float32
  conversion of V, rsqrt and the product: eps(p) = dS/sqrt(V) + 4 u |SN|.

A candidate decision (S/N against the threshold, S/N against a neighbour, order
against another candidate) whose float64 margin is within the summed eps of the
pixels involved may come out either way in float32: such decisions are
"marginal" and are counted, not failed.  Everything else must match exactly.
"""

from __future__ import annotations

import numpy as np

U = 2.0 ** -24
SAFETY = 2.0


def flux_bound(n: int, A: np.ndarray, c: np.ndarray, bmax: float) -> np.ndarray:
    return SAFETY * (n * U * A + c * U * bmax) + 1e-30


def snr_eps(n, A, c, V, SN, bmax, extra_flux=0.0, extra_rel=0.0):
    """S/N error bound per pixel; extra_flux (absolute, per pixel or scalar)
    and extra_rel (relative to |SN|) widen it for inputs that differ from the
    oracle's by a bounded amount (16-bit storage)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        e = (flux_bound(n, A, c, bmax) + extra_flux) / np.sqrt(np.where(V > 0, V, 1.0)) \
            + (SAFETY * 4 * U + extra_rel) * np.abs(SN)
    return np.where(np.isfinite(SN), e, 0.0)


def _shift(a, dy, dx, fill):
    h, w = a.shape
    out = np.full_like(a, fill)
    ys = slice(max(0, dy), h + min(0, dy))
    yd = slice(max(0, -dy), h + min(0, -dy))
    xs = slice(max(0, dx), w + min(0, dx))
    xd = slice(max(0, -dx), w + min(0, -dx))
    out[yd, xd] = a[ys, xs]
    return out


def candidate_status(SN, c, eps, thr, c_min):
    """(robust_yes, marginal) masks of the candidate decision of every pixel."""
    yes = (c >= c_min) & (SN - thr > eps)
    no = (c < c_min) | (SN - thr < -eps)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            q = _shift(SN, dy, dx, -np.inf)  # q[y, x] = SN[y+dy, x+dx]
            eq = _shift(eps, dy, dx, 0.0)
            tol = eps + eq
            with np.errstate(invalid="ignore"):
                d = SN - q
            yes &= d > tol
            no |= d < -tol
    marg = ~yes & ~no
    return yes, marg


def compare_velocity(got, got_count, ref, n, bmax, thr, c_min, k_max, w, extra_flux=0.0, extra_rel=0.0):
    """Check one velocity's GPU list against the oracle (keep_maps entry).

    Returns the number of marginal decisions met.  Raises AssertionError on
    any disagreement that is not marginal.  extra_flux / extra_rel widen the
    error bounds (see snr_eps) when the GPU ran on inputs that differ from
    the oracle's by a bounded amount."""
    SN, c, V, S, A = ref["SN"], ref["c"], ref["V"], ref["S"], ref["A"]
    eps = snr_eps(n, A, c, V, SN, bmax, extra_flux, extra_rel)
    yes, marg = candidate_status(SN, c, eps, thr, c_min)
    n_yes, n_marg = int(yes.sum()), int(marg.sum())
    assert ref["count"] >= n_yes and ref["count"] <= n_yes + n_marg
    assert n_yes <= got_count <= n_yes + n_marg, (got_count, n_yes, n_marg)
    nv = min(k_max, got_count)
    g = got[:nv]
    assert np.all(got["rank"][:nv] == np.arange(nv))
    assert np.all(got["rank"][nv:] == -1)
    ras = g["y"].astype(np.int64) * w + g["x"]
    # every listed pixel is a candidate or a marginal one
    gy, gx = g["y"], g["x"]
    ok = yes[gy, gx] | marg[gy, gx]
    assert np.all(ok), list(zip(gx[~ok], gy[~ok]))
    # per-item values
    assert np.array_equal(g["coverage"], c[gy, gx])
    assert np.all(np.abs(g["snr"] - SN[gy, gx]) <= eps[gy, gx] + 1e-30)
    xf = extra_flux[gy, gx] if np.ndim(extra_flux) else extra_flux
    fb = flux_bound(n, A[gy, gx], c[gy, gx], bmax) + xf
    assert np.all(np.abs(g["flux"] - S[gy, gx]) <= fb)
    # the GPU list is in its own key order
    key_ok = (g["snr"][:-1] > g["snr"][1:]) | ((g["snr"][:-1] == g["snr"][1:]) & (ras[:-1] < ras[1:]))
    assert np.all(key_ok)
    # compare with the oracle's list
    oref = ref["all"]  # raster indices of every oracle candidate, key order
    osn = SN.reshape(-1)[oref]
    oeps = eps.reshape(-1)[oref]
    n_order = 0
    for i in range(min(len(oref), k_max + 1) - 1):
        if osn[i] - osn[i + 1] <= oeps[i] + oeps[i + 1]:
            n_order += 1
    if n_marg == 0 and n_order == 0:
        assert got_count == ref["count"]
        assert np.array_equal(ras, oref[:k_max]), (ras[:8], oref[:8])
        return 0
    # marginal case: robust candidates clearly inside the top k_max must be listed
    if len(oref) > k_max:
        cut = osn[k_max - 1]
        cut_eps = oeps[k_max - 1]
    else:
        cut, cut_eps = -np.inf, 0.0
    ys, xs = np.nonzero(yes)
    must = (SN[ys, xs] - eps[ys, xs] > cut + cut_eps + (eps.max() if n_marg else 0.0))
    listed = set(ras.tolist())
    for y, x in zip(ys[must], xs[must]):
        assert y * w + x in listed, (x, y)
    return n_marg + n_order
