"""Plain float64 oracle of the synthetic-tracking search (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the GPU library.

What is computed (paper Sec. 1 and Sec. 2.1; O1-O6 below are this file's own
step names):

O1  Integer shifts.  For frame i and trial velocity component v (px/h) the
    frame is sampled at an integer offset d = RHA(v * (t_i - t_ref)), one
    float64 product with no fused multiply-add, rounded half away from zero.
O2  Frame statistics.  b_i = mean of frame i, s2_i = population variance
    (two passes, ddof = 0).  These normalise the stack (Sec. 2.1 removes the
    static sky before stacking; the S/N needs each frame's noise level).
O3  Shift-and-stack.  For velocity (vx[a], vy[b]) and pixel p = (x, y) of the
    frame grid at t_ref: I(p) = frames whose sample p + d_i lies inside the
    frame; S'(p) = sum over i in I(p), ascending i, of (F_i(p + d_i) - b_i);
    c(p) = |I(p)|; V(p) = sum over i in I(p) of s2_i.
O4  S/N.  SN = S' / sqrt(V) when c >= 1 (and 0 when V == 0); -inf when c = 0.
O5  Candidates.  p is a candidate iff c >= c_min, SN > threshold and p's key
    beats every 8-neighbour inside the grid, key = (SN, -raster index), so a
    plateau resolves to its lowest raster index.
O6  Lists.  Per velocity, candidates sorted by key, descending; the first
    k_max are kept, `count` is the number before truncation.

Readings where the paper is silent (each is a choice):
  R1 frames are sampled at p + d (the stacked grid is the sky at t_ref);
  R2 t_ref is an explicit argument;
  R3 rounding is half away from zero (C llround);
  R4 the velocity grid is the outer product vx x vy, index k = b*nvx + a;
  R5 out-of-frame samples contribute nothing; c_min defaults to ceil(N/2),
     following the paper's requirement that an object show in no fewer than
     half of the frames (Sec. 2.1);
  R6 background = frame mean, noise = population variance;
  R7 per-pixel S/N, no PSF matched filter;
  R8 strict comparison SN > threshold;
  R9 8-neighbourhood, ties to the lower raster index;
  R10 the plain stack is a SUM, or a MEAN = S/c (0 where c = 0);
  R13 the output grid is the W x H frame grid at t_ref.
"""

from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

CAND_DTYPE = np.dtype([
    ("ivx", np.int32), ("ivy", np.int32), ("x", np.int32), ("y", np.int32),
    ("snr", np.float64), ("flux", np.float64), ("coverage", np.int32), ("rank", np.int32),
])


# --------------------------------------------------------------------- O1 --
def rha(x) -> np.ndarray:
    """Round half away from zero, exactly, for float64 input (R3).

    |x| is split as r + f with r = floor(|x|); f = |x| - r is exact in float64
    (for |x| < 2^52 the subtraction is exact: both operands share the ulp grid
    of |x|), so the half-way test f >= 0.5 is exact and
    0.49999999999999994 rounds to 0 while 0.5 rounds to 1.
    """
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    r = np.floor(a)
    f = a - r
    m = r + (f >= 0.5)
    return np.where(x < 0, -m, m).astype(np.int64)


def shift_table(t: Sequence[float], t_ref: float, v: Sequence[float]) -> np.ndarray:
    """d[i][a] = RHA(v[a] * (t[i] - t_ref)), int64 [N][nv] (O1, R1-R3)."""
    t = np.asarray(t, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    tau = t - np.float64(t_ref)
    prod = tau[:, None] * v[None, :]
    return rha(prod)


# --------------------------------------------------------------------- O2 --
def frame_stats(frames: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Per-frame mean and population variance in float64, two passes (O2, R6)."""
    n = frames.shape[0]
    b = np.empty(n, dtype=np.float64)
    s2 = np.empty(n, dtype=np.float64)
    npx = frames.shape[1] * frames.shape[2]
    for i in range(n):
        f = frames[i].astype(np.float64)
        b[i] = np.sum(f) / npx
        s2[i] = np.sum((f - b[i]) ** 2) / npx
    return b, s2


def default_min_coverage(n: int, c_min: int) -> int:
    """R5: a mover must be seen in at least half of the frames."""
    return int(c_min) if c_min > 0 else (n + 1) // 2


# --------------------------------------------------------------------- O3 --
def _overlap(d: int, size: int) -> Tuple[int, int]:
    """Output index range [lo, hi) whose sample lo + d .. hi - 1 + d lies in
    [0, size)."""
    lo = max(0, -d)
    hi = min(size, size - d)
    return lo, max(lo, hi)


def stack_velocity(frames: np.ndarray, dx: Sequence[int], dy: Sequence[int],
                   offsets: Optional[Sequence[float]] = None,
                   weights: Optional[Sequence[float]] = None,
                   absolute: bool = False):
    """Stack of all frames along one trial velocity (O3).

    dx[i], dy[i]: the integer offsets of frame i.  Returns (S, c, V[, A]) with
    S = sum of (F_i(p + d_i) - offsets[i]) over in-frame samples in ascending
    frame order, c the number of in-frame samples, V = sum of weights[i] over
    the same frames, and (if `absolute`) A = sum of |F_i(p + d_i) - offsets[i]|.
    """
    n, h, w = frames.shape
    S = np.zeros((h, w), dtype=np.float64)
    c = np.zeros((h, w), dtype=np.int64)
    V = np.zeros((h, w), dtype=np.float64)
    A = np.zeros((h, w), dtype=np.float64) if absolute else None
    for i in range(n):
        ddx, ddy = int(dx[i]), int(dy[i])
        x0, x1 = _overlap(ddx, w)
        y0, y1 = _overlap(ddy, h)
        if x0 >= x1 or y0 >= y1:
            continue
        src = frames[i, y0 + ddy:y1 + ddy, x0 + ddx:x1 + ddx].astype(np.float64)
        if offsets is not None:
            src = src - np.float64(offsets[i])
        S[y0:y1, x0:x1] += src
        c[y0:y1, x0:x1] += 1
        if weights is not None:
            V[y0:y1, x0:x1] += np.float64(weights[i])
        if absolute:
            A[y0:y1, x0:x1] += np.abs(src)
    if absolute:
        return S, c, V, A
    return S, c, V


def stack(frames: np.ndarray, t, t_ref: float, vx, vy, bg=None, mode: str = "sum"):
    """Plain stacks of every velocity: out[b][a][y][x] (R4, R10) and coverage.

    bg: optional per-frame values subtracted from every sample (None: raw).
    mode 'sum' or 'mean' (mean = S / c, 0 where c == 0).
    """
    dx = shift_table(t, t_ref, vx)
    dy = shift_table(t, t_ref, vy)
    n, h, w = frames.shape
    out = np.zeros((len(vy), len(vx), h, w), dtype=np.float64)
    cov = np.zeros((len(vy), len(vx), h, w), dtype=np.int64)
    for b in range(len(vy)):
        for a in range(len(vx)):
            S, c, _ = stack_velocity(frames, dx[:, a], dy[:, b], offsets=bg)
            if mode == "mean":
                S = np.where(c > 0, S / np.maximum(c, 1), 0.0)
            elif mode != "sum":
                raise ValueError(mode)
            out[b, a] = S
            cov[b, a] = c
    return out, cov


# --------------------------------------------------------------------- O4 --
def snr_velocity(frames, dx_col, dy_col, b, s2, absolute: bool = False) -> Dict[str, np.ndarray]:
    """S', c, V and SN of one velocity (O3, O4, R7)."""
    res = stack_velocity(frames, dx_col, dy_col, offsets=b, weights=s2, absolute=absolute)
    S, c, V = res[:3]
    with np.errstate(divide="ignore", invalid="ignore"):
        sn = np.where(V > 0, S / np.sqrt(np.where(V > 0, V, 1.0)), 0.0)
    sn = np.where(c >= 1, sn, -np.inf)
    out = {"S": S, "c": c, "V": V, "SN": sn}
    if absolute:
        out["A"] = res[3]
    return out


# --------------------------------------------------------------------- O5 --
def local_max_mask(sn: np.ndarray) -> np.ndarray:
    """True where the key (SN, -raster) beats every in-grid 8-neighbour (R9).

    A neighbour earlier in raster order (row above, or left in the same row)
    must be strictly smaller; a later one may be equal (the earlier pixel of a
    tie has the larger key).  Out-of-grid neighbours are ignored (padded -inf).
    """
    h, w = sn.shape
    P = np.full((h + 2, w + 2), -np.inf)
    P[1:-1, 1:-1] = sn
    ok = np.ones((h, w), dtype=bool)
    for ddy in (-1, 0, 1):
        for ddx in (-1, 0, 1):
            if ddx == 0 and ddy == 0:
                continue
            q = P[1 + ddy:1 + ddy + h, 1 + ddx:1 + ddx + w]
            earlier = ddy < 0 or (ddy == 0 and ddx < 0)
            ok &= (sn > q) if earlier else (sn >= q)
    return ok


def candidates_from_maps(sn: np.ndarray, c: np.ndarray, threshold: float, c_min: int) -> np.ndarray:
    """Raster indices of the candidates of one velocity, sorted by key
    descending (O5, O6 before truncation)."""
    h, w = sn.shape
    mask = (c >= c_min) & (sn > np.float64(threshold)) & local_max_mask(sn)
    ys, xs = np.nonzero(mask)
    raster = ys.astype(np.int64) * w + xs
    order = np.lexsort((raster, -sn[ys, xs]))
    return raster[order]


# --------------------------------------------------------------------- O6 --
def velocity_list(ras: np.ndarray, m: Dict[str, np.ndarray], ia: int, ib: int, w: int, k_max: int):
    """One velocity's output (O6): the first k_max candidates of `ras` (raster
    indices already in key order) as records with their S/N, flux, coverage
    and 0-based rank, and the number of candidates before truncation."""
    top = ras[:k_max]
    rec = np.zeros(len(top), dtype=CAND_DTYPE)
    ys, xs = top // w, top % w
    rec["ivx"], rec["ivy"] = ia, ib
    rec["x"], rec["y"] = xs, ys
    rec["snr"] = m["SN"][ys, xs]
    rec["flux"] = m["S"][ys, xs]
    rec["coverage"] = m["c"][ys, xs]
    rec["rank"] = np.arange(len(top))
    return rec, int(len(ras))


def detect(frames: np.ndarray, t, t_ref: float, vx, vy, threshold: float,
           min_coverage: int, k_max: int,
           velocities: Optional[Sequence[int]] = None,
           keep_maps: bool = False):
    """Per-velocity candidate lists (O1-O6).

    velocities: optional subset of flat velocity indices k = b*nvx + a (R4).
    Returns dict k -> {'cand': CAND_DTYPE array (<= k_max rows), 'count': int,
    and with keep_maps also 'S','c','V','SN','A'}, plus key 'stats' = (b, s2).
    """
    n, h, w = frames.shape
    nvx, nvy = len(vx), len(vy)
    dx = shift_table(t, t_ref, vx)
    dy = shift_table(t, t_ref, vy)
    b, s2 = frame_stats(frames)
    c_min = default_min_coverage(n, min_coverage)
    ks = range(nvx * nvy) if velocities is None else velocities
    out: Dict = {"stats": (b, s2), "c_min": c_min}
    for k in ks:
        ia, ib = k % nvx, k // nvx
        m = snr_velocity(frames, dx[:, ia], dy[:, ib], b, s2, absolute=keep_maps)
        ras = candidates_from_maps(m["SN"], m["c"], threshold, c_min)
        rec, count = velocity_list(ras, m, ia, ib, w, k_max)
        entry = {"cand": rec, "count": count}
        if keep_maps:
            entry.update(m)
            entry["all"] = ras
        out[k] = entry
    return out


# ------------------------------------------------------------ brute force --
def brute_force_stack(frames: np.ndarray, t, t_ref: float, vx, vy, offsets=None) -> List:
    """Pure-Python loop over (velocity, pixel, frame) with explicit bounds
    checks; for tiny inputs only.  Rounding uses the decimal module (an
    implementation independent of `rha`).  Returns [b][a] -> (S, c) lists."""
    from decimal import Decimal, ROUND_HALF_UP

    def rnd(x: float) -> int:
        # decimal's ROUND_HALF_UP rounds ties away from zero; Decimal(float)
        # is the exact binary value.
        return int(Decimal(x).quantize(Decimal(1), rounding=ROUND_HALF_UP))

    n, h, w = frames.shape
    res = []
    for vyv in vy:
        row = []
        for vxv in vx:
            S = [[0.0] * w for _ in range(h)]
            C = [[0] * w for _ in range(h)]
            shifts = []
            for i in range(n):
                tau = float(t[i]) - float(t_ref)
                shifts.append((rnd(float(vxv) * tau), rnd(float(vyv) * tau)))
            for y in range(h):
                for x in range(w):
                    s, cc = 0.0, 0
                    for i in range(n):
                        xs, ys = x + shifts[i][0], y + shifts[i][1]
                        if 0 <= xs < w and 0 <= ys < h:
                            val = float(frames[i, ys, xs])
                            if offsets is not None:
                                val = val - float(offsets[i])
                            s = s + val
                            cc += 1
                    S[y][x] = s
                    C[y][x] = cc
            row.append((S, C))
        res.append(row)
    return res


def fsum_frames(frames: np.ndarray) -> np.ndarray:
    """Correctly rounded per-pixel sum over frames (math.fsum), for pins."""
    n, h, w = frames.shape
    out = np.empty((h, w), dtype=np.float64)
    for y in range(h):
        for x in range(w):
            out[y, x] = math.fsum(float(v) for v in frames[:, y, x])
    return out
