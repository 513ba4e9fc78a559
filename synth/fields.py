"""Seeded generators for the image groups the search runs on.

Shapes follow the survey instrument of the paper (Sec. 3): a 2K x 2K CCD at
0.35 arcsec/px, binned 2x2 for the fast-mover search (Sec. 2.3), nights of a
few hours, groups of tens of frames.  Movers are injected as point-sampled
Gaussian PSFs moving linearly (Sec. 2.1 assumes linear motion; Sec. 2.3
injects synthetic movers with the frame's PSF FWHM).  Time is in hours and
velocities in px/h throughout.

Nothing here implements the search itself: no integer shift tables, no
stacking, no signal-to-noise.  A mover's centre at time t is p0 + v (t - t_ref)
in continuous coordinates; that is the physical model of the data, not the
method's rounded shift.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 230307293

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclasses.dataclass
class Mover:
    x0: float  # position at t_ref, px
    y0: float
    vx: float  # px/h
    vy: float
    amp: float  # PSF peak value per frame, same unit as the frames
    fwhm: float  # px


@dataclasses.dataclass
class Field:
    name: str
    frames: np.ndarray  # float32 [N][H][W], C-contiguous
    t: np.ndarray  # float64 [N], strictly increasing, hours
    t_ref: float
    vx: np.ndarray  # float64 [nvx], px/h
    vy: np.ndarray  # float64 [nvy], px/h
    threshold: float = 5.0
    min_coverage: int = 0  # <= 0 means ceil(N/2)
    k_max: int = 64
    movers: List[Mover] = dataclasses.field(default_factory=list)
    sky: float = 0.0
    sigma: float = 1.0

    @property
    def n(self) -> int:
        return int(self.frames.shape[0])

    @property
    def h(self) -> int:
        return int(self.frames.shape[1])

    @property
    def w(self) -> int:
        return int(self.frames.shape[2])

    @property
    def updates(self) -> int:
        """Nominal frame*pixel*velocity updates of one full search."""
        return self.n * self.h * self.w * len(self.vx) * len(self.vy)


def render_movers(img: np.ndarray, tau: float, movers: List[Mover]) -> None:
    """Add every mover's PSF, point-sampled at integer pixel centres, into the
    float64 image `img` at time offset `tau` = t - t_ref (hours)."""
    h, w = img.shape
    for m in movers:
        s = m.fwhm * FWHM_TO_SIGMA
        cx = m.x0 + m.vx * tau
        cy = m.y0 + m.vy * tau
        r = int(math.ceil(6.0 * s)) + 1
        x_lo, x_hi = max(0, int(math.floor(cx)) - r), min(w, int(math.floor(cx)) + r + 2)
        y_lo, y_hi = max(0, int(math.floor(cy)) - r), min(h, int(math.floor(cy)) + r + 2)
        if x_lo >= x_hi or y_lo >= y_hi:
            continue
        xs = np.arange(x_lo, x_hi, dtype=np.float64) - cx
        ys = np.arange(y_lo, y_hi, dtype=np.float64) - cy
        g = np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2.0 * s * s))
        img[y_lo:y_hi, x_lo:x_hi] += m.amp * g


def _frames(rng, t, t_ref, h, w, sky, sigma, movers, noise=True) -> np.ndarray:
    n = len(t)
    out = np.empty((n, h, w), dtype=np.float32)
    for i in range(n):
        if noise:
            img = rng.normal(sky, sigma, size=(h, w))
        else:
            img = np.full((h, w), float(sky))
        render_movers(img, float(t[i] - t_ref), movers)
        out[i] = img.astype(np.float32)
    return out


def tiny_field(noise: bool = True) -> Field:
    """Tiny plain case: 32 frames of 128x128, background 0, N(0,1) noise,
    timestamps evenly spaced over 1 h (t_i = i/31), 3 movers of peak 1.5 sigma
    and FWHM 2.5 px at integer velocities within +-10 px/h whose whole track
    stays >= 4 px inside the frame, 21x21 grid at 1 px/h, 5 sigma."""
    rng = np.random.default_rng(SEED_BASE + 1)
    n, h, w = 32, 128, 128
    t = np.arange(n, dtype=np.float64) / 31.0
    t_ref = float(t[0])
    movers = []
    while len(movers) < 3:
        vx, vy = (int(v) for v in rng.integers(-10, 11, size=2))
        x0, y0 = (int(p) for p in rng.integers(0, 128, size=2))
        ends = [(x0 + vx * tt, y0 + vy * tt) for tt in (0.0, 1.0)]
        if all(4 <= ex <= w - 5 and 4 <= ey <= h - 5 for ex, ey in ends):
            movers.append(Mover(float(x0), float(y0), float(vx), float(vy), 1.5, 2.5))
    frames = _frames(rng, t, t_ref, h, w, 0.0, 1.0, movers, noise=noise)
    grid = np.arange(-10, 11, dtype=np.float64)
    return Field("plain-tiny 32x128x128 grid21x21", frames, t, t_ref, grid, grid.copy(),
                 threshold=5.0, min_coverage=16, k_max=64, movers=movers, sky=0.0, sigma=1.0)


def full_field_times(rng) -> np.ndarray:
    """71 evenly spaced slots over [0, 4] h with 7 dropped at random (a 10%
    gap fraction), leaving 64 frames."""
    slots = np.arange(71, dtype=np.float64) * (4.0 / 70.0)
    drop = rng.choice(71, size=7, replace=False)
    keep = np.setdiff1d(np.arange(71), drop)
    return slots[keep]


def full_field(n_movers: int = 50, h: int = 1024, w: int = 1024) -> Field:
    """Full field: 64 frames of 1024x1024 (a 2048^2 CCD binned 2x2), sky 100
    with Gaussian noise sigma=10, 4 h with 10% gaps, 50 movers with
    log-uniform peak 0.2-3 sigma and velocities uniform in +-40 px/h,
    81x81 grid at 1 px/h, S/N threshold 5, top-64 per velocity."""
    rng = np.random.default_rng(SEED_BASE + 2)
    t = full_field_times(rng)
    t_ref = float(t[0])
    movers = []
    for _ in range(n_movers):
        amp = float(math.exp(rng.uniform(math.log(2.0), math.log(30.0))))
        vx, vy = (float(v) for v in rng.uniform(-40.0, 40.0, size=2))
        x0 = float(rng.uniform(0, w))
        y0 = float(rng.uniform(0, h))
        movers.append(Mover(x0, y0, vx, vy, amp, 2.5))
    frames = _frames(rng, t, t_ref, h, w, 100.0, 10.0, movers)
    grid = np.arange(-40, 41, dtype=np.float64)
    return Field("plain-full 64x1024x1024 grid81x81", frames, t, t_ref, grid, grid.copy(),
                 threshold=5.0, min_coverage=32, k_max=64, movers=movers, sky=100.0, sigma=10.0)


@dataclasses.dataclass
class FieldSpec:
    """A field of a batch whose frames are made on demand (`make`)."""
    name: str
    seed: int
    n: int
    side: int
    grid: int  # odd: velocities -(grid//2) .. grid//2 px/h at 1 px/h on both axes
    t: np.ndarray
    n_movers: int

    @property
    def updates(self) -> int:
        return self.n * self.side * self.side * self.grid * self.grid

    def make(self) -> Field:
        rng = np.random.default_rng(self.seed)
        vmax = self.grid // 2
        movers = []
        for _ in range(self.n_movers):
            amp = float(math.exp(rng.uniform(math.log(2.0), math.log(30.0))))
            vx, vy = (float(v) for v in rng.uniform(-vmax, vmax, size=2))
            movers.append(Mover(float(rng.uniform(0, self.side)), float(rng.uniform(0, self.side)), vx, vy, amp, 2.5))
        frames = _frames(rng, self.t, float(self.t[0]), self.side, self.side, 100.0, 10.0, movers)
        g = np.arange(-vmax, vmax + 1, dtype=np.float64)
        return Field(self.name, frames, self.t, float(self.t[0]), g, g.copy(), threshold=5.0,
                     min_coverage=(self.n + 1) // 2, k_max=64, movers=movers, sky=100.0, sigma=10.0)


def uneven_batch(n_fields: int = 16) -> List[FieldSpec]:
    """Batch of uneven fields: frame counts uniform in 24..160, sides drawn
    from {512, 768, 1024, 2048}, velocity grids n x n with n odd in 41..121
    (1 px/h), timestamps over 4 h with 10% of the slots dropped, the full field's
    noise and movers (50 per 1024^2, scaled by area)."""
    rng = np.random.default_rng(SEED_BASE + 3)
    out = []
    for k in range(n_fields):
        n = int(rng.integers(24, 161))
        side = int(rng.choice([512, 768, 1024, 2048]))
        grid = int(rng.choice(np.arange(41, 122, 2)))
        m = int(round(n / 0.9))
        slots = np.arange(m, dtype=np.float64) * (4.0 / (m - 1))
        keep = np.sort(rng.choice(m, size=n, replace=False))
        t = slots[keep]
        n_movers = max(1, int(round(50 * side * side / 1024 ** 2)))
        out.append(FieldSpec(f"batch{k} {n}x{side}x{side} grid{grid}x{grid}", int(SEED_BASE + 300 + k), n, side, grid,
                             t, n_movers))
    return out


def diagnostic_field(n_frames: int = 32) -> Field:
    """Diagnostic shape for the stack's HBM roof: the full field's noise and grid
    with fewer frames (the materialised stack is HBM-bound only for small N)."""
    f = full_field()
    idx = np.linspace(0, f.n - 1, n_frames).round().astype(int)
    idx = np.unique(idx)
    return Field(f"diagnostic {len(idx)}x{f.h}x{f.w} grid81x81", np.ascontiguousarray(f.frames[idx]),
                 f.t[idx].copy(), float(f.t[idx][0]), f.vx, f.vy, f.threshold,
                 (len(idx) + 1) // 2, f.k_max, f.movers, f.sky, f.sigma)


def pure_noise(seed: int, n: int, h: int, w: int, sigma: float = 1.0, sky: float = 0.0,
               t: Optional[np.ndarray] = None) -> Field:
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    if t is None:
        t = np.arange(n, dtype=np.float64) / max(1, n - 1)
    frames = _frames(rng, t, float(t[0]), h, w, sky, sigma, [])
    grid = np.arange(-2, 3, dtype=np.float64)
    return Field(f"noise {n}x{h}x{w}", frames, t, float(t[0]), grid, grid.copy(), sky=sky, sigma=sigma)


def small_case(seed: int, n: int, h: int, w: int, nvx: int, nvy: int,
               vmax: float = 3.0, sky: float = 0.0, sigma: float = 1.0,
               ties: bool = True, n_movers: int = 2, t_ref: Optional[float] = None) -> Field:
    """Random small case for parity: irregular timestamps (optionally on a
    half-integer lattice so that v*(t - t_ref) hits exact .5 values), negative,
    zero and fractional velocities, a few movers."""
    rng = np.random.default_rng(SEED_BASE + 100 + seed)
    if ties:
        steps = rng.integers(1, 4, size=n).astype(np.float64) * 0.25
    else:
        steps = rng.uniform(0.05, 0.4, size=n)
    t = np.cumsum(steps)
    t -= t[0]
    if ties:
        vx = rng.integers(-int(2 * vmax), int(2 * vmax) + 1, size=nvx).astype(np.float64) * 0.5
        vy = rng.integers(-int(2 * vmax), int(2 * vmax) + 1, size=nvy).astype(np.float64) * 0.5
        vx[0] = 0.0
    else:
        vx = rng.uniform(-vmax, vmax, size=nvx)
        vy = rng.uniform(-vmax, vmax, size=nvy)
    if t_ref is None:
        t_ref = float(t[rng.integers(0, n)])
    movers = []
    for _ in range(n_movers):
        movers.append(Mover(float(rng.uniform(0, w)), float(rng.uniform(0, h)),
                            float(rng.uniform(-vmax, vmax)), float(rng.uniform(-vmax, vmax)),
                            float(rng.uniform(2, 6)) * sigma, 2.5))
    frames = _frames(rng, t, t_ref, h, w, sky, sigma, movers)
    return Field(f"small{seed} {n}x{h}x{w} grid{nvx}x{nvy}", frames, t, float(t_ref), vx, vy,
                 threshold=3.0, min_coverage=0, k_max=8, movers=movers, sky=sky, sigma=sigma)


# Pixels of the tile-border case: single bright pixels on the borders between
# 64 x 32 pixel tiles, and pairs of neighbours across a border given equal
# values in every frame (the first of each pair is the earlier in raster
# order).
BORDER_PEAKS = [(63, 10), (64, 20), (10, 31), (20, 32), (64, 32), (127, 5), (128, 64), (0, 0), (139, 69),
                (0, 45)]
BORDER_TIES = [((63, 40), (64, 40)), ((50, 31), (50, 32)), ((127, 31), (128, 32)), ((100, 63), (99, 64))]


def tile_border_case(seed: int = 0) -> Field:
    """6 frames of 70 x 140 N(0, 1) noise with stationary bright pixels
    (amplitude 40) at BORDER_PEAKS and equal-valued pairs at BORDER_TIES;
    velocities (0, 1.5, -2) x (0, 1) px/h, timestamps 0.5 h apart."""
    rng = np.random.default_rng(SEED_BASE + 500 + seed)
    n, h, w = 6, 70, 140
    t = np.arange(n, dtype=np.float64) * 0.5
    frames = rng.normal(0.0, 1.0, size=(n, h, w)).astype(np.float32)
    for x, y in BORDER_PEAKS:
        frames[:, y, x] += np.float32(40.0)
    for (x1, y1), (x2, y2) in BORDER_TIES:
        frames[:, y1, x1] += np.float32(40.0)
        frames[:, y2, x2] = frames[:, y1, x1]
    return Field(f"tile-borders{seed} {n}x{h}x{w}", frames, t, 0.0, np.array([0.0, 1.5, -2.0]),
                 np.array([0.0, 1.0]), threshold=5.0, min_coverage=0, k_max=32)
