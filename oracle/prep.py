"""The steps the paper runs just before the search (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the GPU library.

Plain float64 NumPy of the definitions (frames are read as their exact
float32 values):

* static-source removal (Sec. 2.1): each frame minus the per-pixel median of
  the group's frames (for an even count, the mean of the two middle values);
* co-adding (Sec. 2.1, Sec. 2.2): the sum of every `group` consecutive frames,
  complete groups only, with the group's mean timestamp;
* 2x2 binning (Sec. 2.3): the sum of each 2x2 pixel block, an odd last row or
  column dropped.
"""

from __future__ import annotations

import numpy as np


def median_subtract(frames: np.ndarray):
    """(out, med): float64 F_i - med and the per-pixel median med."""
    f = np.asarray(frames, np.float64)
    med = np.median(f, axis=0)
    return f - med[None], med


def coadd(frames: np.ndarray, group: int, t=None):
    """(out, t_out): float64 [n // group][h][w] group sums and mean times."""
    f = np.asarray(frames, np.float64)
    ng = f.shape[0] // group
    out = f[: ng * group].reshape(ng, group, *f.shape[1:]).sum(axis=1)
    t_out = None
    if t is not None:
        t = np.asarray(t, np.float64)
        t_out = t[: ng * group].reshape(ng, group).mean(axis=1)
    return out, t_out


def bin2x2(frames: np.ndarray) -> np.ndarray:
    f = np.asarray(frames, np.float64)
    n, h, w = f.shape
    ho, wo = h // 2, w // 2
    return f[:, : 2 * ho, : 2 * wo].reshape(n, ho, 2, wo, 2).sum(axis=(2, 4))
