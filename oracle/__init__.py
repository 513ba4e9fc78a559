"""CPU oracle for the synthetic-tracking search.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of
`__graft_entry__` and the CPU-baseline leg of `bench.py` may import this
package.  The GPU library never calls it and shares no code with it.

Everything is plain NumPy in float64 (frames are read as their exact float32
values), written from the paper's statement of the method:

* Sec. 1 and Sec. 2.1: stationary sources removed, linear motion assumed with
  no constraint on position angle, each frame shifted according to the trial
  motion and the frames summed ("shift and stack" / synthetic tracking);
* Sec. 2.1: each track comes back with its motion, pixel position and S/N;
  trial motions are spaced by about half a pixel of shift; the pipeline only
  finds movers that show in half or more of a group's frames.

The readings taken where the paper is silent are listed in `sst_oracle.py`.
`quant.py` holds the 16-bit storage format (a data-layout step, not part of
the paper's method); `prep.py` the steps the paper runs before the search
(static-source removal by the median, co-adding, 2x2 binning); `refine.py`
the differentiable sub-pixel refinement of a detection.
"""

from .sst_oracle import (  # noqa: F401
    CAND_DTYPE,
    brute_force_stack,
    candidates_from_maps,
    default_min_coverage,
    detect,
    frame_stats,
    rha,
    shift_table,
    snr_velocity,
    stack,
    stack_velocity,
)
from .quant import dequantize_frames, frame_offsets, frame_scales, quantize_frames  # noqa: F401,E402
from .prep import bin2x2, coadd, median_subtract  # noqa: F401,E402
from . import refine  # noqa: F401,E402
