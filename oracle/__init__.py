"""CPU oracle for the synthetic-tracking search.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of
`__graft_entry__` and the CPU-baseline leg of `bench.py` may import this
package.  The GPU library never calls it and shares no code with it.

Everything is plain NumPy in float64 (frames are read as their exact float32
values), written from the paper's statement of the method:

* Sec. 1 and Sec. 2.1: stationary sources removed, linear motion assumed with
  no constraint on position angle, each frame shifted according to the trial
  motion and the frames summed ("shift and stack" / synthetic tracking);
* Sec. 2.1: a track is reported with its speed, position angle, pixel
  coordinates and S/N; the minimum useful shift is half a pixel; a mover must
  be above threshold for at least half of the frames of a group.

The readings taken where the paper is silent are listed in `sst_oracle.py`.
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
