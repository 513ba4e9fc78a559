"""Seeded synthetic inputs shaped like the survey's image groups.

This package holds only input generation: timestamps, velocity grids and
frames of sky noise with injected linear movers (the injection model of the
paper's injection-retrieval tests, Sec. 2.3).  It contains none of the
search's arithmetic (no shift tables, no stacking, no S/N), so that both the
CPU oracle and the GPU library can be fed identical bytes without sharing any
code of the method.
"""

from .fields import (  # noqa: F401
    Field,
    FieldSpec,
    Mover,
    tiny_field,
    full_field,
    uneven_batch,
    diagnostic_field,
    pure_noise,
    render_movers,
    small_case,
    tile_border_case,
    BORDER_PEAKS,
    BORDER_TIES,
    SEED_BASE,
)
