"""FP64 CPU oracle for the fast DVM collision operator (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does.
"""
from .oracle import (  # noqa: F401
    build,
    lines,
    first_lines,
    default_weights,
    default_ntilde,
    collide,
    collide_bilinear,
    collide_terms,
    vjp,
    num_threads,
    set_num_threads,
    index_maxwellian,
    collide_near_equilibrium,
    equilibrium_distance,
    adaptive_levels,
)
