"""FP64 CPU oracle of the swept-contact docking search.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
the two share no code (the seeded input generators in `synth` feed both).

  search  -- Sec. IV: object grid, swept occupancy, trilinear rotation,
             circular correlation, peak and pose, top-K
  refine  -- Sec. V: SE(3) refinement (pose update, proximity score,
             distance queries, sensitivities, damped Gauss-Newton)
  sampling -- Sec. IV-C: Super-Fibonacci and GeoBall-SF orientation samplers
"""
from . import search  # noqa: F401
from .search import GridParams  # noqa: F401
from . import refine  # noqa: F401
from . import sampling  # noqa: F401
