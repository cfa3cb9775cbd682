"""FP64 CPU oracle of the grain-envelope step: test infrastructure only.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  The product path never does.
"""
from .oracle import Oracle, build_oracle, f32_cells, f32_contain  # noqa: F401
