"""CPU FP64 oracle -- test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  The product path (the HIP
library and its Python binding) never imports it, and it never imports the
product path.  Inputs come from ``gwsynth`` (random draws only).
"""
from . import polarization, mlp, surrogate, precision, selfenergy  # noqa: F401
