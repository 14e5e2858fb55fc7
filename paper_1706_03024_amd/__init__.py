"""fpt: MI355X-native fluorescent spectral path tracer (arXiv 1706.03024 model).

The transport runs in hand-written HIP kernels behind the C ABI declared in
include/fpt.h (libfpt.so, built in-tree); this package is its Python binding.
"""
from ._abi import FptError, TALLY_NAMES, EXIT_NAMES  # noqa: F401
from .renderer import Scene, Batch, render, new_tallies, tallies_dict, RECORD_DTYPE  # noqa: F401
