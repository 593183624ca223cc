"""MI355X-native per-CTU coding-tree search (multi-resolution encoding, arxiv 2301.12191).

The product is libmr.so (HIP kernels for gfx950 behind the C ABI in include/mr.h);
``paper_2301_12191_amd.mr`` is its thin Python binding.
"""
from . import mr  # noqa: F401
