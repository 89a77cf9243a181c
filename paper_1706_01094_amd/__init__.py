"""MI355X-native Monte Carlo Lattice Gas (Blommel & Wagner, arXiv:1706.01094).

The compute path is libmclg.so (hand-written HIP for gfx950) behind the C ABI
declared in include/mclg.h; ``mclg`` is its Python binding.
"""
from . import mclg  # noqa: F401
from .mclg import Lattice, Server  # noqa: F401
