"""MI355X-native D3Q27 CHM-MRT lattice Boltzmann hot path.

The compute lives in ``liblbm.so`` (HIP for gfx950, C ABI in include/lbm.h);
``paper_2101_11107_amd.lbm`` is its thin Python binding.
"""

from . import lbm  # noqa: F401
