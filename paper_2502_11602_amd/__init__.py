"""MI355X-native Cheesemap grid point index (Laso & Yermo, arXiv 2502.11602).

The index, its fixed-radius and k-NN searches run as hand-written HIP kernels
for gfx950 in ``libchs.so`` behind the C ABI of ``include/chs.h``; this
package only marshals torch tensors into that ABI."""
from ._lib import ChsError, lib  # noqa: F401
from .index import GridIndex  # noqa: F401
from .agg import GaussAgg, gauss_aggregate, neighbour_lists  # noqa: F401

__all__ = ["GridIndex", "GaussAgg", "gauss_aggregate", "neighbour_lists", "ChsError", "lib"]
