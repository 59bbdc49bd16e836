"""MI355X-native nodal DG solver for the velocity-stress elastic wave equation.

The compute path is the C-ABI library ``libdgw.so`` (hand-written HIP for
gfx950, declared in ``include/dgw.h``); this package is its thin Python
binding: argument marshalling only.  PyTorch supplies device memory (through
the library's allocator hook) and streams.
"""

from ._lib import LibraryMissingError, library_path, load  # noqa: F401
from .dgw import (Solver, ElasticMisfit, ref_nodes, ref_operators,  # noqa: F401
                  order_elements, permute_mesh, DGWError)

__all__ = ["Solver", "ElasticMisfit", "ref_nodes", "ref_operators",
           "order_elements", "permute_mesh", "DGWError",
           "LibraryMissingError", "load", "library_path"]
