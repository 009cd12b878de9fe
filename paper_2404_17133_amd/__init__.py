"""MI355X-native rid-preconditioned Davidson solver for TDDFT.

The solver itself is librid.so (HIP kernels for gfx950 behind a C ABI, see
include/rid.h); this package is its thin Python binding.  Importing it loads
the library and fails when it is not built.
"""

from . import _binding as binding  # noqa: F401  (status codes and structs)
from ._binding import LIB_PATH, lib  # noqa: F401  (raises ImportError if the library is missing)
from .solver import (  # noqa: F401
    Context,
    Problem,
    RidError,
    Server,
    aux_tensor,
    batch_solve,
    default_opts,
    make_request,
    make_result,
    molecule_problem,
    request_footprint,
)
