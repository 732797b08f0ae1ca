"""Material-aware smoothed-aggregation AMG and AMG-preconditioned CG on MI355X.

The compute path is the HIP library libmatamg.so (C ABI in include/amg.h);
this package is its Python binding.  Importing the package does not load the
library; the first call that needs it does, and raises if it is not built.
"""

from ._lib import (  # noqa: F401
    EXPORTED,
    LIB_PATH,
    AmgError,
    Hierarchy,
    Server,
    load,
    options,
    trim_cache,
)
