"""MI355X object heap and parallel do-all (DynaSOAr, arXiv 1809.07444).

The compute path is libdsoar.so (HIP kernels for gfx950 behind the C ABI of
include/dsoar.h); this package only marshals arguments to it.  Importing the
package does not load the library; the first heap operation does, and fails
loudly if the library is missing."""
from ._capi import DsoarError, load  # noqa: F401
