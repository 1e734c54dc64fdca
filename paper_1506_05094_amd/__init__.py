"""MI355X-native short-range molecular dynamics (pair forces over a Verlet list,
cell-sorted list builds, leapfrog NVE / Nose-Hoover NVT) behind the C-ABI of
include/srmd.h.  Importing the package does not load the HIP library;
``srmd.load()`` does, and fails loudly when it has not been built."""
from . import srmd  # noqa: F401
from .srmd import Batch, System, SrmdError, system_from_state  # noqa: F401
