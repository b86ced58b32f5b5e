"""MI355X-native spin–orbit tracking (Abell, Meiser, Ranjbar & Barber, 2015).

The hot path — orbit maps fused with Romberg-accelerated quaternion spin
integration — runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/spintrack.h (libspintrack.so).  This package holds the ctypes
binding (`binding`), a torch-tensor convenience wrapper (`tracker`) and the
build script (`build`).
"""

from . import binding  # noqa: F401  (fails loudly if the library is missing)
from .tracker import SpinTracker  # noqa: F401
