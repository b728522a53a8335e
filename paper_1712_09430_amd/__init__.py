"""MI355X-native (gfx950) TPC sector-tracking hot path: cellular-automaton
neighbour finding and Kalman tracklet construction (arXiv:1712.09430, Sec. 2),
behind the catpc C ABI (include/catpc.h).

`catpc` is the ctypes binding of that ABI; `tracker` wraps it with torch
device buffers and streams.  Importing `tracker` needs torch; the binding
itself only needs the built library.
"""
from . import catpc  # noqa: F401
