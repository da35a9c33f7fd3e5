"""MI355X-native unsplit second-order Godunov hydro step (FP64, HIP/gfx950).

The compute path is the C-ABI library ``libhydro.so`` built from ``csrc/``;
``hydro`` is its thin Python binding (argument marshalling over torch device
memory and streams).  ``ics`` holds the seeded synthetic inputs.  The HIP
library is loaded lazily, on first use of the binding, and loading fails
loudly when it has not been built.
"""
__all__ = ["ics", "hydro"]
