"""Stereo Whitted ray tracing on AMD Instinct MI355X (gfx950).

The compute path is the HIP library libstereort.so behind the C ABI in
include/stereort.h; ``rt`` is its ctypes binding and ``stereo`` the
PyTorch-facing helpers (device memory and streams only).  Importing this
package loads nothing; the library is opened on first use and its absence is
an error.
"""

__all__ = ["rt", "stereo", "build"]
