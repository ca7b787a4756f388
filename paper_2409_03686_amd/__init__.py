"""MI355X-native walk-on-ellipsoids elliptic-measure engine (libwos) and its Python binding.

The compute path is the HIP library libwos.so (include/wos.h); `paper_2409_03686_amd.wos` is a
ctypes binding with the same entry-point names.  Build with `python paper_2409_03686_amd/build.py`.
"""
from . import wos  # noqa: F401
from .wos import WosError, lib  # noqa: F401
