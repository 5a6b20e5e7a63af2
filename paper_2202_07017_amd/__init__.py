"""MI355X-native state-vector simulation hot path (libqsv.so, gfx950 HIP).

The compute lives in the C-ABI library declared by include/qsv.h; the
``qsv`` module is its ctypes binding (argument marshalling only).
"""
from . import qsv  # noqa: F401

__all__ = ["qsv"]
