"""MI355X-native multi-mode difference-map ptychography (arXiv:1808.10375).

The iteration runs in hand-written gfx950 HIP kernels behind the C-ABI
library ``libdm.so`` (declared in ``include/dm.h``); ``dm`` is its thin ctypes
binding.  ``synth`` generates seeded synthetic scans.  Importing the package
loads nothing: the library is opened on first use of ``dm``.
"""
__all__ = ["dm", "synth"]
