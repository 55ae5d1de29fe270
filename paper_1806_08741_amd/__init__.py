"""MI355X-native Scalable SLIC (SSLIC) superpixels.

The compute path lives in ``libsslic.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/sslic.h``); ``paper_1806_08741_amd.sslic`` is the
thin ctypes binding that marshals torch device tensors and streams into it.
Importing this package loads nothing; the library is opened on first use.
"""

__all__ = ["sslic", "synth"]
