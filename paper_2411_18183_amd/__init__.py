"""libasjoin: signature-accelerated hash equi-join on one MI355X (gfx950).

The join runs in the HIP kernels of ``libasjoin.so`` behind the C interface
declared in ``include/asjoin.h``; ``paper_2411_18183_amd.asjoin`` is the
Python binding (argument marshalling only).
"""
__all__ = ["asjoin", "build"]
