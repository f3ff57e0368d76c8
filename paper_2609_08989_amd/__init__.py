"""MI355X (gfx950) Kerr null-geodesic ray tracer: HIP kernels behind a C ABI.

The compute path lives in ``libtartarus.so`` (``csrc/``); ``tartarus`` is the
ctypes binding with the C function names.  Build with ``build.build()``.
"""
__all__ = ["tartarus", "build"]
