"""MI355X-native level-of-detail strand-hair renderer (arxiv 2405.10565).

The renderer is the HIP library libhair.so (C-ABI in include/hair.h); `binding` is its
ctypes binding, `autograd` wraps the backward pass for LoD fitting, `serve` is the
continuous-batching render server.  Build the library with `build.build()`.
"""
__all__ = ["binding", "build"]
