"""MI355X-native hot path of the SGN constraint solver (arXiv 2506.16045).

The compute lives in libsgn.so (HIP, gfx950) behind a C ABI declared in
include/sgn.h; `paper_2506_16045_amd.sgn` is the thin ctypes binding that
marshals PyTorch device tensors into it.  `paper_2506_16045_amd.inputs` builds
seeded synthetic inputs and imports neither the library nor any checker.
Importing this package loads nothing; the library is loaded on first use of
`paper_2506_16045_amd.sgn`.
"""
__all__ = ["inputs", "sgn"]
