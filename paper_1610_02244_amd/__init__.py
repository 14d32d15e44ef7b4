"""MI355X-native two-site DMRG hot path (HIP library + ctypes binding).

The compute lives in libtnt_mi355x.so (include/tnt.h); `binding` marshals
block tensors into it.  Importing this package loads nothing; call
`binding.load()` for a context on cuda:0.
"""
__all__ = ["binding", "build"]
