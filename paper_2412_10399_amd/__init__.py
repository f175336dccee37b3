"""MI355X-native compact-kernel MPM step (CK-MPM, arXiv 2412.10399).

The product is the HIP library `libckmpm.so` (sources in `csrc/`, C ABI in
`include/ckmpm.h`); `ckmpm` is its thin Python binding.
"""
from . import ckmpm  # noqa: F401

__all__ = ["ckmpm"]
