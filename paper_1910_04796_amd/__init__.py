"""MI355X-native local block-sparse FP64 multiply (block-CSR), after the
DBCSR paper's local multiplication (stacks of small block products) and its
densification (one large GEMM over merged panels).

The compute lives in the HIP library ``libbsmm.so`` (sources in ``csrc/``,
C-ABI in ``include/bsmm.h``); ``bsmm`` is its ctypes binding.
"""
from . import bsmm  # noqa: F401  (fails loudly when libbsmm.so is missing)
from .bsmm import BsmmError, Matrix, multiply, use_torch_allocator  # noqa: F401
