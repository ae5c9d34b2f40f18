"""MI355X-native D3Q27 cascaded lattice Boltzmann method (arXiv:1801.04586).

The collide-and-stream update, its adjoint and the reduced-precision storage
variants run in hand-written HIP kernels for gfx950 (``csrc/``), behind the C
ABI of ``include/clbm.h`` (``libclbm.so``).  This package is the thin Python
side: ``clbm`` marshals torch tensors through ctypes, ``adjoint`` wraps the
adjoint kernels in a ``torch.autograd.Function`` with checkpointing.
"""
from .clbm import (CLBM_BF16, CLBM_F16, CLBM_F32, CLBM_F64, ClbmError, Context, Desc, Lattice, LIB_PATH,
                   RATE_NAMES, STORAGE, load_library, make_desc, strerror)

__all__ = ["CLBM_BF16", "CLBM_F16", "CLBM_F32", "CLBM_F64", "ClbmError", "Context", "Desc", "Lattice", "LIB_PATH",
           "RATE_NAMES", "STORAGE", "load_library", "make_desc", "strerror"]
