"""MI355X (gfx950) RNS-CKKS hot path for encrypted CNN inference.

The library is libfhe.so (C ABI in include/fhe.h); `fhe` is its Python
binding.  Importing this package fails if the library has not been built.
"""
from . import fhe  # noqa: F401
from .fhe import Context, Ciphertext, CtArray, Plaintext, EvalKey, FheError, BatchOp, Graph, capture_graph  # noqa: F401
