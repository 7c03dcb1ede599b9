"""MI355X-native syndrome belief-propagation decoder for MET-LDPC codes.

Python binding over the C ABI in ``include/met_bp.h`` (library
``libmetbp.so`` built in this directory).  This layer only marshals arguments:
every step of decoding runs in the library's HIP kernels.  PyTorch provides
device memory and the current stream.  There is no fallback: without the
built library, importing this package raises ImportError.

Method: arXiv:1711.01783 (Wang, Zhang, Yu, Guo), Methods Steps 1-5 and
eq. (1)-(5): flooding sum-product BP against a syndrome, many codewords at
once, degree-1 variable nodes left out of the iterations.
"""
from ._lib import (
    MET_EARLY_EXIT,
    MET_FIXED_ITERS,
    MetError,
    lib,
    library_path,
)
from .api import (BatchedDecoder, Code, DecodeOutput, Job, batched_workspace_bytes, decode, decode_batched, decode_noalloc, mdr_alice, mdr_bob,
                  syndrome,
                  timing_collect, timing_enable, workspace_bytes)

__all__ = [
    "BatchedDecoder",
    "Code",
    "DecodeOutput",
    "Job",
    "batched_workspace_bytes",
    "decode_batched",
    "decode_noalloc",
    "mdr_alice",
    "mdr_bob",
    "MET_EARLY_EXIT",
    "MET_FIXED_ITERS",
    "MetError",
    "decode",
    "lib",
    "library_path",
    "syndrome",
    "timing_collect",
    "timing_enable",
    "workspace_bytes",
]
