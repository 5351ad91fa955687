"""MI355X-native F-engine channelizer (Merry, "Efficient channelization on a
Graphics Processing Unit").

The data path runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/fengine.h``; :mod:`.fengine` is a thin ctypes binding
with the same names, taking torch device tensors (PyTorch supplies device
memory and streams only).
"""
from .fengine import (FE_OK, FE_EINVAL, FE_ENOMEM, FE_EHIP, FE_EDELAY, FE_ESIZE,
                      FE_PREC_FP32, FE_PREC_FP16, FE_PREC_BF16, PRECISIONS,
                      FE_PATH_AUTO, FE_PATH_SPLIT, FE_PATH_FUSED, FE_PATH_MATRIX_FIR, FE_PATH_SPLIT_FOLDED, PATHS,
                      FEngineError, Stream, Batch, load_library, debug_unpack10, version)

__all__ = ["FE_OK", "FE_EINVAL", "FE_ENOMEM", "FE_EHIP", "FE_EDELAY", "FE_ESIZE",
           "FE_PREC_FP32", "FE_PREC_FP16", "FE_PREC_BF16", "PRECISIONS",
           "FE_PATH_AUTO", "FE_PATH_SPLIT", "FE_PATH_FUSED", "FE_PATH_MATRIX_FIR", "FE_PATH_SPLIT_FOLDED", "PATHS",
           "FEngineError", "Stream", "Batch", "load_library", "debug_unpack10", "version"]
