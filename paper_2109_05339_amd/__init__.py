"""MI355X-native slice-and-match for single-particle imaging (arXiv
2109.05339): type-2 NUFFT slicing, Euclidean orientation matching (FP32 or
BF16 with FP32 rescoring), the type-1 adjoint spread and the Toeplitz
normal equations of regularised merging and phasing (ER, HIO,
shrinkwrap), as hand-written
gfx950 kernels behind the C ABI of include/spfel.h.
"""
from ._lib import (SpfelError, SpfelInvalidArgument, SpfelStateError,  # noqa: F401
                   SpfelUnsupported, SpfelOutOfMemory, LIB_PATH, lib)
from .ops import (Plan, Normal, Phase, PHASE_ER, PHASE_HIO, row_norm2, match, match_bf16, match_noalloc, match_workspace_bytes,  # noqa: F401
                  new_best, column_mean, bf16_centred, scale_columns, ImagesF32, ImagesBF16, REAL, COMPLEX,
                  MATCH_FP32, MATCH_BF16_RESCORE8, MERGE_ACCUMULATE, MERGE_DEFER)
from .autograd import SliceFn, SliceLossFn, slice_model, slice_loss  # noqa: F401

# The library is loaded on first use (lib()); a missing build raises
# ImportError there.  There is no fallback path.
