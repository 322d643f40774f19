"""MI355X primal-dual solver for positive-contrast susceptibility MRI.

Wang, Cai et al., arXiv:2006.09808: dipole-kernel deconvolution by the
first-order primal-dual iteration, slice by slice, with an L1 prior on chi or
the weighted total-variation model of Eq. (1).  The
solve runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/pd.h; this package is its Python binding (argument marshalling only).
"""
from .pdlib import (  # noqa: F401
    Solver, PdError, load_library, validate, kernel_norm, status_string, now,
    make_request, LIB_PATH, EXPORTS, SUPPORTED_SIZES, MAX_BLUESTEIN,
    PD_OK, PD_PENDING, PD_ERR_ARG, PD_ERR_SIZE, PD_ERR_STEP, PD_ERR_BUDGET,
    PD_ERR_NONFINITE, PD_ERR_HIP, PD_ERR_CANCELLED, PD_ERR_TICKET, PD_ERR_NODEVICE, PD_ERR_SCRATCH,
    PD_STATIC_SCRATCH_BYTES, PD_FLAG_TEST_BARRIER_GIVEUP,
    PD_FP32, PD_FP64, KIND_COLUMN, KIND_ROW, KIND_RESIDENT, KIND_TV_COLUMN, KIND_TV_ROW, KIND_Z, KIND_MULTI, KIND_TV_RESIDENT,
    PD_FLAG_NO_RESIDENT, PD_MODEL_L1, PD_MODEL_TV, PD_KERNEL_DIPOLE_3D,
)
