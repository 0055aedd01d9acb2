"""MI355X (gfx950) HIP implementation of the voxel hex8 SIMP state solve,
compliance sensitivity, filters and density-to-SDF transfer.

The computation lives in the HIP library libtopo_mi355x.so (C ABI in
include/to.h); `api` is its Python binding.  Importing this package does not
load the library; the first call does, and fails if it is not built.
"""
from ._lib import (BC_CANTILEVER, BC_MBB, BC_CUSTOM, PREC_FP64, PREC_FP32_REFINE,  # noqa: F401
                   PREC_FP32_REFINE_BF16, FILTER_DENS, FILTER_DENS_T, FILTER_SENS)
