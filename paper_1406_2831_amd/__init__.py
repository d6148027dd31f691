"""MI355X-native recycling BiCGSTAB (Ahuja, Benner, de Sturler, Feng, arXiv:1406.2831).

The solver lives in the HIP library ``librbicgstab.so`` (C ABI in
include/rbicgstab.h); ``paper_1406_2831_amd.rbicgstab`` is its thin binding.
"""
from .rbicgstab import (Context, Stats, RbsError, load_library, device_csr,  # noqa: F401
                        rbicgstab_workspace_bytes, rbicgstab_setup, rbicgstab_solve,
                        recycle_update, rbicgstab_get_blocks, rbicgstab_setup_matvecs,
                        rbicgstab_time_pass,
                        rbicgstab_destroy, LIB_PATH)
