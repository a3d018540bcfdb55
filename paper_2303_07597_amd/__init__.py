"""Group-sparse smooth-dual optimal transport on MI355X (gfx950).

The computation lives in ``libotgs.so`` (hand-written HIP kernels behind the
C ABI of ``include/otgs.h``); :mod:`paper_2303_07597_amd.otgs` is its ctypes
binding.  PyTorch provides device memory and streams only.
"""
from .otgs import (  # noqa: F401
    Handle, OTGSError, ot_gs_rho_to_mu, ot_gs_version,
    OT_GS_DENSE, OT_GS_SCREENED, OT_GS_SNAPSHOT,
    OT_GS_COST_GIVEN, OT_GS_COST_MATERIALIZE, OT_GS_COST_ONTHEFLY,
    KERNEL_GRAD, KERNEL_SCREEN, KERNEL_REDUCE, KERNEL_LBFGS,
)
