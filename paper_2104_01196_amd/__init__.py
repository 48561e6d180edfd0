"""MI355X (gfx950) two-stage Gauss-Seidel (GS2) preconditioners and GMRES.

The compute path is the HIP library libgs2.so (C ABI in include/gs2.h); this
package only builds it and binds it through ctypes.
"""
from .native import (  # noqa: F401
    gs2_profile, gs2_profile_read, gs2_graphs,
    BACKWARD, FORWARD, SYMMETRIC, FP16_SCALED, FP32, FP64,
    PREC_GS2, PREC_GS_TRISOLVE, PREC_JR, PREC_NONE, PREC_MTGS, mtgs_apply,
    DeviceCSR, Gs2Error, Handle, BatchHandle,
    gs2_setup, gs2_apply, jr_apply, gs_trisolve_apply, gmres_solve, cg_solve, gs2_destroy, gs2_handle_query,
    gs2_setup_batched, gmres_solve_batched, gs2_destroy_batched, gs2_batched_schedule, status_string, lib,
    gs2_handle_schedule, gs2_gmres_schedule, gs2_gmres_basis_schedule, gs2_inner_residuals, XCD_AUTO, XCD_DISPATCH_ORDER, XCD_RANGES, gs2_inner_residuals_noalloc, ERR_SCRATCH, STAGNATED, NOT_CONVERGED, FORMAT_AUTO, FORMAT_SELL, FORMAT_DIA, FORMAT_BLOCK3, LDS_AUTO, LDS_OFF, LDS_ON,
)
