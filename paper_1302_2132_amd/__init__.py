"""MI355X gas-kinetic flux/update library: Python binding of libgks.so.

Every step of the solver runs in the HIP kernels of libgks.so; this package only
marshals arguments through the C ABI (include/gks.h) and uses PyTorch to allocate
device workspaces and obtain HIP streams.  There is no CPU fallback: importing the
binding without a built library raises.
"""
from .gks import (  # noqa: F401
    GKS_OK, GKS_ERR_ARG, GKS_ERR_NONPHYSICAL, GKS_ERR_NOMEM, GKS_ERR_DEVICE, GKS_ERR_STATE,
    GksError, lib, lib_path, config_from_case, gks_workspace_bytes, gks_init, gks_step,
    gks_residual, gks_fields, gks_destroy, gks_last_error, gks_face_flops, gks_kw_face_flops, gks_face_flops_multid,
    gks_face_flops_recon,
    gks_state_device_ptr, gks_resume,
    gks_set_timing, gks_kernel_times,
    gks_batch_workspace_bytes, gks_batch_create, gks_batch_set_members, gks_batch_step,
    gks_batch_capture, gks_batch_set_launch, gks_batch_status, gks_batch_destroy,
    gks_batch_create_static, GKS_BATCH_STATIC_CAPACITY, gks_batch_capture_steps,
    Solver, Batch, EXPORTED,
)
