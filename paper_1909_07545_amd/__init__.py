"""MI355X (gfx950) non-rectified variational fisheye stereo.

Thin Python binding over the C ABI of ``libvfs.so`` (declared in
``include/vfs.h``): argument marshalling only, every step of the method runs
in the library's HIP kernels.  torch provides device memory and streams.

Importing loads torch first (its HIP runtime) and then the library, so both
share one runtime.  If the built library is missing the import fails: there
is no fallback path.
"""
from ._lib import (  # noqa: F401
    LIB_PATH, Rig, Server, VfsError, default_params, diff_stats, lib, profile_enable, profile_read, rectify,
    rectify_rotations, solve, unrectify,
    solve_batch, solve_probe, step_energy, step_gradient, step_linearise, step_pd, step_pd_energy, step_rank, step_tensor,
    step_triangulate,
    step_upsample, FIELD_TRAJECTORY, FIELD_CALIBRATION, FIELD_FLAGS, F_MASK, F_MX, F_MY, F_DATA, F_EPI,
)
