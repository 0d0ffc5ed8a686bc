"""Dense Chebyshev Fermi-operator expansion on MI355X (gfx950).

The computation lives in ``libchebdm.so`` (hand-written HIP kernels behind the
C ABI of ``include/chebdm.h``); this package is its thin Python binding with
the same entry-point names.  PyTorch provides device memory and streams.
"""
from ._binding import (  # noqa: F401
    BF16X3, BF16X6, COMPOSITION, EXPORTED, FP32, FP64, LIB_PATH, POWER,
    Batch, ChebdmError, Handle, Info, Opts, Profile, chebdm_batch_create, chebdm_block_coeffs, chebdm_bounds, chebdm_bounds_lanczos, chebdm_bounds_noalloc, chebdm_commutator_norm,
    chebdm_coeffs, chebdm_density, chebdm_mlp_adam, chebdm_mlp_backward, chebdm_mlp_forward, chebdm_mlp_num_params,
    chebdm_moments, chebdm_mu_search, chebdm_profile_enable, chebdm_profile_read, chebdm_workspace_size,
    load_library, make_opts,
)
