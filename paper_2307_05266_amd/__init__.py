"""MI355X-native solver for Stokes flow in periodic voxel geometries.

Conjugate gradients on the pressure Schur complement S = B A^{-1} B^T of the
staggered (MAC) discretization, with the Uzawa (identity) or SIMPLE
(B diag(A)^{-1} B^T) preconditioner, computing permeabilities of porous media
(Pimanov, Iliev, Oseledets, Muravleva, arXiv 2307.05266).  The solver is a
HIP library for gfx950 behind a C ABI (include/stokes.h); this package holds
its sources (csrc/), the build script and a thin ctypes binding.
"""

from .stokes import (  # noqa: F401
    Server,
    Stokes,
    StokesBatch,
    StokesError,
    stokes_estimate_bytes,
    stokes_setup_on_stream,
    load,
    stokes_apply,
    stokes_apply_device,
    stokes_apply_device_noalloc,
    stokes_destroy,
    stokes_get_fields,
    stokes_history,
    stokes_info,
    stokes_kernel_timing,
    stokes_permeability,
    stokes_preprocess,
    stokes_set_option,
    stokes_set_stream,
    stokes_setup,
    stokes_solve,
    STOKES_UZAWA,
    STOKES_SIMPLE,
    STOKES_OP_A,
    STOKES_OP_B,
    STOKES_OP_BT,
    STOKES_OP_SHAT,
    STOKES_OP_DIAG_A,
    STOKES_OP_DIAG_SHAT,
    STOKES_OP_PROJECT,
    STOKES_OP_S,
    STOKES_OP_MG_SHAT,
    STOKES_OP_MG_A,
    STOKES_FLAG_NO_FLOW,
    STOKES_FLAG_ZERO_RHS,
    STOKES_FLAG_INNER_MAXIT,
    STOKES_FLAG_MG_TWO_VISITS,
    STOKES_OK,
    STOKES_NOT_CONVERGED,
    STOKES_E_ARG,
    STOKES_E_NOMEM,
    STOKES_E_DEVICE,
    STOKES_E_BREAKDOWN,
    STOKES_E_STATE,
    STOKES_E_LIMIT,
)
