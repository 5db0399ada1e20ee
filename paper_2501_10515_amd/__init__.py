"""Python binding of libascc (include/ascc.h): argument marshalling only.

Every step of the residual, update and solve runs in the HIP kernels of libascc.so; this
module checks torch tensors (device, dtype, shape, contiguity), passes their device pointers
and the current HIP stream through ctypes, and turns non-zero status codes into exceptions.
There is no CPU fallback: without the built library every call raises.

The function names are the C entry points' names.
"""
from __future__ import annotations

from ._lib import (  # noqa: F401
    ASCC_E_ARG,
    ASCC_E_HIP,
    ASCC_E_NOMEM,
    ASCC_E_NONFINITE,
    ASCC_E_NOT_CONVERGED,
    ASCC_E_SHAPE,
    ASCC_E_STATE,
    ASCC_PREC_BF16X3,
    ASCC_PREC_FP32,
    ASCC_PREC_FP64,
    ASCC_VVVV_FULL,
    ASCC_VVVV_PACKED,
    AsccError,
    Diis,
    Ints,
    Server,
    ascc_batch_reserve,
    ascc_batch_reserve_ws,
    ascc_batch_workspace_bytes,
    ascc_build_ints,
    ascc_build_ints_hbar,
    ascc_build_ints_hbar_ws,
    ascc_build_ints_ws,
    ascc_diis_create,
    ascc_diis_create_ws,
    ascc_diis_reset,
    ascc_initial_guess,
    ascc_last_error,
    ascc_phase_count,
    ascc_phase_name,
    ascc_reference_energy,
    ascc_timing_enable,
    ascc_timing_read,
    ascc_two_ansatz,
    ascc_get_precision,
    ascc_residual,
    ascc_residual_batch,
    ascc_plascc_workspace_bytes,
    ascc_set_plascc,
    ascc_set_plascc_ws,
    ascc_set_precision,
    ascc_solve,
    ascc_solve_noalloc,
    ascc_update,
    ascc_workspace_bytes,
    library_path,
    load_library,
)
