"""SplitSolve hot path for one AMD MI355X (gfx950): HIP kernels behind a C ABI, with a ctypes binding.

The library computes, for many (E, k) instances of a block-tridiagonal Hamiltonian/overlap pair,
the lead self-energies, the first and last block columns of (E S - H)^{-1} (SplitSolve pre-processing),
the open-boundary correction with the wave function and the corner of G^R (post-processing), and the
Caroli transmission.  See include/splitsolve.h for the ABI.
"""
from .splitsolve import (  # noqa: F401
    Context,
    Instance,
    MLP,
    Plan,
    SplitSolveError,
    load_library,
    SS_PREC_FP32,
    SS_PREC_FP32_LU,
    SS_PREC_BF16,
    SS_PREC_FP64,
    ss_apply_obc,
    ss_energy_integral,
    ss_observables,
    ss_injection_left,
    ss_lead_selfenergy,
    ss_lead_selfenergy_warm,
    ss_sigma_decode,
    ss_sigma_encode,
    ss_sigma_moments,
    ss_warm_features,
    ss_precompute_columns,
    ss_precompute_columns_spike,
    ss_lu_factor,
    ss_refine_psi,
    ss_transmission,
    ss_transmission_noalloc,
    ss_transmission_psi,
    ss_workspace_size,
)
