"""Seeded synthetic inputs shared by the CPU oracle's tests, the GPU tests and the benchmark.

This package only *draws* inputs: block-tridiagonal Hamiltonian/overlap pairs, lead cells, energy grids
and injection blocks.  It holds none of the solver's arithmetic (no self-energy, no inversion, no
transmission), so that the oracle and the HIP path stay independent of each other.
"""
from .generators import (  # noqa: F401
    BTDInstance,
    chain_cell,
    scalar_chain_cell,
    ladder_cell,
    dft_like_cell,
    DFTLikeCell,
    device_from_cell,
    gauge_rotate,
    random_unitary,
    overlap_scale,
    random_btd,
    injection_block,
    SLAB_SHAPES,
)
