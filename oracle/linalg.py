"""Block-tridiagonal linear algebra by definition (oracle; test infrastructure only).

A block-tridiagonal matrix is given by its blocks: ``diag[i] = M_{i,i}``, ``upper[i] = M_{i,i+1}``,
``lower[i] = M_{i+1,i}`` (Sec. 3B: T and A have n_B diagonal blocks).
"""
from __future__ import annotations

import numpy as np


def assemble_dense(diag, upper, lower):
    """Dense N x N matrix from its blocks (N = nb * s)."""
    nb, s, _ = diag.shape
    n = nb * s
    m = np.zeros((n, n), dtype=np.complex128)
    for i in range(nb):
        m[i * s:(i + 1) * s, i * s:(i + 1) * s] = diag[i]
    for i in range(nb - 1):
        m[i * s:(i + 1) * s, (i + 1) * s:(i + 2) * s] = upper[i]
        m[(i + 1) * s:(i + 2) * s, i * s:(i + 1) * s] = lower[i]
    return m


def btd_solve(diag, upper, lower, rhs):
    """Solve M X = rhs for block-tridiagonal M by block Gaussian elimination (block Thomas).

    Top-down elimination of the sub-diagonal blocks, then back substitution.  Each block solve uses
    LAPACK's partially pivoted LU (numpy.linalg.solve).  ``rhs`` has shape [nb, s, m].  No fill appears
    outside the blocks, so this is Gaussian elimination of the whole system up to the pivot order.
    """
    nb = diag.shape[0]
    dt = [None] * nb
    rt = [None] * nb
    dt[0] = diag[0].copy()
    rt[0] = rhs[0].copy()
    for i in range(1, nb):
        # multiplier L = lower[i-1] dt[i-1]^{-1}, computed as a solve with the transpose
        mult = np.linalg.solve(dt[i - 1].T, lower[i - 1].T).T
        dt[i] = diag[i] - mult @ upper[i - 1]
        rt[i] = rhs[i] - mult @ rt[i - 1]
    x = np.empty_like(rhs, dtype=np.complex128)
    x[nb - 1] = np.linalg.solve(dt[nb - 1], rt[nb - 1])
    for i in range(nb - 2, -1, -1):
        x[i] = np.linalg.solve(dt[i], rt[i] - upper[i] @ x[i + 1])
    return x


def lu_partial_pivot(a):
    """Gaussian elimination with partial pivoting, written out (the block solver of Alg. 1, Sec. 3B).

    Column by column: the pivot is the remaining row with the largest |Re| + |Im| in the column (the
    lowest such row on ties), it is swapped into place, the entries below it become the multipliers
    (divided by the pivot) and the trailing block takes the rank-1 update.  An exactly zero pivot is
    recorded (1 + column, first one only) and its column is skipped.  Returns (lu, perm, info) with lu
    holding unit-lower L below and U on and above the diagonal of P a = L U, and row i of P a being
    row perm[i] of a.
    """
    lu = np.array(a, dtype=np.complex128, copy=True)
    n = lu.shape[0]
    perm = np.arange(n)
    info = 0
    for j in range(n):
        mag = np.abs(lu[j:, j].real) + np.abs(lu[j:, j].imag)
        p = j + int(np.argmax(mag))  # argmax returns the first maximum
        if p != j:
            lu[[j, p]] = lu[[p, j]]
            perm[[j, p]] = perm[[p, j]]
        piv = lu[j, j]
        if piv == 0:
            if info == 0:
                info = j + 1
            continue
        lu[j + 1:, j] /= piv
        lu[j + 1:, j + 1:] -= np.outer(lu[j + 1:, j], lu[j, j + 1:])
    return lu, perm, info


def boundary_rhs(nb: int, s: int, top, bottom):
    """Right-hand side whose only non-zero block rows are the first (``top``) and last (``bottom``).

    With nb == 1 both land in the single block row and add.
    """
    m = top.shape[1]
    rhs = np.zeros((nb, s, m), dtype=np.complex128)
    rhs[0] += top
    rhs[nb - 1] += bottom
    return rhs
