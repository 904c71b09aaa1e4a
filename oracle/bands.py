"""Open-channel count of a periodic lead from its band structure (oracle; test infrastructure only).

A perfect crystal transmits one unit per right-moving Bloch state at energy E, so T(E) must equal the
number of bands that cross E upwards as the Bloch phase q runs over [-pi, pi).  The lead's Bloch
matrices are H(q) = H00 + H01 e^{iq} + H01^H e^{-iq} and likewise S(q) (Sec. 3A, Eq. (bound) with
nearest-cell coupling and lam = e^{iq}).  This module never touches the self-energy or the solver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def bloch_bands(H00, H01, S00, S01, q):
    """Sorted generalized eigenvalues of (H(q), S(q)) for each q; shape [len(q), s]."""
    out = []
    for qq in np.atleast_1d(q):
        ph = np.exp(1j * qq)
        hq = H00 + H01 * ph + H01.conj().T / ph
        sq = S00 + S01 * ph + S01.conj().T / ph
        hq = 0.5 * (hq + hq.conj().T)
        sq = 0.5 * (sq + sq.conj().T)
        out.append(scipy.linalg.eigh(hq, sq, eigvals_only=True))
    return np.array(out)


def channel_count(H00, H01, S00, S01, E: float, nq: int = 2048, bands=None):
    """(N_ch, gap) where N_ch = half the total variation of #bands-below-E around the q loop.

    ``gap`` is the smallest |E_n(q) - E| over the grid points next to a crossing: a small value warns
    that E sits near a band extremum where a finite grid can miss a pair of crossings.
    """
    if bands is None:
        q = np.linspace(-np.pi, np.pi, nq, endpoint=False)
        bands = bloch_bands(H00, H01, S00, S01, q)
    below = (bands < E).sum(axis=1)
    loop = np.concatenate([below, below[:1]])
    tv = int(np.abs(np.diff(loop)).sum())
    return tv // 2, float(np.min(np.abs(bands - E)))
