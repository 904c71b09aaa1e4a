"""Observables from the wave function over the (E, k) grid, by definition (oracle; test infrastructure
only).

Sec. 2B: once Eq. (wf) is solved at every energy E (and momentum k), the charge and current densities
follow from c(E) (psi here); the paper's Sec. 5C shows them as an electron distribution, a current map
and a spectral current.  With psi injected from the left lead, psi psi^H = G Gamma_L G^H is the part
of the spectral function that the left reservoir fills, so for each instance:

* orbital density (Mulliken, the basis is non-orthogonal): n_mu = Re sum_c psi_{mu c} conj((S psi)_{mu c})
  = Re (psi psi^H S)_{mu mu};
* bond current between blocks i and i+1: J_i = 2 Im Tr[psi_i^H A_{i,i+1} psi_{i+1}] with
  A_{i,i+1} = E S_{i,i+1} - H_{i,i+1} (in units of e/h per spin).  Inside the device
  (E S - H) psi vanishes row block by row block, so J_i is the same for every i, and at the right end it
  equals Tr[psi_n^H Gamma_R psi_n], i.e. the transmission T_RL when psi = G W_L with W_L W_L^H = Gamma_L;
* energy integration: a weighted sum over instances, sum_b w_b x_b, with the caller's quadrature
  weights (for instance dE dk / (2 pi)^2 times a Fermi function f((E - mu) / kT)).
"""
from __future__ import annotations

import numpy as np


def s_times_psi(Sd, Su, psi):
    """(S psi)_i = S_{i,i-1} psi_{i-1} + S_{i,i} psi_i + S_{i,i+1} psi_{i+1}, S_{i+1,i} = S_{i,i+1}^H."""
    nb = psi.shape[0]
    out = np.empty_like(psi)
    for i in range(nb):
        v = Sd[i] @ psi[i]
        if i > 0:
            v = v + Su[i - 1].conj().T @ psi[i - 1]
        if i < nb - 1:
            v = v + Su[i] @ psi[i + 1]
        out[i] = v
    return out


def orbital_density(Sd, Su, psi):
    """n [nb, s]: n_mu = Re sum_c psi_{mu c} conj((S psi)_{mu c}) (Mulliken density of psi psi^H)."""
    return np.real(np.sum(psi * np.conj(s_times_psi(Sd, Su, psi)), axis=2))


def bond_currents(Hu, Su, E: float, psi):
    """J [nb - 1]: J_i = 2 Im Tr[psi_i^H (E S_{i,i+1} - H_{i,i+1}) psi_{i+1}]."""
    nb = psi.shape[0]
    out = np.empty(nb - 1)
    for i in range(nb - 1):
        a = E * Su[i] - Hu[i]
        out[i] = 2.0 * np.imag(np.trace(psi[i].conj().T @ a @ psi[i + 1]))
    return out


def fermi(E, mu: float, kT: float):
    """Fermi-Dirac occupation 1 / (1 + exp((E - mu) / kT))."""
    x = (np.asarray(E, dtype=np.float64) - mu) / kT
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def integrate(weights, values):
    """sum_b w_b values_b over the leading (instance) axis."""
    w = np.asarray(weights, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    return np.tensordot(w, v, axes=(0, 0))
