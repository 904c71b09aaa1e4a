"""Pins of the observables oracle (density and current from psi, energy integration) — no GPU.

* one-orbital chain (onsite eps0, hopping -t): the left-injected state of the perfect chain is one
  Bloch wave, so the density is 1 / (2 t sin k) on every site (E - eps0 = -2 t cos k) and the current
  is one channel;
* any device: the bond current is the same across every block interface (current conservation) and
  equals the Caroli T_RL of the corner of G^R (an independent route through T^{-1});
* the density agrees with Re diag(G_{:,1} Gamma_L G_{:,1}^H S) from a dense inverse of the assembled
  open-system matrix, and neither observable depends on the factor W_L of Gamma_L;
* the Fermi function and the weighted sum by their definitions at hand-checked points.
"""
import numpy as np
import pytest

import synth
from oracle import linalg, observables, selfenergy, transport


def _left_factor(sigma_l):
    lam, v = np.linalg.eigh(selfenergy.broadening(sigma_l))
    keep = lam > 1e-14 * max(lam.max(), 1e-300)
    return v[:, keep] * np.sqrt(lam[keep])


def _left_state(inst, E, eta):
    a0, a1, am1 = selfenergy.lead_blocks(inst.H00, inst.H01, inst.S00, inst.S01, E, eta)
    sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
    w = _left_factor(sl)
    s = inst.Hd.shape[1]
    inj = np.vstack([w, np.zeros((s, w.shape[1]), np.complex128)])
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    psi = transport.wave_function(ad, au, al, sl, sr, inj)
    return psi, sl, sr, w


@pytest.mark.parametrize("E", [-1.5, 0.0, 0.8, 2.0])
def test_scalar_chain_density_and_current_closed_form(E):
    eps0, t = 0.3, 1.2
    inst = synth.device_from_cell(synth.scalar_chain_cell(eps0, t), 7)
    psi, _, _, _ = _left_state(inst, E, 1e-12)
    k = np.arccos(-(E - eps0) / (2 * t))
    n = observables.orbital_density(inst.Sd, inst.Su, psi)
    assert np.allclose(n, 1.0 / (2 * t * np.sin(k)), rtol=1e-9, atol=0)
    J = observables.bond_currents(inst.Hu, inst.Su, E, psi)
    assert np.allclose(J, 1.0, rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed,E", [(5, -0.4), (6, 0.25), (7, 0.6)])
def test_current_is_conserved_and_equals_caroli(seed, E):
    inst = synth.random_btd(6, 10, seed=seed)
    eta = 1e-10
    psi, sl, sr, _ = _left_state(inst, E, eta)
    J = observables.bond_currents(inst.Hu, inst.Su, E, psi)
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    _, t_rl = transport.caroli(transport.corner_greens(ad, au, al, sl, sr), sl, sr)
    assert t_rl > 1e-3  # something flows
    assert np.abs(J - t_rl).max() <= 1e-8 * max(1.0, t_rl), (J, t_rl)


def test_density_matches_dense_spectral_function_and_ignores_the_factor():
    inst = synth.random_btd(4, 8, seed=21)
    E, eta = 0.3, 1e-10
    psi, sl, sr, w = _left_state(inst, E, eta)
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    tmat = linalg.assemble_dense(transport.open_diag(ad, sl, sr), au, al)
    g1 = np.linalg.inv(tmat)[:, :8]
    a_left = g1 @ selfenergy.broadening(sl) @ g1.conj().T
    s_dense = linalg.assemble_dense(inst.Sd, inst.Su, np.conj(np.transpose(inst.Su, (0, 2, 1))))
    ref = np.real(np.diag(a_left @ s_dense)).reshape(4, 8)
    n = observables.orbital_density(inst.Sd, inst.Su, psi)
    assert np.abs(n - ref).max() <= 1e-9 * np.abs(ref).max()
    # W_L -> W_L U leaves psi psi^H, hence n and J, unchanged
    u = synth.random_unitary(w.shape[1], 4)
    psi_u = psi @ u
    assert np.abs(observables.orbital_density(inst.Sd, inst.Su, psi_u) - n).max() <= 1e-12 * np.abs(n).max()
    J = observables.bond_currents(inst.Hu, inst.Su, E, psi)
    assert np.abs(observables.bond_currents(inst.Hu, inst.Su, E, psi_u) - J).max() <= 1e-12


def test_fermi_and_weighted_sum():
    assert observables.fermi(0.2, 0.2, 0.05) == 0.5
    x = np.array([0.1, 0.37, 2.0])
    assert np.allclose(observables.fermi(0.2 + x, 0.2, 0.05) + observables.fermi(0.2 - x, 0.2, 0.05), 1.0)
    assert abs(observables.fermi(1.0, 0.0, 1.0) - 1.0 / (1.0 + np.e)) < 1e-15
    vals = np.array([[1.0, 2.0], [3.0, -1.0], [0.5, 0.0]])
    assert np.array_equal(observables.integrate([2.0, 1.0, 4.0], vals), np.array([7.0, 3.0]))
