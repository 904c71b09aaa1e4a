"""The SplitSolve hot path computed by definition (oracle; test infrastructure only).

For one (E, k) instance:

* A = E S - H (Sec. 3B and 3C: the matrix A = (E S - H)), blocks ``A_{i,i}``, ``A_{i,i+1}``,
  ``A_{i+1,i} = A_{i,i+1}^H``.
* Q = A^{-1} B, the first and last block columns of A^{-1} (Sec. 3B, Step 1; B is N x 2s, zero except
  identity blocks at the top-left and bottom-right).
* T = A - Sigma with Sigma = B C, C = [[Sigma_L, 0, ...], [..., 0, Sigma_R]] (Sec. 3B).
* G^R = T^{-1} (Sec. 2B, Eq. (negf)); its corner blocks come from T X = B.
* psi = T^{-1} b with b = B b' (Sec. 2B, Eq. (wf); b' = the non-zero rows of Inj).
* R = 1 - C Q and z = R^{-1} C y with y = Q b' (Sec. 3B, Eq. (x)).
* Caroli transmission T_LR = Re Tr[Gamma_L G_1n Gamma_R G_1n^H], T_RL = Re Tr[Gamma_R G_n1 Gamma_L G_n1^H]
  with Gamma = i (Sigma - Sigma^H).

Everything that needs an inverse goes through ``linalg.btd_solve`` (block Thomas on the open or
closed device matrix itself, top-down), never through the bottom-up recursion of Alg. 1.
"""
from __future__ import annotations

import numpy as np

from .linalg import boundary_rhs, btd_solve
from .selfenergy import broadening, decimation, lead_blocks, quadratic_residuals


def device_blocks(Hd, Hu, Sd, Su, E: float):
    """Blocks of A = E S - H at real energy E: (diag, upper, lower)."""
    ad = E * Sd - Hd
    au = E * Su - Hu
    al = np.conj(np.transpose(au, (0, 2, 1)))
    return ad, au, al


def _unit_columns(s: int):
    eye = np.eye(s, dtype=np.complex128)
    zero = np.zeros((s, s), dtype=np.complex128)
    return np.hstack([eye, zero]), np.hstack([zero, eye])


def first_last_columns(ad, au, al):
    """Q = [A^{-1}_{:,1}, A^{-1}_{:,n_B}] as an array [nb, s, 2s] (Sec. 3B, Step 1: solve A Q = B)."""
    nb, s, _ = ad.shape
    top, bottom = _unit_columns(s)
    return btd_solve(ad, au, al, boundary_rhs(nb, s, top, bottom))


def first_last_columns_mirrored(ad, au, al):
    """Q by the same definition but eliminated in the opposite block order (block Thomas on the
    reversed matrix).  Both results are exact up to rounding; their difference measures how strongly
    this instance amplifies rounding (used only to set comparison tolerances)."""
    s = ad.shape[1]
    qr = first_last_columns(ad[::-1].copy(), al[::-1].copy(), au[::-1].copy())
    return np.concatenate([qr[::-1][:, :, s:], qr[::-1][:, :, :s]], axis=2)


def open_diag(ad, sigma_l, sigma_r):
    """Diagonal blocks of T = A - Sigma: Sigma_L enters block 1, Sigma_R block n_B."""
    td = ad.copy()
    td[0] = td[0] - sigma_l
    td[-1] = td[-1] - sigma_r
    return td


def corner_greens(ad, au, al, sigma_l, sigma_r):
    """Corner of G^R = T^{-1} as a 2s x 2s array [[G_11, G_1n], [G_n1, G_nn]] (Sec. 2B, Eq. (negf))."""
    nb, s, _ = ad.shape
    top, bottom = _unit_columns(s)
    x = btd_solve(open_diag(ad, sigma_l, sigma_r), au, al, boundary_rhs(nb, s, top, bottom))
    return np.vstack([x[0], x[nb - 1]])


def wave_function(ad, au, al, sigma_l, sigma_r, inj):
    """psi = T^{-1} B b' as [nb, s, m] (Sec. 2B, Eq. (wf)); ``inj`` = b' (2s x m)."""
    nb, s, _ = ad.shape
    return btd_solve(open_diag(ad, sigma_l, sigma_r), au, al, boundary_rhs(nb, s, inj[:s], inj[s:]))


def smw_terms(q, sigma_l, sigma_r, inj):
    """R = 1 - C Q and z = R^{-1} C y, y = Q b' (Sec. 3B, Eq. (x) and Step 3).

    C Q stacks Sigma_L times block row 1 of Q over Sigma_R times block row n_B of Q.
    """
    s = sigma_l.shape[0]
    cq = np.vstack([sigma_l @ q[0], sigma_r @ q[-1]])
    r = np.eye(2 * s, dtype=np.complex128) - cq
    z = np.linalg.solve(r, cq @ inj)
    return r, z


def caroli(gc, sigma_l, sigma_r):
    """(T_LR, T_RL) = Re Tr[Gamma_L G_1n Gamma_R G_1n^H], Re Tr[Gamma_R G_n1 Gamma_L G_n1^H]."""
    s = sigma_l.shape[0]
    g1n = gc[:s, s:]
    gn1 = gc[s:, :s]
    gam_l = broadening(sigma_l)
    gam_r = broadening(sigma_r)
    t_lr = np.trace(gam_l @ g1n @ gam_r @ g1n.conj().T).real
    t_rl = np.trace(gam_r @ gn1 @ gam_l @ gn1.conj().T).real
    return float(t_lr), float(t_rl)


def solve_instance(Hd, Hu, Sd, Su, H00, H01, S00, S01, E: float, eta: float, inj=None,
                   want_q: bool = True, tol: float = 1e-14, max_iter: int = 200):
    """One (E, k) solve: Sigma_L/R, Q, corner of G^R, psi (if ``inj``), T_LR, T_RL.

    Returns a dict with keys sigma_l, sigma_r, iters, converged, resid (L, R), q, gc, psi, t_lr, t_rl.
    """
    a0, a1, am1 = lead_blocks(H00, H01, S00, S01, E, eta)
    sig_l, sig_r, iters, conv = decimation(a0, a1, am1, tol=tol, max_iter=max_iter)
    res = quadratic_residuals(a0, a1, am1, sig_l, sig_r)
    ad, au, al = device_blocks(Hd, Hu, Sd, Su, E)
    out = dict(sigma_l=sig_l, sigma_r=sig_r, iters=iters, converged=conv, resid=res)
    out["q"] = first_last_columns(ad, au, al) if want_q else None
    gc = corner_greens(ad, au, al, sig_l, sig_r)
    out["gc"] = gc
    out["t_lr"], out["t_rl"] = caroli(gc, sig_l, sig_r)
    out["psi"] = wave_function(ad, au, al, sig_l, sig_r, inj) if inj is not None else None
    return out
