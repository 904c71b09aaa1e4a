"""Lead self-energies for the open boundary conditions (oracle; test infrastructure only).

Notation.  A lead is a semi-infinite repetition of one cell.  With a complex energy z = E + i*eta the
lead blocks in the A = E*S - H convention are

    a0  = (E + i eta) S00 - H00          (diagonal cell; eta enters only here)
    a1  = E S01 - H01                    (cell q -> q+1)
    am1 = a1^H = E S10 - H10             (cell q+1 -> q)

The right lead's surface Green's function obeys g_R = (a0 - a1 g_R am1)^{-1} and Sigma_R = a1 g_R am1;
the left lead's obeys g_L = (a0 - am1 g_L a1)^{-1} and Sigma_L = am1 g_L a1.  The device matrix with
open boundaries is T = E S - H - Sigma with Sigma_L in the first and Sigma_R in the last diagonal block
(Sec. 2B, Eq. (negf) and (wf)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def lead_blocks(H00, H01, S00, S01, E: float, eta: float):
    """(a0, a1, am1) of the lead cell at energy E with broadening eta on the diagonal cell only."""
    a0 = (E + 1j * eta) * S00 - H00
    a1 = E * S01 - H01
    am1 = a1.conj().T
    return a0, a1, am1


def _maxabs(a) -> float:
    return float(np.max(np.abs(a))) if a.size else 0.0


def decimation(a0, a1, am1, tol: float = 1e-14, max_iter: int = 200):
    """Sancho-Rubio decimation (the iterative decimation technique named in Sec. 3A).

    Each pass eliminates every other cell of the chain: with G = eps^{-1},
        eps_s  <- eps_s  - alpha G beta          (right-lead surface: neighbour to the right)
        eps_sL <- eps_sL - beta G alpha          (left-lead surface: neighbour to the left)
        eps    <- eps - alpha G beta - beta G alpha
        alpha  <- -alpha G alpha,   beta <- -beta G beta
    starting from eps = eps_s = eps_sL = a0, alpha = a1, beta = am1.  Stop when
    max|alpha| + max|beta| <= tol * max|a0|.  Then g_R = eps_s^{-1}, g_L = eps_sL^{-1}.

    Returns (sigma_L, sigma_R, iterations, converged).
    """
    eps_s = a0.copy()
    eps_sl = a0.copy()
    eps = a0.copy()
    alpha = a1.copy()
    beta = am1.copy()
    scale = _maxabs(a0)
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        g_beta = np.linalg.solve(eps, beta)
        g_alpha = np.linalg.solve(eps, alpha)
        a_g_b = alpha @ g_beta
        b_g_a = beta @ g_alpha
        eps_s = eps_s - a_g_b
        eps_sl = eps_sl - b_g_a
        eps = eps - a_g_b - b_g_a
        alpha = -(alpha @ g_alpha)
        beta = -(beta @ g_beta)
        if _maxabs(alpha) + _maxabs(beta) <= tol * scale:
            converged = True
            break
    sigma_r = a1 @ np.linalg.solve(eps_s, am1)
    sigma_l = am1 @ np.linalg.solve(eps_sl, a1)
    return sigma_l, sigma_r, it, converged


def decimation_conditioning(a0, a1, am1, tol: float = 1e-14, max_iter: int = 200) -> float:
    """Largest 1-norm condition estimate of eps over the passes of ``decimation`` (same recursion).

    Every pass solves with eps; a solve carries a forward error of order u * cond(eps), so this bounds
    how far two correct finite-precision runs of the decimation may drift apart.  Used only to set
    comparison tolerances.
    """
    import scipy.linalg as sla

    eps = a0.copy()
    alpha = a1.copy()
    beta = am1.copy()
    scale = _maxabs(a0)
    worst = 1.0
    for _ in range(max_iter):
        lu, piv = sla.lu_factor(eps)
        rcond, _info = sla.lapack.zgecon(lu, np.linalg.norm(eps, 1), norm="1")
        worst = max(worst, 1.0 / max(float(rcond), 1e-300))
        g_beta = sla.lu_solve((lu, piv), beta)
        g_alpha = sla.lu_solve((lu, piv), alpha)
        eps = eps - alpha @ g_beta - beta @ g_alpha
        alpha, beta = -(alpha @ g_alpha), -(beta @ g_beta)
        if _maxabs(alpha) + _maxabs(beta) <= tol * scale:
            break
    return worst


def quadratic_residuals(a0, a1, am1, sigma_l, sigma_r):
    """Relative Frobenius residuals of the fixed-point equations of Sigma_R and Sigma_L.

    res_R = ||Sigma_R - a1 (a0 - Sigma_R)^{-1} am1|| / ||Sigma_R||,
    res_L = ||Sigma_L - am1 (a0 - Sigma_L)^{-1} a1|| / ||Sigma_L||.
    """
    rr = sigma_r - a1 @ np.linalg.solve(a0 - sigma_r, am1)
    rl = sigma_l - am1 @ np.linalg.solve(a0 - sigma_l, a1)
    nr = max(np.linalg.norm(sigma_r), 1e-300)
    nl = max(np.linalg.norm(sigma_l), 1e-300)
    return float(np.linalg.norm(rl) / nl), float(np.linalg.norm(rr) / nr)


def broadening(sigma):
    """Gamma = i (Sigma - Sigma^H)."""
    return 1j * (sigma - sigma.conj().T)


def _decaying_modes(c0, c1, c2):
    """Solve (c0 + c1 lam + c2 lam^2) u = 0 and return (lam, U) for the s roots with |lam| < 1.

    Companion pencil: [[0, I], [-c0, -c1]] [u; v] = lam [[I, 0], [0, c2]] [u; v] with v = lam u.
    """
    s = c0.shape[0]
    eye = np.eye(s)
    zero = np.zeros((s, s))
    a = np.block([[zero, eye], [-c0, -c1]])
    b = np.block([[eye, zero], [zero, c2]])
    lam, vec = scipy.linalg.eig(a, b)
    finite = np.isfinite(lam)
    mag = np.where(finite, np.abs(lam), np.inf)
    order = np.argsort(mag)
    keep = order[:s]
    return lam[keep], vec[:s, keep], mag[order]


def selfenergy_modes(a0, a1, am1):
    """Independent route to Sigma through the lead modes (Sec. 3A, Eq. (bound), one-cell range).

    Bloch solutions psi_{q+1} = lam psi_q of the lead satisfy (am1 + a0 lam + a1 lam^2) u = 0.  With
    eta > 0 exactly s roots have |lam| < 1: the modes that decay or propagate to the right.  With
    F_R = U diag(lam) U^{-1} the right lead gives Sigma_R = -a1 F_R.  The left lead uses the mirrored
    polynomial (a1 + a0 mu + am1 mu^2) u = 0, mu = 1/lam, and Sigma_L = -am1 F_L.

    Returns (sigma_L, sigma_R, sorted |lam| of the right pencil) .
    """
    lam_r, u_r, mags = _decaying_modes(am1, a0, a1)
    f_r = u_r @ np.diag(lam_r) @ np.linalg.inv(u_r)
    mu_l, u_l, _ = _decaying_modes(a1, a0, am1)
    f_l = u_l @ np.diag(mu_l) @ np.linalg.inv(u_l)
    return -am1 @ f_l, -a1 @ f_r, mags


def is_retarded(a0, a1, am1, sigma_l, sigma_r, tol: float = 1e-8) -> bool:
    """Retarded branch: Gamma >= 0 (up to tol*||Gamma||) and the Bloch propagators have spectral radius <= 1+tol.

    F_R = -(a0 - Sigma_R)^{-1} am1 and F_L = -(a0 - Sigma_L)^{-1} a1 propagate the lead solution away from
    the device; a non-retarded root of the fixed-point equation has a growing mode.
    """
    ok = True
    for sig, c in ((sigma_r, am1), (sigma_l, a1)):
        gam = broadening(sig)
        w = np.linalg.eigvalsh(0.5 * (gam + gam.conj().T))
        scale = max(np.max(np.abs(w)), 1e-300)
        ok &= bool(w.min() >= -tol * scale)
        f = -np.linalg.solve(a0 - sig, c)
        ok &= bool(np.max(np.abs(np.linalg.eigvals(f))) <= 1.0 + tol)
    return ok
