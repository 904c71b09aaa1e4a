"""Learned warm start of the lead self-energies (oracle; test infrastructure only).

The decimation of Sec. 3A has no starting iterate: its convergence is set by the broadening alone.
A warm start therefore needs a solver that takes one.  Here that is Newton's method on the fixed-point
equation of the self-energy (right lead; the left lead swaps a1 and am1):

    F(Sigma) = Sigma - a1 (a0 - Sigma)^{-1} am1 = 0.

With g = (a0 - Sigma)^{-1}, M = a1 g and N = g am1, the derivative of F at Sigma maps D to D - M D N,
so a Newton step solves the Stein equation

    D - M D N = -F(Sigma),        Sigma <- Sigma + D.

Two routes for the Stein equation: the Kronecker system (I - N^T (x) M) vec(D) = vec(C) (small s only;
an independent check) and Smith's doubling, which sums the series D = sum_k M^k C N^k in 2^j terms:

    D_0 = C, M_0 = M, N_0 = N;   D_{j+1} = D_j + M_j D_j N_j,  M_{j+1} = M_j^2,  N_{j+1} = N_j^2.

The retarded self-energy is the solution whose propagator -N has spectral radius below one
(``selfenergy.is_retarded``); Newton may land on another root from a poor start, which the judge
(the residual plus the retardedness test) rejects in favour of the decimation.

The starting iterate comes from a multilayer perceptron: tanh hidden layers, a linear output layer,
mean squared error over all outputs, Adam updates.  Its forward and backward passes are written out
below in float64 (the GPU trains in FP32).
"""
from __future__ import annotations

import numpy as np

# ------------------------------------------------------------------ features and targets


def features(E, k, nfreq: int = 8, e_scale: float = 5.0):
    """Input features of the network for energies E and momenta k (arrays of equal length).

    [E / e_scale, cos k, sin k, sin(j pi E / e_scale), cos(j pi E / e_scale) (j = 1..nfreq),
     cos(j k), sin(j k) (j = 2..nfreq+1)]  ->  3 + 4 nfreq columns.
    """
    E = np.asarray(E, dtype=np.float64).reshape(-1)
    k = np.asarray(k, dtype=np.float64).reshape(-1)
    cols = [E / e_scale, np.cos(k), np.sin(k)]
    for j in range(1, nfreq + 1):
        cols += [np.sin(j * np.pi * E / e_scale), np.cos(j * np.pi * E / e_scale)]
    for j in range(2, nfreq + 2):
        cols += [np.cos(j * k), np.sin(j * k)]
    return np.stack(cols, axis=1)


def encode_sigma(sigma_l, sigma_r):
    """Real target vector [Re Sigma_L, Im Sigma_L, Re Sigma_R, Im Sigma_R] (row-major, 4 s^2 values)."""
    return np.concatenate([sigma_l.real.ravel(), sigma_l.imag.ravel(), sigma_r.real.ravel(), sigma_r.imag.ravel()])


def decode_sigma(y, s: int):
    """Inverse of ``encode_sigma``: (Sigma_L, Sigma_R)."""
    q = s * s
    sl = y[:q].reshape(s, s) + 1j * y[q:2 * q].reshape(s, s)
    sr = y[2 * q:3 * q].reshape(s, s) + 1j * y[3 * q:].reshape(s, s)
    return sl, sr


# ------------------------------------------------------------------ multilayer perceptron


def mlp_init(dims, seed: int):
    """Weights W_l [d_{l-1}, d_l] ~ N(0, 1/d_{l-1}), biases zero."""
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((dims[i], dims[i + 1])) / np.sqrt(dims[i]), np.zeros(dims[i + 1]))
            for i in range(len(dims) - 1)]


def mlp_forward(params, X):
    """Outputs of every layer: A_0 = X, A_l = tanh(A_{l-1} W_l + b_l), the last layer linear."""
    acts = [X]
    for i, (W, b) in enumerate(params):
        z = acts[-1] @ W + b
        acts.append(np.tanh(z) if i < len(params) - 1 else z)
    return acts


def mlp_loss_grad(params, X, T):
    """Mean squared error L = sum (Y - T)^2 / (n d_out) and its gradients by back-propagation."""
    acts = mlp_forward(params, X)
    Y = acts[-1]
    n, d = Y.shape
    loss = float(np.sum((Y - T) ** 2) / (n * d))
    dz = 2.0 * (Y - T) / (n * d)
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        grads[i] = (acts[i].T @ dz, dz.sum(axis=0))
        if i > 0:
            dz = (dz @ W.T) * (1.0 - acts[i] ** 2)  # tanh' = 1 - tanh^2
    return loss, grads


def adam_step(params, grads, state, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

    state: dict updated in place ({} before the first step).  Returns the new parameters."""
    flat_p = [p for Wb in params for p in Wb]
    flat_g = [g for Wb in grads for g in Wb]
    if not state:
        state.update(t=0, m=[np.zeros_like(p) for p in flat_p], v=[np.zeros_like(p) for p in flat_p])
    state["t"] += 1
    t = state["t"]
    new = []
    for i, (p, g) in enumerate(zip(flat_p, flat_g)):
        state["m"][i] = beta1 * state["m"][i] + (1 - beta1) * g
        state["v"][i] = beta2 * state["v"][i] + (1 - beta2) * g * g
        mhat = state["m"][i] / (1 - beta1 ** t)
        vhat = state["v"][i] / (1 - beta2 ** t)
        new.append(p - lr * mhat / (np.sqrt(vhat) + eps))
    return [(new[2 * i], new[2 * i + 1]) for i in range(len(params))]


# ------------------------------------------------------------------ Newton on the fixed-point equation


def stein_kron(M, N, C):
    """Solve D - M D N = C through the Kronecker system (column-major vec)."""
    s = M.shape[0]
    K = np.eye(s * s) - np.kron(N.T, M)
    d = np.linalg.solve(K, C.reshape(-1, order="F"))
    return d.reshape(s, s, order="F")


def stein_smith(M, N, C, steps: int, tol: float = 1e-16):
    """Solve D - M D N = C by Smith's doubling with at most ``steps`` doublings (2^steps terms).

    The factors are rebalanced at every doubling (M_j c, N_j / c leaves every term unchanged).  Stops
    when the newest block of terms M_j D_j N_j falls below tol ||D_j||; gives up when it exceeds
    1e10 ||D_j|| (the series diverges when the spectral radii of M and N multiply to more than one;
    single blocks may grow transiently, the factors being far from normal).
    Returns (D, converged)."""
    D, Mj, Nj = C.copy(), M.copy(), N.copy()
    for _ in range(steps):
        c = np.sqrt(max(np.linalg.norm(Nj), 1e-300) / max(np.linalg.norm(Mj), 1e-300))
        Mj, Nj = Mj * c, Nj / c
        term = Mj @ D @ Nj
        tn, dn = np.linalg.norm(term), np.linalg.norm(D)
        if not np.isfinite(tn) or tn > 1e10 * dn:
            return D, False
        D = D + term
        if tn <= tol * dn:
            return D, True
        Mj = Mj @ Mj
        Nj = Nj @ Nj
    return D, False


def fixed_point_parts(a0, c, cp, sigma):
    """(F, M, N) for Sigma = c (a0 - Sigma)^{-1} cp: F = Sigma - c N, M = c g, N = g cp, g = (a0 - Sigma)^{-1}."""
    g = np.linalg.inv(a0 - sigma)
    N = g @ cp
    M = c @ g
    return sigma - c @ N, M, N


def newton_selfenergy(a0, a1, am1, sigma_l0, sigma_r0, tol: float = 1e-10, max_newton: int = 12,
                      stein: str = "smith", smith_steps: int = 40):
    """Newton's method for both leads from (sigma_l0, sigma_r0).

    Right lead: Sigma_R = a1 (a0 - Sigma_R)^{-1} am1; left lead: Sigma_L = am1 (a0 - Sigma_L)^{-1} a1.
    Stops a side when ||F||_F <= tol ||Sigma||_F.  Returns dict(sigma_l, sigma_r, iters=(l, r),
    resid=(l, r), converged=(l, r))."""
    out = {}
    for name, sig0, c, cp in (("l", sigma_l0, am1, a1), ("r", sigma_r0, a1, am1)):
        sig = np.array(sig0, dtype=np.complex128)
        it, res, conv = 0, np.inf, False
        for it in range(max_newton + 1):
            F, M, N = fixed_point_parts(a0, c, cp, sig)
            res = float(np.linalg.norm(F) / max(np.linalg.norm(sig), 1e-300))
            if res <= tol:
                conv = True
                break
            if it == max_newton or not np.isfinite(res):
                break
            if stein == "kron":
                D = stein_kron(M, N, -F)
            else:
                D, ok = stein_smith(M, N, -F, smith_steps)
                if not ok:
                    break
            sig = sig + D
        out[name] = (sig, it, res, conv)
    return dict(sigma_l=out["l"][0], sigma_r=out["r"][0], iters=(out["l"][1], out["r"][1]),
                resid=(out["l"][2], out["r"][2]), converged=(out["l"][3], out["r"][3]))
