"""Pins of the warm-start oracle (``oracle/warmstart.py``) against definitions it does not use itself.

* back-propagation against central differences of the loss (float64, every parameter of a small net);
* the first Adam step against its closed form (theta - lr * g / (|g| + eps));
* Smith's doubling against the Kronecker solution of the Stein equation, and both against the
  equation itself;
* Newton from a nearby start converges to the decimation's self-energy and to the independent mode
  route, with quadratic decrease of the residual; Smith's series diverges from such a start (the
  reason the GPU warm start falls back to the decimation) and reports it;
* a non-retarded root built from the lead modes (one growing mode in place of a decaying one) is an
  exact fixed point that the retardedness test rejects, and Newton started on it stays there.
"""
import numpy as np
import pytest

import synth
from oracle import selfenergy, warmstart


def test_features_shape_and_periodicity():
    E = np.array([-5.0, 0.0, 2.5])
    k = np.array([0.0, np.pi / 2, np.pi])
    f = warmstart.features(E, k, nfreq=8)
    assert f.shape == (3, 35)
    g = warmstart.features(E, k + 2 * np.pi, nfreq=8)
    assert np.allclose(f, g, atol=1e-12)  # k enters through its phase only


def test_sigma_encoding_round_trip():
    rng = np.random.default_rng(3)
    sl = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    sr = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    y = warmstart.encode_sigma(sl, sr)
    assert y.shape == (100,)
    dl, dr = warmstart.decode_sigma(y, 5)
    assert np.array_equal(dl, sl) and np.array_equal(dr, sr)


def test_backprop_against_central_differences():
    dims = [5, 7, 6, 7, 4]
    params = warmstart.mlp_init(dims, seed=1)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 4))
    _, grads = warmstart.mlp_loss_grad(params, X, T)
    h = 1e-6
    worst = 0.0
    for li in range(len(params)):
        for pi in range(2):
            base = params[li][pi]
            for idx in np.ndindex(base.shape):
                def loss_at(delta):
                    p2 = [(W.copy(), b.copy()) for W, b in params]
                    p2[li][pi][idx] += delta
                    return warmstart.mlp_loss_grad(p2, X, T)[0]
                fd = (loss_at(h) - loss_at(-h)) / (2 * h)
                an = grads[li][pi][idx]
                worst = max(worst, abs(fd - an) / max(1e-8, abs(fd) + abs(an)))
    assert worst < 1e-6, worst


def test_adam_first_step_closed_form():
    params = [(np.array([[1.0, -2.0]]), np.array([0.5, 0.0]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([1e-3, 0.0]))]
    state = {}
    lr, eps = 0.01, 1e-8
    new = warmstart.adam_step(params, grads, state, lr, eps=eps)
    for (p, g), q in zip(((params[0][0], grads[0][0]), (params[0][1], grads[0][1])), new[0]):
        # after one step the bias-corrected moments are g and g^2
        assert np.allclose(q, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert state["t"] == 1


def test_adam_second_step_worked_example():
    """Two steps on one scalar with gradients +1 then -1, beta1 = 0.9, beta2 = 0.999 (Kingma & Ba).
    Worked by hand: after step 2 the first moment is 0.9*0.1 - 0.1 = -0.01 and its bias correction
    1 - 0.81 = 0.19, so m_hat = -1/19; the second moment is 0.999*0.001 + 0.001 = 0.001999 with
    correction 1 - 0.998001 = 0.001999, so v_hat = 1 exactly.  Step 1 moves by -lr/(1 + eps), step 2 by
    +lr/19/(1 + eps).  A beta1/beta2 slip in either moment, or a bias correction taken at t = 1 again,
    changes the second move."""
    lr, eps = 0.01, 1e-8
    params = [(np.array([[0.0]]), np.array([0.0]))]
    state = {}
    p1 = warmstart.adam_step(params, [(np.array([[1.0]]), np.array([1.0]))], state, lr, eps=eps)
    p2 = warmstart.adam_step(p1, [(np.array([[-1.0]]), np.array([-1.0]))], state, lr, eps=eps)
    first = -lr / (1.0 + eps)
    assert abs(p1[0][0][0, 0] - first) <= 1e-17
    assert abs(p2[0][0][0, 0] - (first + lr / 19.0 / (1.0 + eps))) <= 1e-17
    assert abs(p2[0][1][0] - p2[0][0][0, 0]) == 0.0
    assert state["t"] == 2


def _contracting_pair(s, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s))
    N = rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s))
    M *= 0.9 / np.max(np.abs(np.linalg.eigvals(M)))
    N *= 0.8 / np.max(np.abs(np.linalg.eigvals(N)))
    C = rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s))
    return M, N, C


def test_stein_routes_agree_and_solve_the_equation():
    M, N, C = _contracting_pair(6, 4)
    dk = warmstart.stein_kron(M, N, C)
    ds, ok = warmstart.stein_smith(M, N, C, steps=12)
    assert ok
    for d in (dk, ds):
        assert np.linalg.norm(d - M @ d @ N - C) <= 1e-12 * np.linalg.norm(C)
    assert np.linalg.norm(dk - ds) <= 1e-12 * np.linalg.norm(dk)


def _lead(E=0.3, k=0.7, eta=1e-8):
    cell = synth.DFTLikeCell(synth.SLAB_SHAPES[24], 4).at(k)
    return selfenergy.lead_blocks(*cell, E, eta)


def test_newton_converges_to_the_retarded_selfenergy():
    """Exact Newton (Kronecker Stein solves) from the self-energy at a 1000x larger broadening."""
    a0, a1, am1 = _lead()
    sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
    ml, mr, _ = selfenergy.selfenergy_modes(a0, a1, am1)
    b0, b1, bm1 = _lead(eta=1e-5)
    l0, r0, _, _ = selfenergy.decimation(b0, b1, bm1)
    assert np.linalg.norm(r0 - sr) > 1e-5 * np.linalg.norm(sr)  # a genuinely different start
    r = warmstart.newton_selfenergy(a0, a1, am1, l0, r0, stein="kron")
    assert all(r["converged"]) and max(r["iters"]) <= 3, r["iters"]
    assert np.linalg.norm(r["sigma_r"] - sr) <= 1e-9 * np.linalg.norm(sr)
    assert np.linalg.norm(r["sigma_l"] - sl) <= 1e-9 * np.linalg.norm(sl)
    assert np.linalg.norm(r["sigma_r"] - mr) <= 1e-6 * np.linalg.norm(mr)  # mode route: O(eta)
    assert selfenergy.is_retarded(a0, a1, am1, r["sigma_l"], r["sigma_r"])


def test_smith_series_diverges_near_the_retarded_root():
    """At the retarded root the spectral radii of M and N multiply to 1 - O(eta); a start a little away
    from it pushes the product above one, so the Neumann (Smith) series of the Stein equation diverges
    although the equation itself is well posed: the doubling reports failure instead of a value."""
    a0, a1, am1 = _lead()
    sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
    _, M, N = warmstart.fixed_point_parts(a0, a1, am1, sr)
    prod = np.max(np.abs(np.linalg.eigvals(M))) * np.max(np.abs(np.linalg.eigvals(N)))
    assert 1 - 1e-6 < prod < 1
    b0, b1, bm1 = _lead(eta=1e-5)
    _, r0, _, _ = selfenergy.decimation(b0, b1, bm1)
    F, M, N = warmstart.fixed_point_parts(a0, a1, am1, r0)
    assert np.max(np.abs(np.linalg.eigvals(M))) * np.max(np.abs(np.linalg.eigvals(N))) > 1
    d, ok = warmstart.stein_smith(M, N, -F, steps=40)
    assert not ok and np.all(np.isfinite(d))
    dk = warmstart.stein_kron(M, N, -F)
    assert np.linalg.norm(dk - M @ dk @ N + F) <= 1e-10 * np.linalg.norm(F)


def test_newton_residual_decreases_quadratically():
    a0, a1, am1 = _lead(E=-1.0)
    sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
    sig = sr * (1 + 3e-3)
    res = []
    for _ in range(3):
        F, M, N = warmstart.fixed_point_parts(a0, a1, am1, sig)
        res.append(np.linalg.norm(F) / np.linalg.norm(sig))
        sig = sig + warmstart.stein_kron(M, N, -F)
    assert res[1] <= 100 * res[0] ** 2 and res[2] <= 100 * res[1] ** 2 + 1e-14, res


def test_non_retarded_fixed_point_is_rejected():
    """A root of the quadratic built from one growing mode is an exact fixed point: Newton keeps it,
    the retardedness test rejects it."""
    a0, a1, am1 = _lead(E=0.3)
    s = a0.shape[0]
    eye, zero = np.eye(s), np.zeros((s, s))
    import scipy.linalg as sla
    lam, vec = sla.eig(np.block([[zero, eye], [-am1, -a0]]), np.block([[eye, zero], [zero, a1]]))
    order = np.argsort(np.abs(lam))
    keep = np.concatenate([order[: s - 1], order[s: s + 1]])  # s-1 decaying modes and one growing one
    u = vec[:s, keep]
    Lam = u @ np.diag(lam[keep]) @ np.linalg.inv(u)
    bad_r = -a1 @ Lam
    F, _, _ = warmstart.fixed_point_parts(a0, a1, am1, bad_r)
    assert np.linalg.norm(F) <= 1e-8 * np.linalg.norm(bad_r)
    sl, _, _, _ = selfenergy.decimation(a0, a1, am1)
    assert not selfenergy.is_retarded(a0, a1, am1, sl, bad_r)
    r = warmstart.newton_selfenergy(a0, a1, am1, sl, bad_r, stein="kron")
    assert r["converged"][1] and not selfenergy.is_retarded(a0, a1, am1, r["sigma_l"], r["sigma_r"])
