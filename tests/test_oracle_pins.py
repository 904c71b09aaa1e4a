"""Pins of the CPU oracle against facts fixed by the mathematics and the physics (no GPU).

Each test is chosen so that a plausible slip in the oracle (a sign in the decimation, a swapped
lead, a transposed coupling, a wrong corner block, a dropped Sigma) fails at least one of them.
"""
import numpy as np
import pytest

import synth
from oracle import bands, linalg, selfenergy, transport


def _solve(inst, E, eta=1e-8, inj=None):
    return transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01,
                                    inst.S00, inst.S01, E, eta, inj=inj)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("E", [-2.0, -0.7, 0.1, 0.9, 2.3, -3.5, 3.1, 4.0])
def test_scalar_chain_selfenergy_closed_form(E):
    """One-orbital chain (onsite eps0, hopping -t): Sigma = a/2 - i sqrt(t^2 - a^2/4) inside the band
    |a| < 2t (a = E - eps0), and the decaying root (a - sign(a) sqrt(a^2 - 4t^2))/2 outside."""
    eps0, t = 0.3, 1.2
    cell = synth.scalar_chain_cell(eps0, t)
    a0, a1, am1 = selfenergy.lead_blocks(*cell, E, 1e-12)
    sl, sr, iters, conv = selfenergy.decimation(a0, a1, am1)
    assert conv
    a = E - eps0
    if abs(a) < 2 * t:
        exact = a / 2 - 1j * np.sqrt(t * t - a * a / 4)
    else:
        exact = (a - np.sign(a) * np.sqrt(a * a - 4 * t * t)) / 2
    assert abs(sr[0, 0] - exact) < 1e-9
    assert abs(sl[0, 0] - exact) < 1e-9


@pytest.mark.parametrize("E,expect", [(-1.5, 1.0), (0.0, 1.0), (1.9, 1.0), (3.0, 0.0), (-2.6, 0.0)])
def test_scalar_chain_transmission(E, expect):
    """A perfect one-orbital chain transmits exactly one channel inside its band and nothing outside."""
    cell = synth.scalar_chain_cell(0.3, 1.2)
    inst = synth.device_from_cell(cell, 6)
    out = _solve(inst, E, eta=1e-10)
    assert abs(out["t_lr"] - expect) < 1e-8
    assert abs(out["t_rl"] - expect) < 1e-8


def test_ladder_counts_and_gauge():
    """s decoupled chains: T(E) = #{k : |E - eps_k| < 2 t_k}; a unitary change of basis leaves T unchanged."""
    rng = np.random.default_rng(11)
    s = 9
    eps = rng.uniform(-1.5, 1.5, s)
    t = rng.uniform(0.4, 1.3, s)
    cell = synth.ladder_cell(eps, t)
    inst = synth.device_from_cell(cell, 5)
    u = synth.random_unitary(s, 3)
    rot = synth.gauge_rotate(inst, u)
    for E in (-2.1, -0.4, 0.35, 1.7):
        d = np.abs(E - eps) - 2 * t
        if np.min(np.abs(d)) < 1e-3:
            continue
        expect = int(np.sum(d < 0))
        out = _solve(inst, E, eta=1e-10)
        out_rot = _solve(rot, E, eta=1e-10)
        assert abs(out["t_lr"] - expect) < 1e-8
        assert abs(out_rot["t_lr"] - expect) < 1e-8
        assert abs(out_rot["t_rl"] - expect) < 1e-8


# ---------------------------------------------------------------- physics: perfect crystals

def test_crystal_chain_recipe_integer_transmission():
    """Random 16-orbital chain crystal (device = lead): T(E) equals the band-crossing count at all 64 energies."""
    cell = synth.chain_cell(16, 0)
    inst = synth.device_from_cell(cell, 32)
    q = np.linspace(-np.pi, np.pi, 2048, endpoint=False)
    bb = bands.bloch_bands(*cell, q)
    seen = set()
    for E in np.linspace(-3, 3, 64):
        nch, gap = bands.channel_count(*cell, E, bands=bb)
        out = _solve(inst, E)
        assert abs(out["t_lr"] - nch) < 1e-8, (E, out["t_lr"], nch)
        assert abs(out["t_rl"] - nch) < 1e-8, (E, out["t_rl"], nch)
        seen.add(nch)
    assert len(seen) >= 4  # the grid really spans several channel counts


@pytest.mark.parametrize("s,seed,k", [(24, 5, 0.4), (40, 6, 1.3)])
def test_crystal_dft_like_integer_transmission(s, seed, k):
    """Lattice-slab crystal with a non-trivial SPD overlap: T(E) = band-crossing count."""
    cell = synth.dft_like_cell(s, seed, k)
    inst = synth.device_from_cell(cell, 4)
    q = np.linspace(-np.pi, np.pi, 4096, endpoint=False)
    bb = bands.bloch_bands(*cell, q)
    tested = 0
    for E in np.linspace(-6, 6, 13):
        # skip energies where two grid resolutions disagree (E too close to a band extremum)
        nch, _ = bands.channel_count(*cell, E, bands=bb)
        nch2, _ = bands.channel_count(*cell, E, nq=1024)
        if nch != nch2:
            continue
        out = _solve(inst, E)
        assert abs(out["t_lr"] - nch) < 1e-7, (E, out["t_lr"], nch)
        assert abs(out["t_rl"] - nch) < 1e-7
        tested += 1
    assert tested >= 10


# ---------------------------------------------------------------- brute force on tiny inputs

def _dense(inst, E):
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    return ad, au, al, linalg.assemble_dense(ad, au, al)


@pytest.mark.parametrize("nb,s", [(1, 5), (2, 3), (5, 7), (9, 4)])
def test_btd_solve_against_dense(nb, s):
    inst = synth.random_btd(nb, s, seed=nb * 10 + s)
    ad, au, al, a = _dense(inst, 0.37)
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal((nb, s, 3)) + 1j * rng.standard_normal((nb, s, 3))
    x = linalg.btd_solve(ad, au, al, rhs)
    xd = np.linalg.solve(a, rhs.reshape(nb * s, 3)).reshape(nb, s, 3)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


@pytest.mark.parametrize("nb,s", [(1, 4), (3, 5), (6, 6)])
def test_first_last_columns_are_inverse_columns(nb, s):
    inst = synth.random_btd(nb, s, seed=3 + nb)
    ad, au, al, a = _dense(inst, -0.21)
    q = transport.first_last_columns(ad, au, al)
    inv = np.linalg.inv(a)
    n = nb * s
    ref = np.concatenate([inv[:, :s], inv[:, n - s:]], axis=1).reshape(nb, s, 2 * s)
    assert np.linalg.norm(q - ref) <= 1e-11 * np.linalg.norm(ref)


def test_mirrored_columns_against_dense():
    inst = synth.random_btd(5, 4, seed=61)
    ad, au, al, a = _dense(inst, 0.11)
    q = transport.first_last_columns_mirrored(ad, au, al)
    inv = np.linalg.inv(a)
    ref = np.concatenate([inv[:, :4], inv[:, -4:]], axis=1).reshape(5, 4, 8)
    assert np.linalg.norm(q - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("nb,s", [(1, 4), (4, 5), (7, 3)])
def test_corner_greens_and_psi_against_dense(nb, s):
    inst = synth.random_btd(nb, s, seed=20 + nb)
    E, eta = 0.15, 1e-8
    out = _solve(inst, E, eta, inj=synth.injection_block(s, 3, 4))
    ad, au, al, a = _dense(inst, E)
    n = nb * s
    t = a.copy()
    t[:s, :s] -= out["sigma_l"]
    t[n - s:, n - s:] -= out["sigma_r"]
    g = np.linalg.inv(t)
    gc = np.block([[g[:s, :s], g[:s, n - s:]], [g[n - s:, :s], g[n - s:, n - s:]]])
    assert np.linalg.norm(out["gc"] - gc) <= 1e-10 * np.linalg.norm(gc)
    b = np.zeros((n, 3), np.complex128)
    inj = synth.injection_block(s, 3, 4)
    b[:s] += inj[:s]
    b[n - s:] += inj[s:]
    psi = np.linalg.solve(t, b).reshape(nb, s, 3)
    assert np.linalg.norm(out["psi"] - psi) <= 1e-10 * np.linalg.norm(psi)
    # Caroli from the dense inverse, written with explicit index sums (no matrix products)
    gl = 1j * (out["sigma_l"] - out["sigma_l"].conj().T)
    gr = 1j * (out["sigma_r"] - out["sigma_r"].conj().T)
    g1n = g[:s, n - s:]
    tlr = sum(gl[i, j] * g1n[j, k] * gr[k, l] * np.conj(g1n[i, l])
              for i in range(s) for j in range(s) for k in range(s) for l in range(s))
    assert abs(out["t_lr"] - tlr.real) < 1e-10 * max(1.0, abs(tlr))


def test_smw_identities():
    """Sec. 3B, Eq. (x): T^{-1} B = Q R^{-1} and T^{-1} b = Q (b' + z) with R = 1 - CQ, z = R^{-1} C Q b'."""
    inst = synth.random_btd(6, 5, seed=42)
    E, eta = -0.4, 1e-8
    inj = synth.injection_block(5, 4, 9)
    out = _solve(inst, E, eta, inj=inj)
    q = out["q"]
    r, z = transport.smw_terms(q, out["sigma_l"], out["sigma_r"], inj)
    qc = np.vstack([q[0], q[-1]])
    gc = qc @ np.linalg.inv(r)
    assert np.linalg.norm(gc - out["gc"]) <= 1e-10 * np.linalg.norm(out["gc"])
    psi = np.einsum("nij,jm->nim", q, inj + z)
    assert np.linalg.norm(psi - out["psi"]) <= 1e-10 * np.linalg.norm(out["psi"])


def _absorbing_split(inst, E, sigma_l, sigma_r, inj, absorb):
    """The split T = A' - B C' of Sec. 3B with the constant part -i*absorb*I of both self-energies moved
    into A: A' = A + i*absorb*I on the first and last diagonal blocks, C' = Sigma + i*absorb*I.
    Returns (corner Q' R'^{-1}, psi Q' (b' + z'))."""
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    eye = np.eye(ad.shape[1])
    ad2 = ad.copy()
    ad2[0] = ad2[0] + 1j * absorb * eye
    ad2[-1] = ad2[-1] + 1j * absorb * eye
    q = transport.first_last_columns(ad2, au, al)
    r, z = transport.smw_terms(q, sigma_l + 1j * absorb * eye, sigma_r + 1j * absorb * eye, inj)
    gc = np.vstack([q[0], q[-1]]) @ np.linalg.inv(r)
    return gc, np.einsum("nij,jm->nim", q, inj + z)


@pytest.mark.parametrize("absorb", [0.3, 1.0, 4.0])
@pytest.mark.parametrize("nb", [1, 2, 6])
def test_smw_with_absorbing_boundary(absorb, nb):
    """Sec. 3B leaves B and C free: moving -i*absorb*I of the self-energies from C into A (A' - B C' = T)
    gives the same corner of T^{-1} and the same psi, for any absorb and also for a single block (where
    both shifts land on the one diagonal block)."""
    inst = synth.random_btd(nb, 5, seed=44 + nb)
    E, eta = 0.25, 1e-8
    inj = synth.injection_block(5, 3, 10)
    out = _solve(inst, E, eta, inj=inj)
    gc, psi = _absorbing_split(inst, E, out["sigma_l"], out["sigma_r"], inj, absorb)
    assert np.linalg.norm(gc - out["gc"]) <= 1e-10 * np.linalg.norm(out["gc"])
    assert np.linalg.norm(psi - out["psi"]) <= 1e-10 * np.linalg.norm(out["psi"])


@pytest.mark.parametrize("which", [100, 260, 400])
def test_absorbing_boundary_next_to_closed_device_eigenvalue(which):
    """At E within 1e-11 of an eigenvalue of the closed device (E S - H singular) the correction of the
    closed split loses digits in proportion to the conditioning of A (here 1e-5 and worse in T, the
    instance itself being well posed), while the absorbing split, whose A' has no real eigenvalues,
    stays at rounding level.  Crystal of the 16-orbital chain cell, 32 blocks: T is an integer."""
    cell = synth.chain_cell(16, 0)
    inst = synth.device_from_cell(cell, 32)
    h = linalg.assemble_dense(inst.Hd, inst.Hu, np.conj(np.transpose(inst.Hu, (0, 2, 1))))
    E = float(np.linalg.eigvalsh(h)[which]) + 1e-11
    ref = _solve(inst, E)
    zero = np.zeros((32, 1), dtype=np.complex128)
    errs = {}
    for absorb in (0.0, 1.0):
        gc, _ = _absorbing_split(inst, E, ref["sigma_l"], ref["sigma_r"], zero, absorb)
        t_lr, t_rl = transport.caroli(gc, ref["sigma_l"], ref["sigma_r"])
        errs[absorb] = max(abs(t_lr - ref["t_lr"]), abs(t_rl - ref["t_rl"]))
    assert abs(ref["t_lr"] - round(ref["t_lr"])) <= 1e-6  # O(eta) from the integer channel count
    assert errs[1.0] <= 1e-12
    assert errs[0.0] >= 1e-7  # the closed split really is ill-conditioned here


def test_alg1_reading_reproduces_first_and_last_columns():
    """Readings of Alg. 1 (Sec. 3B): X_{n_B+1} = 0, A_{1,0} := 1 and Q_0 = -1 give the first block column;
    the mirrored recursion with A_{n_B,n_B+1} := 1 gives the last one."""
    nb, s = 6, 4
    inst = synth.random_btd(nb, s, seed=8)
    ad, au, al, a = _dense(inst, 0.3)
    eye = np.eye(s)
    x = [None] * (nb + 2)
    x[nb + 1] = np.zeros((s, s))
    for i in range(nb, 0, -1):
        rhs = eye if i == 1 else al[i - 2]
        up = au[i - 1] if i < nb else np.zeros((s, s))
        x[i] = np.linalg.solve(ad[i - 1] - up @ x[i + 1], rhs)
    qf = [-eye]
    for i in range(1, nb + 1):
        qf.append(-x[i] @ qf[-1])
    y = [np.zeros((s, s))] * (nb + 2)
    for i in range(1, nb + 1):
        rhs = eye if i == nb else au[i - 1]
        lo = al[i - 2] if i > 1 else np.zeros((s, s))
        y[i] = np.linalg.solve(ad[i - 1] - lo @ y[i - 1], rhs)
    ql = [None] * (nb + 2)
    ql[nb + 1] = -eye
    for i in range(nb, 0, -1):
        ql[i] = -y[i] @ ql[i + 1]
    q = np.stack([np.hstack([qf[i], ql[i]]) for i in range(1, nb + 1)])
    ref = transport.first_last_columns(ad, au, al)
    assert np.linalg.norm(q - ref) <= 1e-11 * np.linalg.norm(ref)


# ---------------------------------------------------------------- self-energy routes and invariants

@pytest.mark.parametrize("E", [-1.1, 0.2, 1.4])
def test_decimation_agrees_with_mode_route(E):
    """Two independent routes to Sigma (decimation vs lead modes of the quadratic pencil) agree to O(eta)."""
    cell = synth.chain_cell(8, 3)
    a0, a1, am1 = selfenergy.lead_blocks(*cell, E, 1e-9)
    sl, sr, _, conv = selfenergy.decimation(a0, a1, am1)
    assert conv
    ml, mr, _ = selfenergy.selfenergy_modes(a0, a1, am1)
    assert np.linalg.norm(sr - mr) <= 1e-6 * np.linalg.norm(mr)
    assert np.linalg.norm(sl - ml) <= 1e-6 * np.linalg.norm(ml)
    rl, rr = selfenergy.quadratic_residuals(a0, a1, am1, sl, sr)
    assert rl < 1e-10 and rr < 1e-10
    assert selfenergy.is_retarded(a0, a1, am1, sl, sr)


def test_dft_like_selfenergy_with_overlap():
    """Same two routes with a non-identity overlap in the lead (S01 != 0)."""
    cell = synth.dft_like_cell(24, 2, 0.9)
    a0, a1, am1 = selfenergy.lead_blocks(*cell, 0.7, 1e-9)
    sl, sr, _, conv = selfenergy.decimation(a0, a1, am1)
    assert conv
    ml, mr, _ = selfenergy.selfenergy_modes(a0, a1, am1)
    assert np.linalg.norm(sr - mr) <= 1e-6 * np.linalg.norm(mr)
    assert np.linalg.norm(sl - ml) <= 1e-6 * np.linalg.norm(ml)
    rl, rr = selfenergy.quadratic_residuals(a0, a1, am1, sl, sr)
    assert rl < 1e-10 and rr < 1e-10


def test_non_retarded_root_is_rejected():
    """The fixed-point equation has other roots; the retardedness check must reject one of them."""
    cell = synth.scalar_chain_cell(0.0, 1.0)
    a0, a1, am1 = selfenergy.lead_blocks(*cell, 0.5, 1e-9)
    sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
    assert selfenergy.is_retarded(a0, a1, am1, sl, sr)
    other = np.conj(sr)  # the advanced root of the same quadratic (Gamma <= 0)
    assert not selfenergy.is_retarded(a0, a1, am1, sl, other)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_disordered_device_invariants(seed):
    """T_LR = T_RL (unitarity), 0 <= T <= s, Gamma positive semi-definite."""
    inst = synth.random_btd(5, 6, seed=100 + seed)
    for E in (-0.8, 0.05, 0.9):
        out = _solve(inst, E)
        assert abs(out["t_lr"] - out["t_rl"]) < 1e-10 * max(1.0, out["t_lr"])
        assert -1e-12 <= out["t_lr"] <= 6 + 1e-10
        for sig in (out["sigma_l"], out["sigma_r"]):
            assert np.linalg.eigvalsh(selfenergy.broadening(sig)).min() > -1e-12


def test_reversal_swaps_directions():
    """Reversing the block order (and mirroring the lead cell) exchanges T_LR and T_RL."""
    inst = synth.random_btd(5, 4, seed=77)
    inst.Hd[2] += np.diag(np.linspace(-0.5, 0.5, 4))
    rev = synth.BTDInstance(
        inst.Hd[::-1].copy(), np.conj(np.transpose(inst.Hu[::-1], (0, 2, 1))).copy(),
        inst.Sd[::-1].copy(), np.conj(np.transpose(inst.Su[::-1], (0, 2, 1))).copy(),
        inst.H00, inst.H01.conj().T.copy(), inst.S00, inst.S01.conj().T.copy())
    for E in (-0.3, 0.6):
        a = _solve(inst, E)
        b = _solve(rev, E)
        assert abs(a["t_lr"] - b["t_rl"]) < 1e-10
        assert abs(a["t_rl"] - b["t_lr"]) < 1e-10


def test_energy_scaling_invariance():
    """Scaling (H, E, eta) by c > 0 with S fixed scales A, Sigma and Gamma by c and leaves T unchanged."""
    inst = synth.random_btd(4, 5, seed=5)
    c = 3.7
    scaled = synth.BTDInstance(c * inst.Hd, c * inst.Hu, inst.Sd, inst.Su, c * inst.H00, c * inst.H01,
                               inst.S00, inst.S01)
    a = _solve(inst, 0.25, 1e-8)
    b = _solve(scaled, 0.25 * c, 1e-8 * c)
    assert abs(a["t_lr"] - b["t_lr"]) < 1e-10
    assert np.linalg.norm(b["sigma_r"] - c * a["sigma_r"]) < 1e-9 * np.linalg.norm(b["sigma_r"])


def test_golden_chain16_channels_match_oracle_transmission():
    """The stored channel counts (tests/golden/chain16_channels.txt, from the band structure) equal the
    oracle's Caroli transmission of the 32-block crystal at every stored energy."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "chain16_channels.txt")
    rows = np.loadtxt(path, comments="#")
    cell = synth.chain_cell(16, 0)
    inst = synth.device_from_cell(cell, 32)
    for E, nch, _gap in rows[::7]:
        out = _solve(inst, E)
        assert abs(out["t_lr"] - nch) < 1e-8


def test_decimation_conditioning_pins():
    """The conditioning estimate used for tolerances: exactly 1 for a one-orbital chain, and for a
    decoupled ladder equal to the worst ratio over the passes of the scalar chains' bulk energies
    (each chain decimated on its own in scalar arithmetic)."""
    cell = synth.scalar_chain_cell(0.2, 1.0)
    a0, a1, am1 = selfenergy.lead_blocks(*cell, 0.4, 1e-8)
    assert selfenergy.decimation_conditioning(a0, a1, am1) == pytest.approx(1.0)
    eps0 = np.array([-0.5, 0.3, 1.1])
    t = np.array([0.4, 0.9, 0.7])
    E, eta = 0.25, 1e-6
    a0, a1, am1 = selfenergy.lead_blocks(*synth.ladder_cell(eps0, t), E, eta)
    est = selfenergy.decimation_conditioning(a0, a1, am1)
    # scalar recursions e <- e - 2 a b / e, a <- -a^2/e, b <- -b^2/e per chain
    e = (E + 1j * eta) - eps0
    al = t.astype(complex)
    be = t.astype(complex)
    worst = 1.0
    for _ in range(200):
        worst = max(worst, np.max(np.abs(e)) / np.min(np.abs(e)))
        e, al, be = e - 2 * al * be / e, -al * al / e, -be * be / e
        if np.max(np.abs(al)) + np.max(np.abs(be)) <= 1e-14 * np.max(np.abs((E + 1j * eta) - eps0)):
            break
    assert est == pytest.approx(worst, rel=1e-8)


def _perm_from_ipiv(ipiv):
    perm = np.arange(len(ipiv))
    for j, p in enumerate(ipiv):
        perm[[j, p]] = perm[[p, j]]
    return perm


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (64, 2), (150, 3)])
def test_lu_partial_pivot_matches_lapack_getrf(n, seed):
    """The written-out elimination takes LAPACK's pivots (izamax: largest |Re| + |Im|, first on ties)
    and reproduces its factors and P a = L U."""
    import scipy.linalg as sla
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lu, perm, info = linalg.lu_partial_pivot(a)
    ref, ipiv = sla.lu_factor(a)
    assert info == 0
    assert np.array_equal(perm, _perm_from_ipiv(ipiv))
    assert np.abs(lu - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    assert np.abs(a[perm] - L @ U).max() <= 1e-12 * np.abs(a).max() * n


def test_lu_partial_pivot_tie_rule_and_zero_pivot():
    # column 0: |Re| + |Im| is 2 for rows 1, 2 and 3 (2, 2j, 1+1j): the lowest such row (1) is the pivot
    a = np.array([[0.5, 1.0, 0.0], [2.0, 0.0, 1.0], [2.0j, 1.0, 0.0], [1.0 + 1.0j, 0.0, 0.0]])[:, :3]
    a = np.concatenate([a, np.zeros((4, 1))], axis=1)  # 4 x 4 with a zero last column
    lu, perm, info = linalg.lu_partial_pivot(a)
    assert perm[0] == 1
    assert info == 4  # the last column is exactly zero after elimination
    # a zero column in the middle: recorded, skipped, elimination continues below it
    b = np.array([[1.0, 0.0, 2.0], [3.0, 0.0, 1.0], [0.5, 0.0, 4.0]], dtype=complex)
    lu, perm, info = linalg.lu_partial_pivot(b)
    assert info == 2 and perm[0] == 1
    L = np.tril(lu, -1) + np.eye(3)
    assert np.allclose(b[perm], L @ np.triu(lu))


def test_golden_dft512_is_consistent():
    """The stored oracle transmissions of the s = 512 crystal (256 instances): T_LR = T_RL (an identity),
    T = the band-structure channel count up to O(eta) terms, and the block-Thomas values equal a dense LU
    solve of the assembled 20480 x 20480 open system on the two instances farthest from the integer."""
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    ref = np.loadtxt(os.path.join(here, "dft512_transmission.txt"), comments="#")
    assert ref.shape == (256, 8)
    assert np.abs(ref[:, 3] - ref[:, 4]).max() <= 1e-10
    assert np.abs(ref[:, 3] - ref[:, 6]).max() <= 1e-6
    assert (ref[:, 5] >= 20).all() and (ref[:, 5] <= 40).all()   # decimation passes at eta = 1e-8
    dense = np.loadtxt(os.path.join(here, "dft512_dense_check.txt"), comments="#")
    assert dense.shape[0] == 2
    for row in dense:
        b = int(row[0])
        assert np.allclose(row[3:5], ref[b, 3:5], rtol=0, atol=1e-14)
        assert np.abs(row[1:3] - row[3:5]).max() <= 1e-10
