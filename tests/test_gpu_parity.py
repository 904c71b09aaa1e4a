"""Parity of the HIP path (through the C ABI) against the CPU oracle, element by element.

Tolerances (FP64 path): relative Frobenius error <= 1e-10 for Q, Sigma, the corner of G^R and psi;
|T - T_ref| / max(1, T_ref) <= 1e-10.  Inputs are seeded synthetic instances from ``synth``; sizes
span several 64-wide tiles, a ragged tail and the degenerate nb = 1 case.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import linalg, selfenergy, transport

pytestmark = pytest.mark.gpu

TOL = 1e-10
UNIT = 2.0 ** -52


def sigma_tol(cell, E, eta):
    """Comparison tolerance for Sigma and everything downstream of it: max(1e-10, 10 u kappa_max),
    kappa_max = the worst condition of the decimation's solves (two correct runs drift by u kappa)."""
    a0, a1, am1 = selfenergy.lead_blocks(*cell, E, eta)
    return max(TOL, 10 * UNIT * selfenergy.decimation_conditioning(a0, a1, am1))


@pytest.fixture(scope="module")
def ctx():
    import paper_1812_01396_amd as ss
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = ss.Context(0)
    yield c
    c.close()


def _dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _stack_sets(insts):
    return [np.stack([getattr(i, f) for i in insts]) for f in ("Hd", "Hu", "Sd", "Su")]


def _shifted_blocks(inst, E, absorb):
    """Blocks of A' = E S - H + i*absorb*I on the first and last diagonal blocks (absorbing boundary)."""
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    ad = ad.copy()
    eye = np.eye(ad.shape[1])
    ad[0] = ad[0] + 1j * absorb * eye
    ad[-1] = ad[-1] + 1j * absorb * eye
    return ad, au, al


@pytest.mark.parametrize("nb,s,absorb", [(1, 5, 0.0), (2, 16, 0.0), (5, 40, 0.0), (3, 72, 0.0), (4, 130, 0.0),
                                         (2, 33, 0.0), (1, 5, 0.7), (5, 40, 0.7), (4, 130, 1.3)])
def test_precompute_columns_vs_oracle(ctx, nb, s, absorb):
    import paper_1812_01396_amd as ss
    print(f"precompute nb={nb} s={s} absorb={absorb}", flush=True)
    insts = [synth.random_btd(nb, s, seed=1000 + 7 * nb + s + k) for k in range(2)]
    Es = np.array([0.31, -0.47, 0.05])
    kidx = np.array([0, 1, 1], dtype=np.int32)
    hd, hu, sd, su = _stack_sets(insts)
    q, info = ss.ss_precompute_columns(ctx, _dev(hd), _dev(hu), _dev(sd), _dev(su), _dev(Es, torch.float64),
                                       kidx=_dev(kidx, torch.int32), absorb=absorb)
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    assert (info.cpu().numpy() == 0).all()
    for b, (E, k) in enumerate(zip(Es, kidx)):
        ref = transport.first_last_columns(*_shifted_blocks(insts[k], E, absorb))
        assert _rel(q[b], ref) <= TOL, (b, _rel(q[b], ref))


@pytest.mark.parametrize("width", [16, 8])
def test_precompute_columns_panel_widths(ctx, width):
    """Alg. 1 with the narrower LU panels (substitution-free matrix-core leaves of 16 or 8 rows instead of
    the fused 64-row ones) agrees with the oracle as the default width does."""
    import paper_1812_01396_amd as ss
    nb, s = 3, 130
    print(f"precompute width={width} nb={nb} s={s}", flush=True)
    insts = [synth.random_btd(nb, s, seed=2000 + width + k) for k in range(2)]
    Es = np.array([0.21, -0.38])
    kidx = np.array([0, 1], dtype=np.int32)
    hd, hu, sd, su = _stack_sets(insts)
    ctx.set_lu_width(width)
    try:
        q, info = ss.ss_precompute_columns(ctx, _dev(hd), _dev(hu), _dev(sd), _dev(su), _dev(Es, torch.float64),
                                           kidx=_dev(kidx, torch.int32))
        torch.cuda.synchronize()
    finally:
        ctx.set_lu_width(0)
    q = q.cpu().numpy()
    assert (info.cpu().numpy() == 0).all()
    for b, (E, k) in enumerate(zip(Es, kidx)):
        ad, au, al = transport.device_blocks(insts[k].Hd, insts[k].Hu, insts[k].Sd, insts[k].Su, E)
        ref = transport.first_last_columns(ad, au, al)
        assert _rel(q[b], ref) <= TOL, (b, _rel(q[b], ref))


def test_precompute_columns_zero_pivot_code(ctx):
    """A decoupled device with E on an onsite level: exactly zero pivots, reported LAPACK-style."""
    import paper_1812_01396_amd as ss
    nb, s = 3, 4
    hd = np.repeat(np.diag([1.0, 2.0, 3.0, 4.0]).astype(np.complex128)[None], nb, 0)
    hu = np.zeros((nb - 1, s, s), np.complex128)
    sd = np.repeat(np.eye(s, dtype=np.complex128)[None], nb, 0)
    su = np.zeros_like(hu)
    E = np.array([2.0, 2.5])
    _, info = ss.ss_precompute_columns(ctx, _dev(hd), _dev(hu), _dev(sd), _dev(su), _dev(E, torch.float64))
    torch.cuda.synchronize()
    # E = 2: block 1 (first system of the last-column recursion) is diag(1, 0, -1, -2) -> column 2 of block 1
    assert info.cpu().tolist() == [2, 0]


@pytest.mark.parametrize("cell_kind,s", [("chain", 16), ("dft", 24), ("dft", 40), ("chain", 70)])
def test_selfenergy_vs_oracle(ctx, cell_kind, s):
    import paper_1812_01396_amd as ss
    print(f"selfenergy {cell_kind} s={s}", flush=True)
    cells = [synth.chain_cell(s, 5), synth.chain_cell(s, 6)] if cell_kind == "chain" else \
        [synth.dft_like_cell(s, 3, 0.4), synth.dft_like_cell(s, 3, 1.7)]
    Es = np.array([-1.3, 0.2, 0.9, 2.7]) if cell_kind == "chain" else np.array([-3.0, -0.5, 1.1, 4.2])
    kidx = np.array([0, 1, 0, 1], dtype=np.int32)
    eta = 1e-8
    h00, h01, s00, s01 = (np.stack([c[i] for c in cells]) for i in range(4))
    sig, iters, resid, info = ss.ss_lead_selfenergy(ctx, _dev(h00), _dev(h01), _dev(s00), _dev(s01),
                                                    _dev(Es, torch.float64), eta, kidx=_dev(kidx, torch.int32))
    torch.cuda.synchronize()
    sig = sig.cpu().numpy()
    assert (info.cpu().numpy() == 0).all(), info
    assert (resid.cpu().numpy() <= 1e-10).all(), resid
    for b, (E, k) in enumerate(zip(Es, kidx)):
        a0, a1, am1 = selfenergy.lead_blocks(*cells[k], E, eta)
        sl, sr, it, conv = selfenergy.decimation(a0, a1, am1)
        tol = sigma_tol(cells[k], E, eta)
        assert abs(int(iters[b]) - it) <= 1
        assert _rel(sig[b, 0], sl) <= tol, (b, _rel(sig[b, 0], sl), tol)
        assert _rel(sig[b, 1], sr) <= tol, (b, _rel(sig[b, 1], sr), tol)


def _pipeline(ctx, inst_sets, Es, kidx, eta, inj, absorb=0.0):
    import paper_1812_01396_amd as ss
    hd, hu, sd, su = _stack_sets(inst_sets)
    leads = [np.stack([getattr(i, f) for i in inst_sets]) for f in ("H00", "H01", "S00", "S01")]
    E_d, k_d = _dev(Es, torch.float64), _dev(kidx, torch.int32)
    sig, iters, resid, info_s = ss.ss_lead_selfenergy(ctx, *(_dev(x) for x in leads), E_d, eta, kidx=k_d)
    q, info_q = ss.ss_precompute_columns(ctx, _dev(hd), _dev(hu), _dev(sd), _dev(su), E_d, kidx=k_d, absorb=absorb)
    psi, gc, info_o = ss.ss_apply_obc(ctx, q, sig, inj=_dev(inj) if inj is not None else None, absorb=absorb)
    T = ss.ss_transmission(ctx, gc, sig)
    torch.cuda.synchronize()
    for i in (info_s, info_q, info_o):
        assert (i.cpu().numpy() == 0).all(), i
    return dict(sigma=sig.cpu().numpy(), q=q.cpu().numpy(), psi=None if psi is None else psi.cpu().numpy(),
                gc=gc.cpu().numpy(), T=T.cpu().numpy())


@pytest.mark.parametrize("nb,s,m,absorb", [(1, 6, 2, 0.0), (4, 40, 3, 0.0), (3, 72, 5, 0.0), (2, 100, 1, 0.0),
                                           (1, 6, 2, 1.0), (4, 40, 3, 1.0), (3, 72, 5, 0.5), (2, 100, 1, 2.0)])
def test_obc_psi_transmission_vs_oracle(ctx, nb, s, m, absorb):
    """The corner of G^R, psi and T do not depend on the split: the absorbing boundary (absorb > 0) gives
    the oracle's direct solve of the open system as the paper's split does."""
    print(f"pipeline nb={nb} s={s} m={m} absorb={absorb}", flush=True)
    insts = [synth.random_btd(nb, s, seed=2000 + s + k) for k in range(2)]
    Es = np.array([0.15, -0.35])
    kidx = np.array([0, 1], dtype=np.int32)
    eta = 1e-8
    inj = np.stack([synth.injection_block(s, m, 50 + b) for b in range(2)])
    out = _pipeline(ctx, insts, Es, kidx, eta, inj, absorb)
    for b in range(2):
        inst = insts[kidx[b]]
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                       inst.S01, Es[b], eta, inj=inj[b])
        tol = sigma_tol((inst.H00, inst.H01, inst.S00, inst.S01), Es[b], eta)
        assert _rel(out["gc"][b], ref["gc"]) <= tol, (b, _rel(out["gc"][b], ref["gc"]), tol)
        assert _rel(out["psi"][b], ref["psi"]) <= tol
        for j, key in enumerate(("t_lr", "t_rl")):
            assert abs(out["T"][b, j] - ref[key]) <= tol * max(1.0, abs(ref[key]))
            if absorb > 0:  # the benchmark's split meets the T target itself, whatever the tolerance allows
                assert abs(out["T"][b, j] - ref[key]) <= 1e-8 * max(1.0, abs(ref[key])), (b, key, tol)


@pytest.mark.parametrize("absorb", [0.0, 1.0])
def test_chain_crystal_all_energies(ctx, absorb):
    """Random 16-orbital chain, 32 blocks, 64 energies in [-3, 3]: T equals the stored channel counts."""
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "chain16_channels.txt"), comments="#")
    cell = synth.chain_cell(16, 0)
    inst = synth.device_from_cell(cell, 32)
    Es = rows[:, 0]
    out = _pipeline(ctx, [inst], Es, np.zeros(len(Es), np.int32), 1e-8, None, absorb)
    for b, E in enumerate(Es):
        assert abs(out["T"][b, 0] - rows[b, 1]) <= 1e-8, (E, out["T"][b], rows[b, 1])
        assert abs(out["T"][b, 1] - rows[b, 1]) <= 1e-8
    # and element-wise against the oracle on a sample of energies
    for b in range(0, len(Es), 9):
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, *cell, Es[b], 1e-8)
        q_ref = transport.first_last_columns(*_shifted_blocks(inst, Es[b], absorb)) if absorb else ref["q"]
        assert _rel(out["q"][b], q_ref) <= TOL
        assert abs(out["T"][b, 0] - ref["t_lr"]) <= TOL * max(1.0, ref["t_lr"])


@pytest.mark.parametrize("n,nmat", [(1, 2), (33, 3), (84, 2), (100, 2), (250, 2), (512, 3), (700, 2), (1100, 1),
                                    (1536, 1), (2048, 1)])
def test_lu_factor_vs_oracle(ctx, n, nmat):
    """The batched LU (panel widths 32, 16 and 8 by order) takes the oracle's pivots exactly and its
    factors agree element by element (rounding-order differences only).  Orders 84 and 250 end in
    panels of 20 and 26 columns: full and partial 8-column quarters.  Orders 1536 and 2048 (the corner
    systems of s = 768 and s = 1024) run the 8-column panel with two rows per thread."""
    import paper_1812_01396_amd as ss
    print(f"lu_factor n={n} nmat={nmat}", flush=True)
    rng = np.random.default_rng(n + nmat)
    a = rng.standard_normal((nmat, n, n)) + 1j * rng.standard_normal((nmat, n, n))
    lu, perm, info = ss.ss_lu_factor(ctx, _dev(a))
    torch.cuda.synchronize()
    lu, perm, info = lu.cpu().numpy(), perm.cpu().numpy(), info.cpu().numpy()
    for b in range(nmat):
        ref, rperm, rinfo = linalg.lu_partial_pivot(a[b])
        assert info[b] == rinfo == 0
        assert np.array_equal(perm[b], rperm), (b, int(np.argmax(perm[b] != rperm)))
        assert np.abs(lu[b] - ref).max() <= 1e-11 * np.abs(ref).max(), (b, np.abs(lu[b] - ref).max())


@pytest.mark.parametrize("width,n", [(16, 100), (16, 512), (16, 700), (8, 250), (8, 512), (32, 512)])
def test_lu_factor_panel_widths(ctx, width, n):
    """Every panel width a context (or a plan's autotuner) can choose gives the oracle's pivots and
    factors: 16-column panels with whole rows in registers, 8-column panels with two rows per thread."""
    import paper_1812_01396_amd as ss
    print(f"lu_factor width={width} n={n}", flush=True)
    rng = np.random.default_rng(width * 1000 + n)
    a = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    ctx.set_lu_width(width)
    try:
        lu, perm, info = ss.ss_lu_factor(ctx, _dev(a))
        torch.cuda.synchronize()
    finally:
        ctx.set_lu_width(0)
    lu, perm, info = lu.cpu().numpy(), perm.cpu().numpy(), info.cpu().numpy()
    for b in range(2):
        ref, rperm, rinfo = linalg.lu_partial_pivot(a[b])
        assert info[b] == rinfo == 0
        assert np.array_equal(perm[b], rperm), (b, int(np.argmax(perm[b] != rperm)))
        assert np.abs(lu[b] - ref).max() <= 1e-11 * np.abs(ref).max(), (b, np.abs(lu[b] - ref).max())


@pytest.mark.parametrize("n", [100, 512, 1100])
def test_lu_factor_half_tile(ctx, n):
    """The 32 x 64 product tile (ss_set_lu_tile(1), an autotuner choice for small batches) gives the
    oracle's pivots and factors, as the 64 x 64 tile does; other tile codes are argument errors."""
    import paper_1812_01396_amd as ss
    print(f"lu_factor tile=1 n={n}", flush=True)
    rng = np.random.default_rng(7000 + n)
    a = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    ctx.set_lu_tile(1)
    try:
        lu, perm, info = ss.ss_lu_factor(ctx, _dev(a))
        torch.cuda.synchronize()
    finally:
        ctx.set_lu_tile(0)
    lu, perm, info = lu.cpu().numpy(), perm.cpu().numpy(), info.cpu().numpy()
    for b in range(2):
        ref, rperm, rinfo = linalg.lu_partial_pivot(a[b])
        assert info[b] == rinfo == 0
        assert np.array_equal(perm[b], rperm), (b, int(np.argmax(perm[b] != rperm)))
        assert np.abs(lu[b] - ref).max() <= 1e-11 * np.abs(ref).max(), (b, np.abs(lu[b] - ref).max())
    for bad in (-1, 2):
        with pytest.raises(ss.splitsolve.SplitSolveError):
            ctx.set_lu_tile(bad)


def test_lu_width_rejects_other_values(ctx):
    import paper_1812_01396_amd as ss
    for bad in (-1, 4, 24, 64):
        with pytest.raises(ss.splitsolve.SplitSolveError):
            ctx.set_lu_width(bad)


def test_lu_factor_zero_pivots(ctx):
    import paper_1812_01396_amd as ss
    rng = np.random.default_rng(9)
    a = rng.standard_normal((2, 40, 40)) + 1j * rng.standard_normal((2, 40, 40))
    a[0, :, 17] = 0.0  # column 17 is exactly zero after any elimination
    a[1, :, 39] = 0.0
    lu, perm, info = ss.ss_lu_factor(ctx, _dev(a))
    torch.cuda.synchronize()
    for b in range(2):
        ref, rperm, rinfo = linalg.lu_partial_pivot(a[b])
        assert info.cpu().numpy()[b] == rinfo
        assert np.array_equal(perm.cpu().numpy()[b], rperm)
        assert np.abs(lu.cpu().numpy()[b] - ref).max() <= 1e-11 * np.abs(ref).max()
    assert list(info.cpu().numpy()) == [18, 40]


@pytest.mark.parametrize("batch,nb,s,m,keep,prec", [(3, 4, 40, 3, False, 0), (2, 3, 130, 5, True, 0),
                                                    (1, 1, 16, 0, False, 0), (2, 3, 130, 5, True, 3)])
def test_workspace_size_matches_a_fresh_context(batch, nb, s, m, keep, prec):
    """ss_workspace_size equals what a fresh context holds after one pass of the four steps (with the
    BF16-term products: also their FP32 coupling blocks)."""
    import paper_1812_01396_amd as ss
    c = ss.Context(0)
    try:
        insts = [synth.random_btd(nb, s, seed=3300 + k) for k in range(batch)]
        hd, hu, sd, su = (_dev(np.stack([getattr(i, f) for i in insts])) for f in ("Hd", "Hu", "Sd", "Su"))
        leads = [_dev(np.stack([getattr(i, f) for i in insts])) for f in ("H00", "H01", "S00", "S01")]
        E = _dev(np.linspace(-0.4, 0.4, batch), torch.float64)
        kidx = torch.arange(batch, dtype=torch.int32, device="cuda")
        sig, _, _, _ = ss.ss_lead_selfenergy(c, *leads, E, 1e-8, kidx=kidx)
        q, _ = ss.ss_precompute_columns(c, hd, hu, sd, su, E, kidx=kidx, keep_factors=keep, absorb=1.0, prec=prec)
        inj = _dev(np.stack([synth.injection_block(s, m, 5 + b) for b in range(batch)])) if m else None
        _, gc, _ = ss.ss_apply_obc(c, q, sig, inj=inj, absorb=1.0)
        ss.ss_transmission(c, gc, sig)
        torch.cuda.synchronize()
        flags = ss.splitsolve.SS_KEEP_FACTORS if keep else 0
        assert c.workspace_bytes() == ss.ss_workspace_size(batch, nb, s, m, prec=prec, flags=flags)
    finally:
        c.close()
