"""Mixed precision and iterative refinement on the GPU against the oracle.

* ss_injection_left: W_L W_L^H reproduces Gamma_L of the oracle's self-energy.
* FP32 recursion products (SS_PREC_FP32) give a psi that is only ~1e-6 accurate; FP64 refinement on
  the full open system (ss_refine_psi) brings it to <= 1e-10 of the oracle's direct solve.
* T from the refined psi (ss_transmission_psi) matches the oracle's Caroli T to 1e-8, including a
  perfect crystal at an energy next to an eigenvalue of the closed device, where the plain SMW route
  loses digits to the closed device's conditioning, and an injection truncated to the open channels
  with the rest of Gamma_L added back through the corner of G^R.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import selfenergy, transport

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    import paper_1812_01396_amd as ss
    c = ss.Context(0)
    yield c
    c.close()


def _run(ctx, insts, Es, kidx, eta, prec, inj=None, mmax=16, refine=True, absorb=0.0, inj_tol=0.0):
    import paper_1812_01396_amd as ss
    hd, hu, sd, su = (_dev(np.stack([getattr(i, f) for i in insts])) for f in ("Hd", "Hu", "Sd", "Su"))
    leads = [_dev(np.stack([getattr(i, f) for i in insts])) for f in ("H00", "H01", "S00", "S01")]
    E_d, k_d = _dev(Es, torch.float64), _dev(kidx, torch.int32)
    sig, _, _, info_s = ss.ss_lead_selfenergy(ctx, *leads, E_d, eta, kidx=k_d)
    q, info_q = ss.ss_precompute_columns(ctx, hd, hu, sd, su, E_d, kidx=k_d, prec=prec, keep_factors=True,
                                         absorb=absorb)
    if inj is None:
        inj_d, rank = ss.ss_injection_left(ctx, sig, mmax, tol=inj_tol)
    else:
        inj_d, rank = _dev(inj), None
    psi, gc, info_o = ss.ss_apply_obc(ctx, q, sig, inj=inj_d, absorb=absorb)
    psi0 = psi.clone()
    out = dict(sig=sig, q=q, gc=gc, psi0=psi0, inj=inj_d, rank=rank)
    if refine:
        psi, iters, resid = ss.ss_refine_psi(ctx, hd, hu, sd, su, E_d, q, sig, inj_d, psi, kidx=k_d, tol=1e-13,
                                             max_iter=12)
        out.update(iters=iters, resid=resid)
    out["psi"] = psi
    out["T_psi"] = ss.ss_transmission_psi(ctx, psi, sig)
    out["T_tail"] = ss.ss_transmission_psi(ctx, psi, sig, psi0=psi0[:, -1].contiguous(), gc=gc)
    torch.cuda.synchronize()
    for i in (info_s, info_q, info_o):
        assert int((i != 0).sum()) == 0
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in out.items()}


def test_injection_factor_reproduces_gamma(ctx):
    inst = synth.random_btd(3, 24, seed=404)
    Es = np.array([-0.3, 0.4])
    out = _run(ctx, [inst], Es, np.zeros(2, np.int32), 1e-8, 0, refine=False, mmax=24)
    for b, E in enumerate(Es):
        a0, a1, am1 = selfenergy.lead_blocks(inst.H00, inst.H01, inst.S00, inst.S01, E, 1e-8)
        sl, _, _, _ = selfenergy.decimation(a0, a1, am1)
        gam = selfenergy.broadening(sl)
        w = out["inj"][b][:24]
        assert np.abs(out["inj"][b][24:]).max() == 0.0
        assert _rel(w @ w.conj().T, gam) <= 1e-9
        assert 1 <= out["rank"][b] <= 24


@pytest.mark.parametrize("prec,absorb", [(0, 0.0), (1, 0.0), (0, 1.0), (1, 1.0), (2, 1.0), (3, 0.0), (3, 1.0)])
def test_refined_psi_matches_oracle(ctx, prec, absorb):
    """Refinement of psi on the open system from the kept factors, for the paper's split and for the
    absorbing one (the factors of A' and C' = Sigma + i*absorb*I)."""
    nb, s, m = 4, 40, 3
    insts = [synth.random_btd(nb, s, seed=700 + k) for k in range(2)]
    Es = np.array([0.21, -0.33])
    kidx = np.array([0, 1], np.int32)
    eta = 1e-8
    inj = np.stack([synth.injection_block(s, m, 90 + b) for b in range(2)])
    out = _run(ctx, insts, Es, kidx, eta, prec, inj=inj, absorb=absorb)
    for b in range(2):
        inst = insts[kidx[b]]
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                       inst.S01, Es[b], eta, inj=inj[b])
        a0, a1, am1 = selfenergy.lead_blocks(inst.H00, inst.H01, inst.S00, inst.S01, Es[b], eta)
        tol = max(1e-10, 10 * 2.0 ** -52 * selfenergy.decimation_conditioning(a0, a1, am1))
        e0 = _rel(out["psi0"][b], ref["psi"])
        e1 = _rel(out["psi"][b], ref["psi"])
        if prec >= 1:
            assert e0 > 1e-9          # FP32 products: the unrefined psi is visibly less accurate
        assert e1 <= tol, (b, e0, e1, tol)
        assert out["resid"][b] <= 1e-12


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_transmission_from_refined_psi(ctx, prec):
    inst = synth.random_btd(5, 32, seed=808)
    Es = np.array([-0.5, 0.1, 0.6])
    eta = 1e-8
    out = _run(ctx, [inst], Es, np.zeros(3, np.int32), eta, prec, mmax=32)
    for b, E in enumerate(Es):
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                       inst.S01, E, eta, want_q=False)
        assert abs(out["T_psi"][b] - ref["t_rl"]) <= 1e-8 * max(1.0, ref["t_rl"]), (E, out["T_psi"][b], ref)


@pytest.mark.parametrize("prec,absorb", [(0, 1.0), (1, 1.0), (1, 0.0), (2, 1.0), (3, 1.0)])
def test_transmission_tail_of_truncated_injection(ctx, prec, absorb):
    """Injection truncated to the open channels (pivoted Cholesky stopped at 1e-5 of the largest pivot):
    T from psi alone misses the broadening tail of Gamma_L (~1e-6 here), and with the tail added back
    through the corner of G^R it matches the oracle's Caroli T_RL (1e-10 in FP64, 1e-8 with FP32
    products, whose corner is ~1e-6 accurate but only weighs the small tail)."""
    inst = synth.random_btd(5, 40, seed=909)
    Es = np.array([-0.5, 0.1, 0.6])
    eta = 1e-8
    out = _run(ctx, [inst], Es, np.zeros(3, np.int32), eta, prec, mmax=12, absorb=absorb, inj_tol=1e-5)
    for b, E in enumerate(Es):
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                       inst.S01, E, eta, want_q=False)
        assert 1 <= out["rank"][b] < 12
        assert abs(out["T_psi"][b] - ref["t_rl"]) > 1e-7        # the tail is visible without the correction
        tol = 1e-10 if prec == 0 else 1e-8
        assert abs(out["T_tail"][b] - ref["t_rl"]) <= tol * max(1.0, ref["t_rl"]), (E, out["T_tail"][b], ref["t_rl"])


@pytest.mark.parametrize("s", [40, 96])
def test_bf16_term_products_reach_fp32_accuracy(ctx, s):
    """Q from the BF16-term products (three BF16 terms per operand, six term products, FP32 accumulation)
    is as accurate as Q from FP32 products, against the FP64 Q of the same inputs: a dropped term or a
    wrong sign of the imaginary parts would leave errors of order 2^-8 or worse; one BF16 term alone
    would leave about 1e-3.  s = 40 and 96 exercise partial 64-wide tiles and partial 32-deep stages."""
    import paper_1812_01396_amd as ss
    nb = 4
    insts = [synth.random_btd(nb, s, seed=1200 + s + k) for k in range(2)]
    Es = np.array([0.17, -0.41])
    kidx = np.array([0, 1], np.int32)
    hd, hu, sd, su = (_dev(np.stack([getattr(i, f) for i in insts])) for f in ("Hd", "Hu", "Sd", "Su"))
    E_d, k_d = _dev(Es, torch.float64), _dev(kidx, torch.int32)
    qs = {}
    for prec in (0, 1, 3):
        q, info = ss.ss_precompute_columns(ctx, hd, hu, sd, su, E_d, kidx=k_d, prec=prec, absorb=1.0)
        torch.cuda.synchronize()
        assert int((info != 0).sum()) == 0
        qs[prec] = q.cpu().numpy()
    for b in range(2):
        e32, ebf = _rel(qs[1][b], qs[0][b]), _rel(qs[3][b], qs[0][b])
        print(f"s={s} b={b}: FP32 products {e32:.2e}, BF16 terms {ebf:.2e}", flush=True)
        assert 0 < ebf <= 4 * e32 + 1e-7, (b, e32, ebf)
        assert ebf <= 1e-5


def test_crystal_near_closed_device_eigenvalue(ctx):
    """Chain crystal, energies across the band: the refined T(psi) is the integer channel count to 1e-8."""
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "chain16_channels.txt"), comments="#")
    cell = synth.chain_cell(16, 0)
    inst = synth.device_from_cell(cell, 32)
    Es = rows[:, 0]
    out = _run(ctx, [inst], Es, np.zeros(len(Es), np.int32), 1e-8, 1, mmax=16)
    assert np.abs(out["T_psi"] - rows[:, 1]).max() <= 1e-8


def test_refinement_without_kept_inverses(ctx):
    """With 16-column panels the recursion keeps no inverses of 32 x 32 diagonal blocks, and the refinement's
    block solves substitute through the triangles instead: both refined psi against the oracle at 1e-10 and
    against each other at the same bar."""
    nb, s, m = 4, 72, 3
    insts = [synth.random_btd(nb, s, seed=1500 + k) for k in range(2)]
    Es = np.array([0.19, -0.27])
    kidx = np.array([0, 1], np.int32)
    inj = np.stack([synth.injection_block(s, m, 70 + b) for b in range(2)])
    with_inv = _run(ctx, insts, Es, kidx, 1e-8, 3, inj=inj, absorb=1.0)
    ctx.set_lu_width(16)
    try:
        without = _run(ctx, insts, Es, kidx, 1e-8, 3, inj=inj, absorb=1.0)
    finally:
        ctx.set_lu_width(0)
    for b in range(2):
        inst = insts[kidx[b]]
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                       inst.S01, Es[b], 1e-8, inj=inj[b])
        for out in (with_inv, without):
            assert _rel(out["psi"][b], ref["psi"]) <= 1e-10, (b, _rel(out["psi"][b], ref["psi"]))
            assert out["resid"][b] <= 1e-12
        # different panel widths round differently: the two agree to the conditioning-limited accuracy
        # that each has against the oracle
        assert _rel(with_inv["psi"][b], without["psi"][b]) <= 1e-10


def test_refine_rejects_mismatched_absorbing_shift(ctx):
    """Kept factors of A' (absorb = 1) and a corner system formed with C' for absorb = 0 do not describe one
    split: the refinement refuses them (host-side argument check, nothing is launched)."""
    import paper_1812_01396_amd as ss
    inst = synth.random_btd(3, 8, seed=31)
    hd, hu, sd, su = (_dev(getattr(inst, f)[None]) for f in ("Hd", "Hu", "Sd", "Su"))
    leads = [_dev(getattr(inst, f)[None]) for f in ("H00", "H01", "S00", "S01")]
    E_d = _dev(np.array([0.2]), torch.float64)
    sig, _, _, _ = ss.ss_lead_selfenergy(ctx, *leads, E_d, 1e-8)
    q, _ = ss.ss_precompute_columns(ctx, hd, hu, sd, su, E_d, keep_factors=True, absorb=1.0)
    inj = _dev(synth.injection_block(8, 2, 3)[None])
    psi, _, _ = ss.ss_apply_obc(ctx, q, sig, inj=inj, absorb=0.0)
    with pytest.raises(ss.splitsolve.SplitSolveError):
        ss.ss_refine_psi(ctx, hd, hu, sd, su, E_d, q, sig, inj, psi)
    torch.cuda.synchronize()
