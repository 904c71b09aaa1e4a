"""ss_transmission_noalloc (the transmission for callers that cannot allocate) against ss_transmission.

Both run the same two kernels in the same order on the same inputs; only where the per-tile partial
sums live differs (the library's fixed per-device scratch instead of the context's workspace), so the
two results must agree exactly, which is stricter than the FP64 parity bar of 1e-10.  Two calls in a
row, the second with a smaller batch and block size, check that the scratch left by the first call
does not leak into the second.  The inputs are the corner of G^R and the self-energies of real solves
(random disordered devices), at a ragged block size (s = 300: tiles of 32 with a tail of 12).
"""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _corner_and_sigma(ctx, nb, s, Es, seed):
    import paper_1812_01396_amd as ss
    inst = synth.random_btd(nb, s, seed=seed)
    E = _dev(Es, torch.float64)
    sig, _, _, info_s = ss.ss_lead_selfenergy(ctx, _dev(inst.H00), _dev(inst.H01), _dev(inst.S00), _dev(inst.S01),
                                              E, 1e-8)
    q, info_q = ss.ss_precompute_columns(ctx, _dev(inst.Hd), _dev(inst.Hu), _dev(inst.Sd), _dev(inst.Su), E,
                                         absorb=1.0)
    _, gc, info_o = ss.ss_apply_obc(ctx, q, sig, absorb=1.0)
    torch.cuda.synchronize()
    assert int(info_s.abs().sum()) == 0 and int(info_q.abs().sum()) == 0 and int(info_o.abs().sum()) == 0
    return gc, sig


def test_noalloc_transmission_matches_allocating_call():
    import paper_1812_01396_amd as ss
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = ss.Context(0)
    ctx_na = ss.Context(0)  # used only for the allocation-free calls
    try:
        cases = [(2, 300, np.array([-0.4, 0.05, 0.3, 0.8, -1.1])), (3, 40, np.array([0.2, -0.6]))]
        for call, (nb, s, Es) in enumerate(cases):
            print(f"noalloc call {call}: batch={len(Es)} nb={nb} s={s}", flush=True)
            gc, sig = _corner_and_sigma(ctx, nb, s, Es, seed=4100 + call)
            T_ref = ss.ss_transmission(ctx, gc, sig)
            T_na = torch.full((len(Es), 2), float("nan"), dtype=torch.float64, device="cuda")
            ss.ss_transmission_noalloc(ctx_na, gc, sig, T_na)
            torch.cuda.synchronize()
            a, b = T_na.cpu().numpy(), T_ref.cpu().numpy()
            assert np.all(np.isfinite(a)), a
            assert np.array_equal(a, b), (call, a, b, np.abs(a - b).max())
            assert ctx_na.workspace_bytes() == 0, "the allocation-free call grew a workspace"
    finally:
        ctx_na.close()
        ctx.close()


def test_noalloc_transmission_rejects_batches_beyond_its_scratch():
    import paper_1812_01396_amd as ss
    from paper_1812_01396_amd import splitsolve
    ctx = ss.Context(0)
    try:
        dummy = torch.zeros(4, dtype=torch.float64, device="cuda")
        p = ctypes.c_void_p(dummy.data_ptr())
        # s = 1024: 32 x 32 tiles per direction, 2048 partial sums per instance; 513 instances need
        # 1050624 > 2^20 doubles.  The size check comes before any launch, so nothing reads `dummy`.
        st = ctx.lib.ss_transmission_noalloc(ctx.handle, 513, 1024, p, p, p)
        assert st == splitsolve.SS_ERR_ARG
        assert b"scratch" in ctx.lib.ss_last_error(ctx.handle)
        assert ctx.workspace_bytes() == 0
    finally:
        ctx.close()
