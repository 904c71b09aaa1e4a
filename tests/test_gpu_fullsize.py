"""Full-size parity in the benchmark's own launch configuration (bench.Pipeline).

dft512: s = 512, nb = 40, 64 energies x 4 momenta (256 instances), Q in chunks of 64 with the
self-energies on a second stream.  The oracle needs seconds per instance here, so it checks sampled
instances element by element; properties that hold at any size are checked on all 256 instances:
the device is a perfect crystal, so T is an integer (the open-channel count) and T_LR = T_RL.
chain16: s = 16, nb = 32, all 64 energies against the stored channel counts.
"""
import os

import numpy as np
import pytest
import torch

from oracle import selfenergy, transport

pytestmark = pytest.mark.gpu

UNIT = 2.0 ** -52


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def dft512():
    import bench
    print("dft512 pipeline: building inputs and running one step", flush=True)
    pipe = bench.Pipeline("dft512")
    pipe.run()
    torch.cuda.synchronize()
    yield pipe
    pipe.ctx.close()
    pipe.ctx_s.close()


def test_dft512_all_instances(dft512):
    p = dft512
    for info in (p.info_s, p.info_q, p.info_o):
        assert int((info != 0).sum()) == 0
    T = p.T.cpu().numpy()
    assert np.isfinite(T).all()
    # T_LR = T_RL and integer channel counts (crystal).  The FP64 SMW route carries the closed
    # device's conditioning kappa(E S - H) into G (it cancels only in exact arithmetic): at energies
    # next to an eigenvalue of the closed device the plain path is good to ~1e-7, which bounds these
    # two checks; the sampled oracle comparisons below hold T to 1e-8.
    assert np.abs(T[:, 0] - T[:, 1]).max() <= 1e-6
    assert np.abs(T - np.round(T)).max() <= 1e-6
    assert T.min() >= -1e-8 and T.max() <= p.w["s"]
    assert len(set(np.round(T[:, 0]).astype(int))) >= 3     # the grid spans several channel counts


@pytest.mark.parametrize("b", [37, 200])
def test_dft512_sampled_vs_oracle(dft512, b):
    p = dft512
    w = p.w
    print(f"dft512 oracle for instance {b}", flush=True)
    inst = p.insts[p.kidx_np[b]]
    E = float(p.E_np[b])
    ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00, inst.S01,
                                   E, w["eta"], inj=p.inj_np[b], want_q=(b >= p.n - p.chunk))
    a0, a1, am1 = selfenergy.lead_blocks(inst.H00, inst.H01, inst.S00, inst.S01, E, w["eta"])
    tol = max(1e-10, 10 * UNIT * selfenergy.decimation_conditioning(a0, a1, am1))
    sig = p.sigma[b].cpu().numpy()
    assert _rel(sig[0], ref["sigma_l"]) <= tol
    assert _rel(sig[1], ref["sigma_r"]) <= tol
    assert _rel(p.gc[b].cpu().numpy(), ref["gc"]) <= tol
    assert _rel(p.psi[b].cpu().numpy(), ref["psi"]) <= tol
    T = p.T[b].cpu().numpy()
    assert abs(T[0] - ref["t_lr"]) <= 1e-8 * max(1.0, ref["t_lr"])
    assert abs(T[1] - ref["t_rl"]) <= 1e-8 * max(1.0, ref["t_rl"])
    if ref["q"] is not None:  # Q of the last chunk is still in the chunk buffer
        q = p.Qbuf[b - (p.n - p.chunk)].cpu().numpy()
        # tolerance: max(1e-10, 10 x the spread of two exact-in-exact-arithmetic oracle routes)
        ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
        spread = _rel(transport.first_last_columns_mirrored(ad, au, al), ref["q"])
        assert _rel(q, ref["q"]) <= max(1e-10, 10 * spread)


def test_chain16_pipeline_matches_channel_counts():
    import bench
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "chain16_channels.txt"), comments="#")
    pipe = bench.Pipeline("chain16")
    pipe.run()
    torch.cuda.synchronize()
    assert np.allclose(pipe.E_np, rows[:, 0])
    T = pipe.T.cpu().numpy()
    assert np.abs(T[:, 0] - rows[:, 1]).max() <= 1e-8
    assert np.abs(T[:, 1] - rows[:, 1]).max() <= 1e-8
    pipe.ctx.close()
    pipe.ctx_s.close()
