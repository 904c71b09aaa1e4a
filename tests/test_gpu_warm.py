"""Learned warm start on the GPU against the oracle.

* The perceptron's forward pass, loss, gradients and Adam step (FP32 matrix-core kernels) against the
  float64 oracle with the same parameters; split-K products included.
* Features and the standardised encoding of Sigma.
* The warm-started self-energy: a start that already solves the fixed-point equation is accepted as is;
  a non-retarded root (an exact fixed point) and poor starts are rejected and replaced by the decimation,
  whose result matches the oracle.
* Training on self-energies of the decimation lowers the loss, and the trained network's prediction on
  held-out (E, k) is closer to the decimation than the best prediction without it (the training mean);
  the warm-started results equal the oracle's decimation on a sample of those points.
* At the learned workload's own lead size (s = 256) and network size: cold and warm self-energies
  against the oracle, and the network's forward pass and gradients against the float64 oracle.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import selfenergy, warmstart

pytestmark = pytest.mark.gpu

ETA = 1e-8
UNIT = 2.0 ** -52


@pytest.fixture(scope="module")
def ctx():
    import paper_1812_01396_amd as ss
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = ss.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _unpack(flat, dims):
    out, o = [], 0
    for i in range(len(dims) - 1):
        W = flat[o:o + dims[i] * dims[i + 1]].reshape(dims[i], dims[i + 1])
        o += dims[i] * dims[i + 1]
        b = flat[o:o + dims[i + 1]]
        o += dims[i + 1]
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


@pytest.mark.parametrize("dims,n", [([35, 64, 48, 64, 100], 70), ([3000, 8, 5], 16), ([35, 8, 4], 5000)])
def test_mlp_forward_and_gradients_match_oracle(ctx, dims, n):
    import paper_1812_01396_amd as ss
    print(f"mlp dims={dims} n={n}", flush=True)
    net = ss.MLP(ctx, dims, seed=3)
    with torch.no_grad():  # non-zero biases so the bias path is exercised
        net.params.add_(0.05 * torch.randn(net.count, device="cuda"))
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, dims[0])).astype(np.float32)
    T = rng.standard_normal((n, dims[-1])).astype(np.float32)
    Xd, Td = torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()
    acts, Y = net.forward(Xd)
    loss = net.backward(Xd, acts, Td)
    torch.cuda.synchronize()
    params = _unpack(net.params.cpu().numpy(), dims)
    ref_acts = warmstart.mlp_forward(params, X.astype(np.float64))
    assert _rel(Y.cpu().numpy(), ref_acts[-1]) <= 1e-5
    ref_loss, ref_grads = warmstart.mlp_loss_grad(params, X.astype(np.float64), T.astype(np.float64))
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * ref_loss
    got = _unpack(net.grads.cpu().numpy(), dims)
    for (gW, gb), (rW, rb) in zip(got, ref_grads):
        assert _rel(gW, rW) <= 1e-4 and _rel(gb, rb) <= 1e-4


def test_adam_matches_oracle(ctx):
    import paper_1812_01396_amd as ss
    dims = [35, 32, 16]
    net = ss.MLP(ctx, dims, seed=1)
    rng = np.random.default_rng(5)
    X = torch.as_tensor(rng.standard_normal((40, 35)).astype(np.float32)).cuda()
    T = torch.as_tensor(rng.standard_normal((40, 16)).astype(np.float32)).cuda()
    params = _unpack(net.params.cpu().numpy(), dims)
    state = {}
    for _ in range(3):
        acts, _ = net.forward(X)
        net.backward(X, acts, T)
        grads = _unpack(net.grads.cpu().numpy(), dims)
        net.adam(1e-2)
        params = warmstart.adam_step(params, grads, state, 1e-2)
    torch.cuda.synchronize()
    for (gW, gb), (rW, rb) in zip(_unpack(net.params.cpu().numpy(), dims), params):
        assert np.abs(gW - rW).max() <= 1e-5 and np.abs(gb - rb).max() <= 1e-5


def test_features_and_sigma_encoding(ctx):
    import paper_1812_01396_amd as ss
    rng = np.random.default_rng(6)
    E = rng.uniform(-5, 5, 37)
    k = rng.uniform(0, np.pi, 37)
    X = ss.ss_warm_features(ctx, torch.as_tensor(E).cuda(), torch.as_tensor(k).cuda())
    assert np.abs(X.cpu().numpy() - warmstart.features(E, k)).max() <= 1e-6
    s = 5
    sig = rng.standard_normal((9, 2, s, s)) + 1j * rng.standard_normal((9, 2, s, s))
    sd = torch.as_tensor(sig).cuda()
    mean, std = ss.ss_sigma_moments(ctx, sd)
    enc = np.stack([warmstart.encode_sigma(x[0], x[1]) for x in sig])
    assert np.abs(mean.cpu().numpy() - enc.mean(0)).max() <= 1e-6
    assert np.abs(std.cpu().numpy() - enc.std(0)).max() <= 1e-5
    y = ss.ss_sigma_encode(ctx, sd, mean, std)
    back = ss.ss_sigma_decode(ctx, y, mean, std, s)
    torch.cuda.synchronize()
    assert _rel(back.cpu().numpy(), sig) <= 1e-6


def _lead_tensors(cells):
    return [torch.as_tensor(np.stack([c[i] for c in cells])).cuda() for i in range(4)]


def test_warm_selfenergy_judge_and_fallback(ctx):
    """Exact start accepted unchanged; a non-retarded exact fixed point and poor starts rejected and
    replaced by the decimation."""
    import scipy.linalg as sla
    import paper_1812_01396_amd as ss
    cell = synth.DFTLikeCell(synth.SLAB_SHAPES[24], 4).at(0.7)
    s = 24
    Es = np.array([0.3, -1.0, 2.0, 0.3, 0.3, -1.0])
    refs, inits = [], []
    for b, E in enumerate(Es):
        a0, a1, am1 = selfenergy.lead_blocks(*cell, E, ETA)
        sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
        refs.append((sl, sr, max(1e-10, 10 * UNIT * selfenergy.decimation_conditioning(a0, a1, am1))))
        if b < 3:
            inits.append(np.stack([sl, sr]))  # exact retarded roots
        elif b == 3:  # a non-retarded exact root: one growing mode in place of a decaying one
            eye, zero = np.eye(s), np.zeros((s, s))
            lam, vec = sla.eig(np.block([[zero, eye], [-am1, -a0]]), np.block([[eye, zero], [zero, a1]]))
            order = np.argsort(np.abs(lam))
            keep = np.concatenate([order[: s - 1], order[s: s + 1]])
            u = vec[:s, keep]
            inits.append(np.stack([sl, -a1 @ (u @ np.diag(lam[keep]) @ np.linalg.inv(u))]))
        elif b == 4:
            inits.append(np.zeros((2, s, s)))
        else:  # the self-energy at a 1000x larger broadening
            b0, b1, bm1 = selfenergy.lead_blocks(*cell, E, 1e-5)
            l0, r0, _, _ = selfenergy.decimation(b0, b1, bm1)
            inits.append(np.stack([l0, r0]))
    lead = _lead_tensors([cell])
    init = torch.as_tensor(np.stack(inits)).cuda()
    sig, it_n, it_d, resid, info = ss.ss_lead_selfenergy_warm(ctx, *lead, torch.as_tensor(Es).cuda(), ETA, init,
                                                              kidx=torch.zeros(len(Es), dtype=torch.int32).cuda())
    torch.cuda.synchronize()
    sig, info, it_n, it_d = sig.cpu().numpy(), info.cpu().numpy(), it_n.cpu().numpy(), it_d.cpu().numpy()
    print("info", info, "newton", it_n, "decimation", it_d, flush=True)
    assert list(info[:3]) == [0, 0, 0] and list(it_n[:3]) == [0, 0, 0]
    assert info[3] == -2 and it_d[3] > 0  # the judge rejects the non-retarded root
    assert all(i in (0, -2) for i in info[4:])
    for b, (sl, sr, tol) in enumerate(refs):
        assert _rel(sig[b, 0], sl) <= tol and _rel(sig[b, 1], sr) <= tol, (b, _rel(sig[b, 0], sl), tol)


def test_training_gains_over_the_mean_prediction(ctx):
    import paper_1812_01396_amd as ss
    shape = synth.SLAB_SHAPES[24]
    s = 24
    base = synth.DFTLikeCell(shape, 4)
    rng = np.random.default_rng(7)
    n_train, n_test = 640, 64
    E = rng.uniform(-5, 5, n_train + n_test)
    k = rng.uniform(0, np.pi, n_train + n_test)
    cells = [base.at(kk) for kk in k]
    lead = _lead_tensors(cells)
    Ed, kd = torch.as_tensor(E).cuda(), torch.as_tensor(k).cuda()
    kidx = torch.arange(len(E), dtype=torch.int32).cuda()
    sigma, _, _, info = ss.ss_lead_selfenergy(ctx, *lead, Ed, ETA, kidx=kidx)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    X = ss.ss_warm_features(ctx, Ed, kd)
    mean, std = ss.ss_sigma_moments(ctx, sigma[:n_train].contiguous(), std_floor=1e-6)
    Y = ss.ss_sigma_encode(ctx, sigma, mean, std)
    dims = [X.shape[1], 128, 128, 128, 4 * s * s]
    net = ss.MLP(ctx, dims, seed=0)
    g = torch.Generator(device="cpu").manual_seed(0)
    losses = []
    for step in range(1500):
        idx = torch.randint(0, n_train, (128,), generator=g).cuda()
        xb, yb = X[idx].contiguous(), Y[idx].contiguous()
        acts, _ = net.forward(xb)
        losses.append(float(net.backward(xb, acts, yb).item()))
        net.adam(2e-3)
    print("loss", losses[0], losses[-1], flush=True)
    assert np.mean(losses[-50:]) < 0.5 * np.mean(losses[:20])
    _, pred = net.forward(X[n_train:].contiguous())
    sig_pred = ss.ss_sigma_decode(ctx, pred.contiguous(), mean, std, s).cpu().numpy()
    ref = sigma[n_train:].cpu().numpy()
    mean_sig = ss.ss_sigma_decode(ctx, torch.zeros(1, 4 * s * s, device="cuda"), mean, std, s).cpu().numpy()[0]
    err_net = np.median([_rel(sig_pred[i], ref[i]) for i in range(n_test)])
    err_mean = np.median([_rel(mean_sig, ref[i]) for i in range(n_test)])
    print("median relative error: network", err_net, "training mean", err_mean, flush=True)
    assert err_net < 0.8 * err_mean
    # the warm-started solve from the prediction returns the decimation's self-energies either way
    out, it_n, it_d, _, info = ss.ss_lead_selfenergy_warm(ctx, *lead, Ed[n_train:].contiguous(), ETA,
                                                          torch.as_tensor(sig_pred).cuda(),
                                                          kidx=kidx[n_train:].contiguous())
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    assert max(_rel(out[i], ref[i]) for i in range(n_test)) <= 1e-8
    print("accepted", int((info == 0).sum()), "of", n_test, flush=True)
    # and the self-energies returned are the oracle's (decimation on the CPU) on a sample of the held-out points
    for i in range(0, n_test, 16):
        j = n_train + i
        a0, a1, am1 = selfenergy.lead_blocks(*cells[j], E[j], ETA)
        sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
        tol = max(1e-10, 10 * UNIT * selfenergy.decimation_conditioning(a0, a1, am1))
        assert _rel(out[i, 0], sl) <= tol and _rel(out[i, 1], sr) <= tol, (i, _rel(out[i, 0], sl), tol)


def test_warm_start_at_the_learned_workload_size(ctx):
    """The learned workload's lead (s = 256, the 4 x 8 x 8 slab of seed 4): cold decimation and the warm
    start against the oracle's decimation; a start at the oracle's roots is accepted with no Newton step,
    a start 1e-3 off is judged and either accepted or replaced, and the result is the oracle's either way.
    The perceptron of that workload (35 -> 512 -> 512 -> 512 -> 4 s^2 = 262144 outputs, FP32) against the
    float64 oracle on a few rows: outputs, loss and the gradients of every layer."""
    import paper_1812_01396_amd as ss
    s = 256
    base = synth.DFTLikeCell(synth.SLAB_SHAPES[s], 4)
    pts = [(-2.5, 0.4), (0.7, 1.9), (3.1, 2.8)]
    cells = [base.at(k) for _, k in pts]
    Es = np.array([e for e, _ in pts])
    refs = []
    for (E, _), cell in zip(pts, cells):
        a0, a1, am1 = selfenergy.lead_blocks(*cell, E, ETA)
        sl, sr, _, _ = selfenergy.decimation(a0, a1, am1)
        refs.append((sl, sr, max(1e-10, 10 * UNIT * selfenergy.decimation_conditioning(a0, a1, am1))))
    lead = _lead_tensors(cells)
    Ed = torch.as_tensor(Es).cuda()
    kidx = torch.arange(len(pts), dtype=torch.int32).cuda()
    cold, _, _, info_c = ss.ss_lead_selfenergy(ctx, *lead, Ed, ETA, kidx=kidx)
    exact = torch.as_tensor(np.stack([np.stack([sl, sr]) for sl, sr, _ in refs])).cuda()
    rng = np.random.default_rng(8)
    pert = exact.cpu().numpy() * (1 + 1e-3 * (rng.standard_normal(exact.shape) + 1j * rng.standard_normal(exact.shape)))
    warm_x, itn_x, _, _, info_x = ss.ss_lead_selfenergy_warm(ctx, *lead, Ed, ETA, exact, kidx=kidx)
    warm_p, _, _, _, info_p = ss.ss_lead_selfenergy_warm(ctx, *lead, Ed, ETA, torch.as_tensor(pert).cuda(),
                                                        kidx=kidx)
    torch.cuda.synchronize()
    assert int((info_c != 0).sum()) == 0
    assert info_x.cpu().tolist() == [0, 0, 0] and itn_x.cpu().tolist() == [0, 0, 0]
    assert all(i in (0, -2) for i in info_p.cpu().tolist())
    for out in (cold, warm_x, warm_p):
        o = out.cpu().numpy()
        for b, (sl, sr, tol) in enumerate(refs):
            assert _rel(o[b, 0], sl) <= tol and _rel(o[b, 1], sr) <= tol, (b, _rel(o[b, 0], sl), tol)
    # the network of that workload, on 6 rows
    dims = [35, 512, 512, 512, 4 * s * s]
    net = ss.MLP(ctx, dims, seed=2)
    X = ss.ss_warm_features(ctx, torch.as_tensor(rng.uniform(-5, 5, 6)).cuda(),
                            torch.as_tensor(rng.uniform(0, np.pi, 6)).cuda())
    T = torch.as_tensor(rng.standard_normal((6, dims[-1])).astype(np.float32)).cuda()
    acts, Y = net.forward(X)
    loss = net.backward(X, acts, T)
    torch.cuda.synchronize()
    params = _unpack(net.params.cpu().numpy(), dims)
    Xh = X.cpu().numpy().astype(np.float64)
    ref_acts = warmstart.mlp_forward(params, Xh)
    assert _rel(Y.cpu().numpy(), ref_acts[-1]) <= 1e-5
    ref_loss, ref_grads = warmstart.mlp_loss_grad(params, Xh, T.cpu().numpy().astype(np.float64))
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * ref_loss
    for (gW, gb), (rW, rb) in zip(_unpack(net.grads.cpu().numpy(), dims), ref_grads):
        assert _rel(gW, rW) <= 1e-4 and _rel(gb, rb) <= 1e-4
