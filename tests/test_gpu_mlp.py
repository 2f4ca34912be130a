"""GPU checks of the learned demapper against the FP64 oracle network.

Tolerances: every product runs in BF16 (8-bit mantissa, unit roundoff 2^-9) with
FP32 accumulation, so a layer's outputs carry a relative error of a few 2^-9 and the
three-layer network about 1e-2 in relative norm; gradients likewise.  Checks:
  forward:   relative Frobenius error <= 2e-2, cosine >= 0.999
  gradients: per parameter group relative error <= 3e-2, cosine >= 0.999
  Adam:      FP32 update vs FP64 update of the same gradient, relative 1e-5
"""
import math
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def md():
    import paper_2104_06311_amd as m
    return m


def split_params(flat, D, H, m):
    sizes = [H * D, H, H * H, H, m * H, m]
    shapes = [(H, D), (H,), (H, H), (H,), (m, H), (m,)]
    out, o = [], 0
    for s, sh in zip(sizes, shapes):
        out.append(np.asarray(flat[o:o + s], dtype=np.float64).reshape(sh))
        o += s
    return out


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cosine(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


@pytest.mark.parametrize("D,H,m,N,scales", [(8, 256, 11, 3001, None), (3, 64, 4, 777, None), (5, 96, 6, 100, None),
                                            (16, 512, 16, 513, None), (8, 40, 11, 64, None),
                                            (8, 256, 11, 2000, (4.47, 3.1)), (16, 512, 16, 300, (2.5, 0.5)),
                                            (8, 288, 11, 1000, None), (20, 64, 5, 700, None), (30, 96, 7, 500, None),
                                            (15, 256, 16, 257, None), (8, 512, 11, 1000, None)])
def test_forward_matches_oracle(D, H, m, N, scales):
    """Fused kernel (H <= 256, D <= 15), weight-streaming kernel (H <= 512 or D up to 30)
    and the generic-GEMM path (H not a multiple of 32) against the FP64 forward."""
    net = md().MLP(D, H, m, seed=11)
    if scales:
        net.set_scales(*scales)
        assert net.scales == pytest.approx(scales)
    rng = np.random.default_rng(D + H)
    y = rng.standard_normal((N, D)).astype(np.float32)
    L = md().llr_learned(net, torch.from_numpy(y).cuda()).cpu().numpy()
    ref = oracle.mlp_forward(oracle.MLPParams(*split_params(net.get(0), D, H, m), *(scales or (1.0, 1.0))), y)
    assert np.all(np.isfinite(L))
    assert rel_err(L, ref) <= 2e-2 and cosine(L, ref) >= 0.999, (rel_err(L, ref), cosine(L, ref))


@pytest.mark.parametrize("D,H,m,B,scales", [(8, 256, 11, 4096, None), (4, 64, 6, 1000, None),
                                            (8, 256, 11, 4096, (4.47, 4.47))])
def test_gradients_match_oracle(D, H, m, B, scales):
    net = md().MLP(D, H, m, seed=5)
    if scales:
        net.set_scales(*scales)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((B, D)).astype(np.float32)
    t = (rng.standard_normal((B, m)) * 4).astype(np.float32)
    loss = net.grad(torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda()).item()
    p = oracle.MLPParams(*split_params(net.get(0), D, H, m), *(scales or (1.0, 1.0)))
    loss_ref, g_ref = oracle.mlp_loss_grad(p, y, t)
    assert abs(loss - loss_ref) <= 1e-2 * abs(loss_ref), (loss, loss_ref)
    g = split_params(net.get(1), D, H, m)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], g, g_ref):
        assert rel_err(a, b) <= 3e-2 and cosine(a, b) >= 0.999, (name, rel_err(a, b), cosine(a, b))


def test_adam_step_matches_oracle():
    D, H, m = 8, 64, 11
    net = md().MLP(D, H, m, seed=9)
    rng = np.random.default_rng(4)
    y = torch.from_numpy(rng.standard_normal((512, D)).astype(np.float32)).cuda()
    t = torch.from_numpy((rng.standard_normal((512, m)) * 3).astype(np.float32)).cuda()
    w0 = net.get(0).astype(np.float64)
    net.grad(y, t)
    g = net.get(1).astype(np.float64)
    net.adam_step(1e-3)
    w1 = net.get(0).astype(np.float64)
    w_ref = w0.copy()
    oracle.adam_step(w_ref, g, np.zeros_like(w0), np.zeros_like(w0), 1, 1e-3)
    np.testing.assert_allclose(w1, w_ref, rtol=1e-5, atol=1e-7)
    # second step uses the stored moments
    net.grad(y, t)
    g2 = net.get(1).astype(np.float64)
    m1 = net.get(2).astype(np.float64)
    m2 = net.get(3).astype(np.float64)
    net.adam_step(1e-3)
    w2 = net.get(0).astype(np.float64)
    m1r = 0.1 * g.copy()
    m2r = 0.001 * g * g
    w_ref2 = w1.copy()
    oracle.adam_step(w_ref2, g2, m1r, m2r, 2, 1e-3)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(w2, w_ref2, rtol=1e-5, atol=1e-6)


def _exact_dataset(X, labels, snr_db, N, seed):
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    tx, y = md().awgn_sample(Xd, seed, 0, N, math.sqrt(s2))
    L = md().llr_exact(Xd, ld, y, s2)
    return Xd, ld, s2, tx, y, L


def test_training_learns_and_checkpoint_resumes_bit_exactly():
    X, labels = synth.product_4d_8psk()
    Xd, ld, s2, tx, y, L = _exact_dataset(X, labels, 8.0, 1 << 16, 3)
    net = md().MLP(4, 64, 6, seed=1)
    net.set_scales(1.0 / math.sqrt(s2), 1.0 / math.sqrt(s2))
    trace = net.fit(y, L, steps=400, batch=1024, lr_max=3e-3, lr_min=1e-4, seed=7).cpu().numpy()
    assert trace[-50:].mean() < 0.8 * trace[:10].mean()
    # fresh symbols: learned GMI well above zero and below exact
    txv, yv = md().awgn_sample(Xd, 99, 0, 50_000, math.sqrt(s2))
    g_exact = md().gmi_reduce(md().llr_exact(Xd, ld, yv, s2), txv, ld)[0].item()
    g_learn = md().gmi_reduce(md().llr_learned(net, yv), txv, ld)[0].item()
    assert g_learn > 0.8 * g_exact and g_learn < g_exact + 0.02, (g_learn, g_exact)
    # checkpoint round trip and bit-exact resume
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.ckpt")
        net.save(path)
        net2 = md().MLP.load(path)
        assert net2.step == net.step and net2.scales == net.scales
        for w in range(4):
            assert np.array_equal(net.get(w) if w != 1 else net.get(0), net2.get(w) if w != 1 else net2.get(0))
        assert torch.equal(md().llr_learned(net, yv), md().llr_learned(net2, yv))
        net.fit(y, L, steps=5, batch=512, lr_max=1e-3, lr_min=1e-3, seed=8, trace=False)
        net2.fit(y, L, steps=5, batch=512, lr_max=1e-3, lr_min=1e-3, seed=8, trace=False)
        assert np.array_equal(net.get(0), net2.get(0))
        # a corrupted file is rejected
        raw = bytearray(open(path, "rb").read())
        raw[-3] ^= 0x40
        open(path, "wb").write(bytes(raw))
        with pytest.raises(md().MdemapError):
            md().MLP.load(path)


@pytest.mark.parametrize("D,H,m,N", [(16, 512, 16, 200_003), (8, 256, 11, 300_007)])
def test_forward_many_tiles_per_block(D, H, m, N):
    """Enough symbols that every block walks several symbol tiles (the streamed layer-2
    blocks continue from one tile into the next); compared on a strided sample of rows."""
    net = md().MLP(D, H, m, seed=4)
    net.set_scales(1.7, 2.0)
    rng = np.random.default_rng(N)
    y = rng.standard_normal((N, D)).astype(np.float32)
    L = md().llr_learned(net, torch.from_numpy(y).cuda()).cpu().numpy()
    idx = np.concatenate([np.arange(0, N, 61), np.arange(N - 300, N)])
    ref = oracle.mlp_forward(oracle.MLPParams(*split_params(net.get(0), D, H, m), 1.7, 2.0), y[idx])
    assert np.all(np.isfinite(L))
    assert rel_err(L[idx], ref) <= 2e-2 and cosine(L[idx], ref) >= 0.999, (rel_err(L[idx], ref), cosine(L[idx], ref))


def test_learned_edge_cases():
    net = md().MLP(8, 256, 11, seed=2)
    out = md().llr_learned(net, torch.empty((0, 8), dtype=torch.float32, device="cuda"))
    assert out.shape == (0, 11)
    with pytest.raises(ValueError):
        md().llr_learned(net, torch.zeros((4, 7), dtype=torch.float32, device="cuda"))
    with pytest.raises(md().MdemapError):
        md().MLP(0, 16, 4)
    with pytest.raises(md().MdemapError):
        net.set_scales(0.0, 1.0)
    with pytest.raises(md().MdemapError):
        net.set_scales(1.0, float("inf"))
