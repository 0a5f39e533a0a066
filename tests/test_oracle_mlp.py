"""Pins of the oracle's learned support proposer: BF16 rounding against torch's own
conversion, loss against torch's BCE-with-logits, gradients against central finite
differences of the unrounded FP64 network, Adam against torch.optim.Adam, and the exact
invariants of the restricted OMP with fallback."""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth


def _net(widths, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    Ws = [scale * rng.standard_normal((o, i)) / np.sqrt(i) for i, o in zip(widths[:-1], widths[1:])]
    bs = [0.1 * rng.standard_normal(o) for o in widths[1:]]
    return Ws, bs


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(30)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, 65504.0, 3e38]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16(x), ref)
    for v in x[:50]:
        assert oracle.lib().ora_bf16(float(v)) == oracle.bf16(v)


def test_forward_and_loss_match_torch():
    widths = [8, 16, 12, 10]
    Ws, bs = _net(widths, 1)
    rng = np.random.default_rng(31)
    X = rng.standard_normal((7, 8))
    T = (rng.random((7, 10)) < 0.3).astype(np.float64)
    oracle.set_bf16_rounding(False)
    try:
        lg = oracle.mlp_forward(Ws, bs, X)
        loss, _, _ = oracle.mlp_grad(Ws, bs, X, T)
    finally:
        oracle.set_bf16_rounding(True)
    h = torch.tensor(X / np.linalg.norm(X, axis=1, keepdims=True))
    for l, (W, b) in enumerate(zip(Ws, bs)):
        h = h @ torch.tensor(W).T + torch.tensor(b)
        if l + 1 < len(Ws):
            h = torch.relu(h)
    np.testing.assert_allclose(lg, h.numpy(), rtol=1e-12, atol=1e-12)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(h, torch.tensor(T)).item()
    assert loss == pytest.approx(ref, rel=1e-12)


def test_gradients_by_central_differences():
    """With rounding switched off the network is smooth; every weight and bias gradient
    must match (L(w + h) - L(w - h)) / 2h, h = 1e-6, to 1e-6 relative."""
    widths = [6, 9, 7, 5]
    Ws, bs = _net(widths, 2)
    rng = np.random.default_rng(32)
    X = rng.standard_normal((4, 6))
    T = (rng.random((4, 5)) < 0.4).astype(np.float64)
    oracle.set_bf16_rounding(False)
    try:
        _, dW, db = oracle.mlp_grad(Ws, bs, X, T)
        h = 1e-6
        for params, grads in ((Ws, dW), (bs, db)):
            for P, G in zip(params, grads):
                num = np.zeros_like(P)
                for i in np.ndindex(P.shape):
                    old = P[i]
                    P[i] = old + h
                    lp, _, _ = oracle.mlp_grad(Ws, bs, X, T)
                    P[i] = old - h
                    lm, _, _ = oracle.mlp_grad(Ws, bs, X, T)
                    P[i] = old
                    num[i] = (lp - lm) / (2 * h)
                np.testing.assert_allclose(G, num, rtol=1e-6, atol=1e-9)
    finally:
        oracle.set_bf16_rounding(True)


def test_bce_gradient_closed_form():
    """For one layer (a linear model) the logit gradient is (sigmoid(z) - t) / (B K),
    so dW = delta^T h0 with h0 the normalised input (rounding off)."""
    Ws, bs = _net([5, 3], 3)
    rng = np.random.default_rng(33)
    X = rng.standard_normal((6, 5))
    T = (rng.random((6, 3)) < 0.5).astype(np.float64)
    oracle.set_bf16_rounding(False)
    try:
        _, dW, db = oracle.mlp_grad(Ws, bs, X, T)
    finally:
        oracle.set_bf16_rounding(True)
    h0 = X / np.linalg.norm(X, axis=1, keepdims=True)
    z = h0 @ Ws[0].T + bs[0]
    d = (1 / (1 + np.exp(-z)) - T) / T.size
    np.testing.assert_allclose(dW[0], d.T @ h0, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(db[0], d.sum(axis=0), rtol=1e-12, atol=1e-15)


def test_adam_matches_torch():
    rng = np.random.default_rng(34)
    w = rng.standard_normal(50)
    tw = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    mom, vel = np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        oracle.adam(w, g.copy(), mom, vel, t, lr=1e-2)
        opt.zero_grad()
        tw.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(w, tw.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_restricted_omp_invariants():
    """Restricted OMP equals full OMP whenever the full support lies inside the candidate
    set (every greedy argmax over the candidates is then the global one); eps_fallback = 0
    sends every signal to full OMP; eps_fallback = inf keeps every restricted code."""
    D, Y, _ = synth.small_problem(35, 32, 64, 4, 0.01, 200)
    full = oracle.omp(D, Y, 4)
    rng = np.random.default_rng(36)
    # logits that rank the true full-OMP support first, then random atoms
    lg = rng.standard_normal((200, 64))
    for n in range(200):
        lg[n, full.idx[n, :full.nnz[n]]] += 100.0
    r = oracle.propose_code(D, Y, lg, 12, 4, np.inf)
    np.testing.assert_array_equal(r.idx, full.idx)
    np.testing.assert_allclose(r.coef, full.coef, rtol=1e-10, atol=1e-12)
    assert not r.fell_back.any()
    for n in range(200):
        assert set(full.idx[n, :full.nnz[n]]) <= set(r.cand[n])
        assert list(r.cand[n]) == sorted(r.cand[n])
    r0 = oracle.propose_code(D, Y, rng.standard_normal((200, 64)), 12, 4, 0.0)
    assert r0.fell_back.all()
    np.testing.assert_array_equal(r0.idx, full.idx)
    ri = oracle.propose_code(D, Y, rng.standard_normal((200, 64)), 12, 4, np.inf)
    assert not ri.fell_back.any()
    for n in range(200):
        assert set(ri.idx[n, :ri.nnz[n]]) <= set(ri.cand[n])


def test_topk_tie_break_lower_index():
    D, Y, _ = synth.small_problem(37, 16, 20, 2, 0.0, 3)
    lg = np.zeros((3, 20))
    lg[:, 7] = 1.0
    r = oracle.propose_code(D, Y, lg, 5, 2, np.inf)
    for n in range(3):
        assert list(r.cand[n]) == [0, 1, 2, 3, 7]
