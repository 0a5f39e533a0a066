"""GPU parity of the learned support proposer: logits and gradients against the FP64 oracle
with the same BF16 rounding points, a training step, the exact invariants of the restricted
OMP with fallback, proposer-path parity against the oracle, and the gain of a trained network
over an untrained one.

Tolerances (derived from the arithmetic): FP32 accumulation against FP64 leaves ~1e-6 relative
error, but a hidden activation whose FP32 and FP64 values straddle a BF16 rounding boundary
rounds differently (one BF16 ulp, 2^-8 relative); such flips are rare (about one unit in 10^3)
and bound the logits and gradients to ~1e-3 relative in Frobenius norm.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth
from tests.parity import compare, correlation_network, proposed_oracle, proposer_parity, to_np

pytestmark = pytest.mark.gpu

REL = 2e-3


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


def _t(a, dev, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def _codes_t(c, dev):
    import paper_1403_4781_amd as smdl
    return smdl.Codes(_t(c.idx, dev, np.int32), _t(c.coef, dev), _t(c.nnz, dev, np.int32))


def _relfro(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def test_logits_parity(h, dev):
    widths = [64, 128, 96, 256]
    Ws, bs = synth.mlp_init(widths, seed=11)
    D, Y, _ = synth.small_problem(4000, 64, 256, 8, 0.02, 777)
    print("case logits", flush=True)
    p = h.proposer(Ws, bs)
    lg = p.logits(_t(Y, dev)).cpu().numpy()
    ref = oracle.mlp_forward(Ws, bs, Y)
    e = _relfro(lg, ref)
    print(f"  logits rel {e:.2e} max abs {np.abs(lg - ref).max():.2e}", flush=True)
    assert e <= REL


def test_gradient_parity(h, dev):
    widths = [64, 128, 96, 256]
    Ws, bs = synth.mlp_init(widths, seed=12)
    D, Y, _ = synth.small_problem(4001, 64, 256, 8, 0.02, 300)     # B not a multiple of 32
    labels = oracle.omp(D, Y, 8)
    print("case gradients", flush=True)
    p = h.proposer(Ws, bs)
    loss, dW, db = p.grad(_t(Y, dev), _codes_t(labels, dev))
    lref, dWr, dbr = oracle.mlp_grad(Ws, bs, Y, oracle.multi_hot(labels, 256))
    print(f"  loss gpu {loss:.6f} oracle {lref:.6f}", flush=True)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    for l in range(3):
        ew, eb = _relfro(dW[l].cpu().numpy(), dWr[l]), _relfro(db[l].cpu().numpy(), dbr[l])
        print(f"  layer {l}: dW rel {ew:.2e} db rel {eb:.2e}", flush=True)
        assert ew <= REL and eb <= REL


def test_wide_network_per_layer_path(h, dev):
    """A network whose activations do not fit in LDS (64-4096-1024: 5.2 KB per batch row) runs
    layer by layer; its logits and gradients pass the same bar."""
    widths = [64, 4096, 1024]
    Ws, bs = synth.mlp_init(widths, seed=17)
    D, Y, _ = synth.small_problem(4006, 64, 1024, 8, 0.02, 200)
    labels = oracle.omp(D, Y, 8)
    print("case wide network logits", flush=True)
    p = h.proposer(Ws, bs)
    lg = p.logits(_t(Y, dev)).cpu().numpy()
    e = _relfro(lg, oracle.mlp_forward(Ws, bs, Y))
    print(f"  logits rel {e:.2e}", flush=True)
    assert e <= REL
    print("case wide network gradients", flush=True)
    loss, dW, db = p.grad(_t(Y, dev), _codes_t(labels, dev))
    lref, dWr, dbr = oracle.mlp_grad(Ws, bs, Y, oracle.multi_hot(labels, 1024))
    print(f"  loss gpu {loss:.6f} oracle {lref:.6f}", flush=True)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    for l in range(2):
        ew, eb = _relfro(dW[l].cpu().numpy(), dWr[l]), _relfro(db[l].cpu().numpy(), dbr[l])
        print(f"  layer {l}: dW rel {ew:.2e} db rel {eb:.2e}", flush=True)
        assert ew <= REL and eb <= REL
    p.close()


def test_wide_network_large_batch_logits(h, dev):
    """Per-layer products with at least 256 tiles of 64 x 64 take the 64 x 64 kernel: the
    inference forward of 64-4096-1024 on 1000 signals (bias, ReLU, fragment-order BF16 hidden
    activations, FP32 logits; a ragged last row tile)."""
    rng = np.random.default_rng(23)
    Y = rng.standard_normal((1000, 64)).astype(np.float32)
    print("case 64-4096-1024 logits, 1000 signals", flush=True)
    Ws, bs = synth.mlp_init([64, 4096, 1024], seed=21)
    p = h.proposer(Ws, bs)
    lg = p.logits(_t(Y, dev)).cpu().numpy()
    e = _relfro(lg, oracle.mlp_forward(Ws, bs, Y))
    print(f"  logits rel {e:.2e}", flush=True)
    assert e <= REL
    p.close()


def test_per_layer_training_large_batch(h, dev):
    """64-1024-1024 (over a million weights) trains layer by layer; on 1000 signals every
    product and the weight gradients take the 64 x 64 kernels (BCE output layer, ReLU masks,
    transposed copies, column sums).  Gradients against the oracle, then one Adam step against
    the oracle's Adam applied to the oracle's gradients."""
    widths = [64, 1024, 1024]
    Ws, bs = synth.mlp_init(widths, seed=24)
    rng = np.random.default_rng(25)
    Y = rng.standard_normal((1000, 64)).astype(np.float32)
    idx = np.stack([rng.choice(1024, 8, replace=False) for _ in range(1000)]).astype(np.int32)
    labels = oracle.Codes(idx, np.ones((1000, 8)), np.full(1000, 8, np.int32))
    print("case 64-1024-1024 gradients, 1000 signals", flush=True)
    p = h.proposer(Ws, bs)
    loss, dW, db = p.grad(_t(Y, dev), _codes_t(labels, dev))
    lref, dWr, dbr = oracle.mlp_grad(Ws, bs, Y, oracle.multi_hot(labels, 1024))
    print(f"  loss gpu {loss:.6f} oracle {lref:.6f}", flush=True)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    for l in range(2):
        ew, eb = _relfro(dW[l].cpu().numpy(), dWr[l]), _relfro(db[l].cpu().numpy(), dbr[l])
        print(f"  layer {l}: dW rel {ew:.2e} db rel {eb:.2e}", flush=True)
        assert ew <= REL and eb <= REL
    print("case 64-1024-1024 Adam step", flush=True)
    p.train(_t(Y, dev), _codes_t(labels, dev), epochs=1, batch=1000, lr=1e-3)
    W1, b1 = p.weights()
    for l in range(2):
        for gpu, w0, g in ((W1[l], Ws[l], dWr[l]), (b1[l], bs[l], dbr[l])):
            w = w0.astype(np.float64).ravel().copy()
            mom, vel = np.zeros_like(w), np.zeros_like(w)
            oracle.adam(w, g.ravel().copy(), mom, vel, 1, lr=1e-3)
            e = _relfro(gpu.astype(np.float64).ravel() - w0.astype(np.float64).ravel(), w - w0.astype(np.float64).ravel())
            print(f"  layer {l} update rel {e:.2e}", flush=True)
            assert e <= 0.05     # Adam's first step is ~lr*sign(g): a tiny |g| may flip sign
    p.close()


def test_training_step_and_loss_decrease(h, dev):
    widths = [64, 128, 96, 256]
    Ws, bs = synth.mlp_init(widths, seed=13)
    D, Y, _ = synth.small_problem(4002, 64, 256, 8, 0.02, 4096)
    labels = oracle.omp(D, Y, 8)
    print("case train step", flush=True)
    p = h.proposer(Ws, bs)
    p.train(_t(Y[:512], dev), _codes_t(oracle.Codes(labels.idx[:512], labels.coef[:512], labels.nnz[:512]), dev),
            epochs=1, batch=512, lr=1e-3)
    W1, b1 = p.weights()
    # oracle: same step in FP64
    _, dWr, dbr = oracle.mlp_grad(Ws, bs, Y[:512], oracle.multi_hot(labels, 256)[:512])
    for l in range(3):
        w = Ws[l].astype(np.float64).ravel().copy()
        mom, vel = np.zeros_like(w), np.zeros_like(w)
        oracle.adam(w, dWr[l].ravel().copy(), mom, vel, 1, lr=1e-3)
        dg = W1[l].astype(np.float64).ravel() - Ws[l].astype(np.float64).ravel()
        do = w - Ws[l].astype(np.float64).ravel()
        e = _relfro(dg, do)
        print(f"  layer {l} update rel {e:.2e}", flush=True)
        assert e <= 0.05     # Adam's first step is ~lr*sign(g): a tiny |g| may flip sign
    print("case train epochs", flush=True)
    p2 = h.proposer(Ws, bs)
    losses = p2.train(_t(Y, dev), _codes_t(labels, dev), epochs=5, batch=256, lr=2e-3, shuffle_seed=5)
    print(f"  losses {losses}", flush=True)
    assert losses[-1] < 0.8 * losses[0]


def test_restricted_invariants(h, dev):
    """eps_fallback = 0: every signal falls back, the codes equal plain OMP exactly;
    eps_fallback = inf: none falls back and every chosen atom is a candidate."""
    widths = [64, 128, 256]
    Ws, bs = synth.mlp_init(widths, seed=14)
    D, Y, _ = synth.small_problem(4003, 64, 256, 8, 0.02, 1000)
    Dt, Yt = _t(D, dev), _t(Y, dev)
    p = h.proposer(Ws, bs)
    print("case restricted eps=0", flush=True)
    X0, fb0, n0, _ = h.omp_code_proposed(p, Dt, Yt, 8, 24, 0.0)
    Xp = h.omp_code(Dt, Yt, 8)
    assert n0 == 1000 and int(fb0.sum()) == 1000
    for a, b in zip(to_np(X0), to_np(Xp)):
        np.testing.assert_array_equal(a, b)
    print("case restricted eps=inf", flush=True)
    Xi, fbi, ni, cand = h.omp_code_proposed(p, Dt, Yt, 8, 24, float("inf"), want_cand=True)
    assert ni == 0 and int(fbi.sum()) == 0
    gi, gc, gn = to_np(Xi)
    cn = cand.cpu().numpy()
    assert (np.diff(cn, axis=1) > 0).all()
    for n in range(1000):
        assert set(gi[n, :gn[n]]) <= set(cn[n])


def test_proposed_path_parity(h, dev):
    """GPU proposer path vs the oracle's at the parity bar: candidates, fallback decisions,
    supports, coefficients (1e-4) and RMSE (1e-5), restricted and fallback signals alike; with
    a random network (every signal falls back) and with the correlation network (a share of the
    signals keeps its restricted code), at two thresholds."""
    D, Y, _ = synth.small_problem(4004, 64, 256, 8, 0.02, 2000)
    plain = oracle.omp(D, Y, 8)
    eps_fb = 1.1 * float(np.sqrt(np.mean(plain.res_norm ** 2)))
    Ws, bs = synth.mlp_init([64, 128, 256], seed=15)
    p = h.proposer(Ws, bs)
    print("case proposed parity, random network", flush=True)
    proposer_parity(h, dev, p, D, Y, 8, 24, eps_fb, Ws, bs, "proposed K256 random net")
    p.close()
    Wc, bc = correlation_network(D)
    p = h.proposer(Wc, bc)
    kept = []
    for mult in (1.1, 5.0):
        print(f"case proposed parity, correlation network, threshold x{mult}", flush=True)
        out = proposer_parity(h, dev, p, D, Y, 8, 24, mult * eps_fb, Wc, bc, f"proposed K256 corr x{mult}")
        kept.append(out["restricted"])
    p.close()
    print(f"  restricted codes kept: {kept}", flush=True)
    assert kept[0] >= 40 and kept[1] >= 400


def test_proposer_network_at_benchmark_shape(h, dev):
    """The benchmark's network 64-512-512-256 at its batch of 1024: logits (inference kernel,
    64-row tiles), loss and gradients (the fused training kernel: 512-deep reductions in
    several rounds of its k-loop) and one Adam step, against the oracle."""
    widths = [64, 512, 512, 256]
    Ws, bs = synth.mlp_init(widths, seed=31)
    D, Y, _ = synth.small_problem(4010, 64, 256, 8, 0.02, 1024)
    labels = oracle.omp(D, Y, 8)
    p = h.proposer(Ws, bs)
    print("case 64-512-512-256 logits, 1024 signals", flush=True)
    lg = p.logits(_t(Y, dev)).cpu().numpy()
    e = _relfro(lg, oracle.mlp_forward(Ws, bs, Y))
    print(f"  logits rel {e:.2e}", flush=True)
    assert e <= REL
    print("case 64-512-512-256 gradients, batch 1024", flush=True)
    loss, dW, db = p.grad(_t(Y, dev), _codes_t(labels, dev))
    lref, dWr, dbr = oracle.mlp_grad(Ws, bs, Y, oracle.multi_hot(labels, 256))
    print(f"  loss gpu {loss:.6f} oracle {lref:.6f}", flush=True)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    for l in range(3):
        ew, eb = _relfro(dW[l].cpu().numpy(), dWr[l]), _relfro(db[l].cpu().numpy(), dbr[l])
        print(f"  layer {l}: dW rel {ew:.2e} db rel {eb:.2e}", flush=True)
        assert ew <= REL and eb <= REL
    print("case 64-512-512-256 Adam step, batch 1024, lr 1e-3", flush=True)
    p.train(_t(Y, dev), _codes_t(labels, dev), epochs=1, batch=1024, lr=1e-3)
    W1, b1 = p.weights()
    for l in range(3):
        for gpu, w0, g in ((W1[l], Ws[l], dWr[l]), (b1[l], bs[l], dbr[l])):
            w = w0.astype(np.float64).ravel().copy()
            mom, vel = np.zeros_like(w), np.zeros_like(w)
            oracle.adam(w, g.ravel().copy(), mom, vel, 1, lr=1e-3)
            e = _relfro(gpu.astype(np.float64).ravel() - w0.astype(np.float64).ravel(), w - w0.astype(np.float64).ravel())
            print(f"  layer {l} update rel {e:.2e}", flush=True)
            assert e <= 0.05     # Adam's first step is ~lr*sign(g): a tiny |g| may flip sign
    p.close()


def test_proposed_path_full_size_sampled(h, dev):
    """The learned-proposal path at the benchmark's evaluation size (100000 signals, m=64, K=256,
    s=8, 24 candidates), in the launch configuration the benchmark times: the network on 64-row
    work groups, the top-k, the restricted OMP and the fallback list coded by the full kernel.
    The correlation network (logits |d_k^T y| / ||y||) keeps a share of restricted codes.  400
    sampled signals against the oracle: the candidates (away from a top-24 logit boundary), the
    fallback decisions and the codes."""
    g = synth.rng_streams(4020)
    D = synth.gaussian_dictionary(g[0], 64, 256).astype(np.float32)
    Y, _, _ = synth.sparse_signals(g[1], D.astype(np.float64), 8, 0.02, 100000)
    # the fallback threshold from the oracle's plain codes of 2000 other signals
    Yc, _, _ = synth.sparse_signals(g[2], D.astype(np.float64), 8, 0.02, 2000)
    eps_fb = 1.1 * float(np.sqrt(np.mean(oracle.omp(D, Yc, 8).res_norm ** 2)))
    Wc, bc = correlation_network(D)
    p = h.proposer(Wc, bc)
    rs = np.sort(np.random.default_rng(4021).choice(100000, 400, replace=False))
    lg = oracle.mlp_forward(Wc, bc, Y[rs])
    srt = -np.sort(-lg, axis=1)
    boundary = (srt[:, 23] - srt[:, 24]) < 1e-3 * np.maximum(np.abs(srt[:, 23]), 1.0)
    for mult in (1.0, 3.0):
        # the benchmark's threshold (1.1x the plain residual), and a looser one that keeps many
        # restricted codes
        eps = mult * eps_fb
        print(f"case proposed full size N=100000, threshold x{1.1 * mult:.1f}", flush=True)
        X, fb, nfb, cand = h.omp_code_proposed(p, _t(D, dev), _t(Y, dev), 8, 24, eps, want_cand=True)
        gi, gc, gn = to_np(X)
        cn = cand.cpu().numpy()
        fbg = fb.cpu().numpy().astype(bool)
        print(f"  fallbacks {nfb} of 100000; restricted codes in the sample {int((~fbg[rs]).sum())}", flush=True)
        assert nfb == int(fbg.sum()) and 0 < nfb < 100000
        ora_c = oracle.propose_code(D, Y[rs], lg, 24, 8, eps)
        same_c = (cn[rs] == ora_c.cand).all(axis=1)
        print(f"  candidates agree {same_c[~boundary].mean():.5f} (logit-boundary signals {boundary.sum()})",
              flush=True)
        assert same_c[~boundary].mean() >= 0.999
        ora, fell, dtie = proposed_oracle(D, Y[rs], cn[rs], 8, eps)
        assert (fbg[rs] == fell)[~dtie].all()
        compare((gi[rs], gc[rs], gn[rs]), ora, D, Y[rs], label=f"proposed N=1e5 sampled x{mult}",
                ties=oracle.tie_mask(ora) | dtie)
        if mult > 1.0:
            assert (~fbg[rs]).sum() >= 40
    p.close()


def test_trained_network_gains(h, dev):
    """What training buys, at the benchmark's settings (network 64-512-512-256, 200000 labelled
    pairs, batch 1024, Adam lr 1e-3, 10 epochs, 24 candidates): on fresh signals the trained
    proposer's candidates hold a far larger share of the plain-OMP support than an untrained
    network's (recall@24; ranking the atoms by |D^T y| is printed beside it); fewer
    signals need the full-OMP fallback at the same residual target; the representation error
    stays within 1 % of plain OMP's under the fallback."""
    widths = [64, 512, 512, 256]
    Ws, bs = synth.mlp_init(widths, seed=16)
    g = synth.rng_streams(4005)
    D = synth.gaussian_dictionary(g[0], 64, 256).astype(np.float32)
    Ytr, _, _ = synth.sparse_signals(g[1], D.astype(np.float64), 8, 0.02, 200000)
    Yev, _, _ = synth.sparse_signals(g[2], D.astype(np.float64), 8, 0.02, 5000)
    Dt = _t(D, dev)
    print("case trained gains", flush=True)
    lab, rn_tr = h.omp_code(Dt, _t(Ytr, dev), 8, res_norm=True)
    plain = h.omp_code(Dt, _t(Yev, dev), 8)
    eps_fb = 1.1 * float(torch.sqrt((rn_tr.double() ** 2).mean()).item())
    untrained = h.proposer(Ws, bs)
    trained = h.proposer(Ws, bs)
    losses = trained.train(_t(Ytr, dev), lab, epochs=10, batch=1024, lr=1e-3, shuffle_seed=1)
    print(f"  losses {losses}", flush=True)
    pi, pc, pn = to_np(plain)
    corr = np.argsort(-np.abs(Yev.astype(np.float64) @ D.astype(np.float64).T), axis=1)[:, :24]
    rc = np.mean([len(set(pi[n, :pn[n]]) & set(corr[n])) / max(pn[n], 1) for n in range(5000)])
    print(f"  correlation top-24 recall {rc:.4f}", flush=True)
    res = {}
    from tests.parity import rmse
    for name, p in (("untrained", untrained), ("trained", trained)):
        X, fb, nfb, cand = h.omp_code_proposed(p, Dt, _t(Yev, dev), 8, 24, eps_fb, want_cand=True)
        gi, gc, gn = to_np(X)
        cn = cand.cpu().numpy()
        recall = np.mean([len(set(pi[n, :pn[n]]) & set(cn[n])) / max(pn[n], 1) for n in range(5000)])
        r = rmse(D, Yev, gi, gc, gn) / rmse(D, Yev, pi, pc, pn)
        res[name] = (nfb / 5000, recall, r)
        print(f"  {name}: fallback {nfb / 5000:.4f} recall {recall:.4f} rmse ratio {r:.5f}", flush=True)
    assert res["trained"][1] > res["untrained"][1] + 0.25
    assert res["trained"][0] < res["untrained"][0]
    assert 0.99 <= res["trained"][2] <= 1.05


def _kaiming_expected(widths, seed):
    """The seeded initial weights as the header defines them, drawn with the oracle's own
    splitmix64 (an independent implementation of the same published generator)."""
    g = oracle.splitmix64(seed)

    def draw(n, lo, hi):
        u = np.array([(next(g) >> 11) for _ in range(n)], np.float64) * 2.0 ** -53
        return (lo + (hi - lo) * u).astype(np.float32)

    Ws, bs = [], []
    for fi, fo in zip(widths[:-1], widths[1:]):
        bw, bb = np.sqrt(6.0 / fi), 1.0 / np.sqrt(fi)
        Ws.append(draw(fi * fo, -bw, bw).reshape(fo, fi))
        bs.append(draw(fo, -bb, bb))
    return Ws, bs


def test_seeded_creation_and_weight_setter(h, dev):
    widths = [64, 128, 256]
    print("case seeded proposer", flush=True)
    p = h.proposer_seeded(widths, 99)
    Ws, bs = p.weights()
    We, be = _kaiming_expected(widths, 99)
    for l in range(2):
        np.testing.assert_array_equal(Ws[l], We[l])
        np.testing.assert_array_equal(bs[l], be[l])
    q = h.proposer_seeded(widths, 100)
    assert not np.array_equal(q.weights()[0][0], Ws[0])
    q.close()
    D, Y, _ = synth.small_problem(4010, 64, 256, 8, 0.02, 512)
    lg = p.logits(_t(Y, dev)).cpu().numpy()
    assert _relfro(lg, oracle.mlp_forward(Ws, bs, Y)) <= REL
    print("case weight setter", flush=True)
    W2, b2 = synth.mlp_init(widths, seed=14)
    labels = _codes_t(oracle.omp(D, Y, 8), dev)
    p.train(_t(Y, dev), labels, epochs=2, batch=256, lr=1e-3)     # moves weights and Adam state
    p.set_weights(W2, b2)
    got_W, got_b = p.weights()
    for l in range(2):
        np.testing.assert_array_equal(got_W[l], W2[l].astype(np.float32))
        np.testing.assert_array_equal(got_b[l], b2[l].astype(np.float32))
    lg2 = p.logits(_t(Y, dev)).cpu().numpy()
    assert _relfro(lg2, oracle.mlp_forward(W2, b2, Y)) <= REL
    # training restarts: one step after the reset matches one step of a fresh proposer
    fresh = h.proposer(W2, b2)
    for r in (p, fresh):
        r.train(_t(Y, dev), labels, epochs=1, batch=512, lr=1e-3)
    Wa, _ = fresh.weights()
    Wb, _ = p.weights()
    for l in range(2):
        e = _relfro(Wb[l].astype(np.float64) - W2[l], Wa[l].astype(np.float64) - W2[l])
        print(f"  layer {l} step after reset vs fresh rel {e:.2e}", flush=True)
        assert e <= 1e-3
    with pytest.raises(ValueError):
        p.set_weights(W2[:1], b2[:1])
    p.close()
    fresh.close()


@pytest.mark.parametrize("widths", [[64, 512, 256], [64, 128, 256]])
def test_candidates_are_the_top_logits(h, dev, widths):
    """The candidate sets are exactly the n_c largest of the network's own logits (lower atom
    first on equal logits), for two networks, 1000 rows (a ragged last work group)."""
    Ws, bs = synth.mlp_init(widths, seed=15)
    D, Y, _ = synth.small_problem(4011, 64, 256, 8, 0.02, 1000)
    print(f"case candidates {widths}", flush=True)
    p = h.proposer(Ws, bs)
    Yt = _t(Y, dev)
    lg = p.logits(Yt).cpu().numpy()
    _, _, _, cand = h.omp_code_proposed(p, _t(D, dev), Yt, 8, 24, float("inf"), want_cand=True)
    idx = np.broadcast_to(np.arange(256), lg.shape)
    order = np.lexsort((idx, -lg.astype(np.float64)), axis=1)
    ref = np.sort(order[:, :24], axis=1)
    np.testing.assert_array_equal(cand.cpu().numpy(), ref)
    p.close()
