"""GPU parity of the Gram kernel and the fused OMP kernel against the FP64 oracle.

Covers every lanes-per-signal / signals-per-item tile the library instantiates for the
tested shapes, ragged signal counts, m not a multiple of 4 or 64, K not a multiple of 64,
both OMP forms (sparsity- and error-constrained), degenerate signals, and the full-size
patch-scale workload (m=64, K=256, s=8, N=100000) on sampled signals.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth
from tests.parity import compare, rmse, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("m,K", [(64, 256), (30, 60), (256, 1024), (16, 50)])
def test_gram_matches_fp64(h, dev, m, K):
    print(f"case gram m={m} K={K}", flush=True)
    D, _, _ = synth.small_problem(100 + K, m, K, 3, 0.0, 4)
    G = h.gram(_t(D, dev)).cpu().numpy()
    Gr = D.astype(np.float64) @ D.astype(np.float64).T
    assert np.abs(G - Gr).max() <= 1e-5 * max(1.0, np.abs(Gr).max())


SHAPES = [
    # m, K, s, N, sigma
    (64, 128, 5, 2000, 0.01),     # oracle-scale workload shape
    (64, 256, 8, 3001, 0.02),     # patch scale, ragged N
    (30, 60, 6, 777, 0.01),       # Section 3.1 sizes (m=30, K=60, s=6)
    (64, 64, 4, 500, 0.02),
    (64, 192, 12, 1200, 0.02),
    (256, 512, 16, 300, 0.02),
    (256, 1024, 16, 200, 0.02),
    (16, 50, 3, 333, 0.0),
]


@pytest.mark.parametrize("m,K,s,N,sigma", SHAPES)
def test_omp_parity_all_tiles(h, dev, m, K, s, N, sigma):
    D, Y, _ = synth.small_problem(1000 + m + K + s, m, K, min(s, 8), sigma, N)
    ora = oracle.omp(D, Y, s, trace=True)
    Dt, Yt = _t(D, dev), _t(Y, dev)
    Kpad = (K + 63) // 64 * 64
    tried = 0
    for lanes in (16, 32, 64):
        for spi in (16, 32, 64):
            try:
                h.set_tile(K, s, lanes, spi)
            except Exception:
                continue
            print(f"case omp m={m} K={K} s={s} N={N} lanes={lanes} spi={spi}", flush=True)
            X = h.omp_code(Dt, Yt, s)
            compare(to_np(X), ora, D, Y, label=f"m{m} K{K} s{s} lanes{lanes} spi{spi}")
            tried += 1
    assert tried >= 1, (m, K, s, Kpad)


def test_error_constrained_form(h, dev):
    """eps > 0: stop once ||r|| <= eps (Section 3.2.2), cap s_max."""
    D, Y, _ = synth.small_problem(2001, 64, 256, 6, 0.05, 2000)
    for eps in (0.6, 1.5):
        print(f"case omp-eps eps={eps}", flush=True)
        ora = oracle.omp(D, Y, 16, eps=eps, trace=True)
        X, r = h.omp_code(_t(D, dev), _t(Y, dev), 16, eps=eps, res_norm=True)
        compare(to_np(X), ora, D, Y, eps=eps, label=f"eps{eps}")
        rn = r.cpu().numpy()
        gi, gc, gn = to_np(X)
        yn = np.linalg.norm(Y.astype(np.float64), axis=1)
        # the returned norm is the explicit residual of the returned code (FP32 sums of m
        # squared rows: a few 2^-24 relative), and equals the oracle's where the codes agree
        # (the least-squares residual moves only to second order with the coefficients)
        rr = np.linalg.norm(Y.astype(np.float64) - np.einsum('ns,nsm->nm', gc, D.astype(np.float64)[np.maximum(gi, 0)]),
                            axis=1)
        assert (np.abs(rn - rr) <= 1e-5 * rr + 2e-6 * yn).all(), np.abs(rn - rr).max()
        same = (gn == ora.nnz) & ~oracle.tie_mask(ora, eps=eps)
        assert (np.abs(rn - ora.res_norm)[same] <= (1e-5 * rr + 2e-6 * yn)[same]).all()
        # the stopping rule on the explicit residual: every code that stopped before s_max
        # meets eps (to the rounding of the final square root)
        ok = gn < 16
        assert (rn[ok] <= eps * (1 + 1e-6)).all()


def test_degenerate_signals(h, dev):
    """Zero signals give empty codes; a signal equal to an atom is coded by that atom;
    duplicate atoms are never both chosen; N = 1 and N = 0 work."""
    D, Y, _ = synth.small_problem(2002, 64, 128, 4, 0.01, 40)
    Y[:5] = 0.0
    Y[5] = 2.5 * D[17]
    Ddup = np.vstack([D, D[:8]])
    for DD in (D, Ddup):
        K = DD.shape[0]
        print(f"case degenerate K={K}", flush=True)
        X = h.omp_code(_t(DD, dev), _t(Y, dev), 6)
        gi, gc, gn = to_np(X)
        assert (gn[:5] == 0).all() and (gi[:5] == -1).all() and (gc[:5] == 0).all()
        assert gn[5] == 1 and gi[5, 0] == 17 and abs(gc[5, 0] - 2.5) < 1e-5
        ora = oracle.omp(DD, Y, 6, trace=True)
        # duplicated atoms tie exactly, in FP64 and in FP32 alike (the same values give the same
        # correlations), and the lowest-index rule decides: no signal is excluded as a tie
        compare((gi, gc, gn), ora, DD, Y, label=f"degenerate K{K}",
                ties=None if K == 128 else np.zeros(len(Y), bool))
        if K > 128:
            for n in range(40):
                sel = set(gi[n, :gn[n]])
                for j in range(8):
                    assert not ({j, 128 + j} <= sel)
    print("case N=1", flush=True)
    X = h.omp_code(_t(D, dev), _t(Y[6:7], dev), 4)
    assert X.nnz.shape == (1,)
    print("case N=0", flush=True)
    X = h.omp_code(_t(D, dev), _t(Y[:0], dev), 4)
    assert X.nnz.shape == (0,)


def test_exact_ties_in_every_tile(h, dev):
    """Exact ties between copies of one atom, placed so that for each group width some copies
    share a lane (same or another row of entries) and others sit in different lanes, including
    copies whose higher index lies in a lower lane: the lowest index must win in every tile.
    Signals are 2-sparse (weights 3 and 1) in the copied atoms, coded with s = 2, so that no other
    pair of atoms comes near a tie and the comparison with the oracle is strict."""
    rng = np.random.default_rng(2031)
    m, K, s, N = 64, 256, 2, 600
    D = rng.standard_normal((K, m))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    # (lower, higher) index of each copied pair; entry t of lane g of a 16-lane group holds atom
    # 64 (t / 4) + 4 g + t % 4 (128 (t / 4) + ... for 32 lanes, 256 (t / 4) + ... for 64)
    pairs = [(0, 4), (9, 10), (16, 80), (24, 156), (44, 236), (50, 131), (60, 65), (100, 228)]
    for a, b in pairs:
        D[b] = D[a]
    D = D.astype(np.float32)
    src = rng.integers(0, len(pairs), size=(N, 2))
    src[:, 1] = (src[:, 0] + 1 + rng.integers(0, len(pairs) - 1, size=N)) % len(pairs)
    lo = np.array([a for a, _ in pairs])
    sg = rng.choice([-1.0, 1.0], size=(N, 2))
    w = np.stack([3.0 * sg[:, 0], rng.uniform(0.8, 1.2, N) * sg[:, 1]], axis=1)
    Y = (w[:, :1] * D[lo[src[:, 0]]] + w[:, 1:] * D[lo[src[:, 1]]]).astype(np.float32)
    ora = oracle.omp(D, Y, s, trace=True)
    assert set(np.unique(ora.idx)) <= set(lo.tolist())
    Dt, Yt = _t(D, dev), _t(Y, dev)
    tried = 0
    for lanes in (16, 32, 64):
        for spi in (16, 32, 64):
            try:
                h.set_tile(K, s, lanes, spi)
            except Exception:
                continue
            print(f"case ties lanes={lanes} spi={spi}", flush=True)
            X = h.omp_code(Dt, Yt, s)
            compare(to_np(X), ora, D, Y, label=f"ties lanes{lanes} spi{spi}", ties=np.zeros(N, bool))
            tried += 1
    assert tried >= 3


def test_output_stride_larger_than_sparsity(h, dev):
    import paper_1403_4781_amd as smdl
    D, Y, _ = synth.small_problem(2003, 64, 128, 4, 0.01, 100)
    print("case stride", flush=True)
    out = smdl.Codes.empty(100, 12, dev)
    out.idx.fill_(7)
    out.coef.fill_(3.0)
    X = h.omp_code(_t(D, dev), _t(Y, dev), 4, out=out)
    gi, gc, gn = to_np(X)
    assert (gi[:, 4:] == -1).all() and (gc[:, 4:] == 0).all()
    ora = oracle.omp(D, Y, 4, trace=True)
    compare((gi[:, :4], gc[:, :4], gn), ora, D, Y, label="stride12")


def test_argument_errors(h, dev):
    import paper_1403_4781_amd as smdl
    D, Y, _ = synth.small_problem(2004, 64, 128, 4, 0.01, 10)
    Dt, Yt = _t(D, dev), _t(Y, dev)
    print("case argument errors", flush=True)
    with pytest.raises(smdl.SmdlError):
        h.omp_code(Dt, Yt, 17)          # s > 16
    with pytest.raises(smdl.SmdlError):
        h.omp_code(Dt, Yt, 4, eps=-1.0)
    with pytest.raises(smdl.SmdlError):
        h.omp_code(Dt, Yt, 4, out=smdl.Codes.empty(10, 2, dev))   # stride < s
    with pytest.raises(smdl.SmdlError):
        h.omp_code(_t(np.zeros((1100, 64)), dev), Yt, 4)          # K > 1024


def test_full_size_patch_workload_sampled(h, dev):
    """m=64, K=256, s=8, N=100000 in the launch configuration the benchmark times; 3000
    sampled signals are compared with the oracle one by one, and every code is checked for
    the invariants that hold at any size (support size, distinct atoms, residual bound)."""
    w = synth.patch_scale()
    D = synth.gaussian_dictionary(np.random.default_rng(7), 64, 256).astype(np.float32)
    Yt = _t(w.Y, dev)
    Dt = _t(D, dev)
    print("case full-size N=100000", flush=True)
    X, r = h.omp_code(Dt, Yt, 8, res_norm=True)
    gi, gc, gn = to_np(X)
    assert (gn == 8).mean() > 0.999
    srt = np.sort(np.where(gi >= 0, gi, 10 ** 6), axis=1)
    assert not ((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] < 10 ** 6)).any()
    rs = np.random.default_rng(8).choice(w.N, 3000, replace=False)
    ora = oracle.omp(D, w.Y[rs], 8, trace=True)
    compare((gi[rs], gc[rs], gn[rs]), ora, D, w.Y[rs], label="N=1e5 sampled")
    rr = np.linalg.norm(w.Y[rs].astype(np.float64) - np.einsum('ns,nsm->nm', gc[rs], D.astype(np.float64)[np.maximum(gi[rs], 0)]), axis=1)
    yn = np.linalg.norm(w.Y[rs].astype(np.float64), axis=1)
    assert (np.abs(r.cpu().numpy()[rs] - rr) <= 1e-5 * rr + 2e-6 * yn).all()


def test_async_calls_match_synchronous(h, dev):
    """SMDL_ASYNC: the coding and Gram calls return once queued; after a device synchronisation
    their outputs equal those of the synchronous calls bit for bit (a second, larger shape in
    between makes the workspace grow while the first call's work may still be queued)."""
    import paper_1403_4781_amd as smdl
    D1, Y1, _ = synth.small_problem(2101, 64, 256, 8, 0.02, 3000)
    D2, Y2, _ = synth.small_problem(2102, 64, 512, 8, 0.02, 5000)
    t = [(_t(D1, dev), _t(Y1, dev)), (_t(D2, dev), _t(Y2, dev))]
    print("case async", flush=True)
    ref = [to_np(h.omp_code(Dt, Yt, 8)) for Dt, Yt in t]
    gref = h.gram(t[1][0]).cpu().numpy()
    h.set_flags(smdl.SMDL_ASYNC)
    try:
        got = [h.omp_code(Dt, Yt, 8) for Dt, Yt in t]
        G = h.gram(t[1][0])
        ms = h.last_kernel_ms()
        torch.cuda.synchronize()
    finally:
        h.set_flags(0)
    assert ms > 0.0
    for a, b in zip(got, ref):
        for x, y in zip(to_np(a), b):
            np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(G.cpu().numpy(), gref)
