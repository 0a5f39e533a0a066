"""The batched split phase of Algorithm 1 (step 2 of Section 2: a dictionary per subset) run as one
persistent launch per stage, against the FP64 oracle element by element: every subset's final
local codes, as the persistent work queue produced them, are compared with the oracle's OMP of
that subset against the same local dictionary (the library's, FP32), at the parity bar.  The
subsets have different dictionary widths, sparsities and ragged sizes, and hold more work items
than the persistent grid has work groups, so that the queue wraps.  Also: the seeded merge start,
the fixed-order (deterministic) mode and the non-finite input check of the boundary."""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth
from tests.parity import compare, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


def _t(a, dev, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def _uneven(seed=91, L=6):
    g = synth.rng_streams(seed)
    sizes = synth.uneven_sizes(g[0], L, 2500, 7000)
    Kl = np.array([64, 128, 192, 256, 256, 128], np.int32)[:L]
    sl = np.array([4, 8, 12, 8, 12, 4], np.int32)[:L]
    w = synth.make_workload("batched_parity", seed=seed + 1, m=64, K0=256, s0=8, sigma=0.02, N=int(sizes.sum()),
                            sizes=sizes, K_local=Kl, s_local=sl, K=128, iters_local=0, iters_merge=0,
                            s_merge=4, s_final=8)
    return w


def _local_parity(h, dev, w, iters_local, label, sample=None, flags=0):
    import paper_1403_4781_amd as smdl
    N = w.N
    Xl = smdl.Codes.empty(N, 16, dev)
    _, _, Dl, _ = h.split_merge_learn(_t(w.Y, dev), torch.from_numpy(w.perm).to(dev), w.offsets, w.K_local,
                                      w.s_local, w.K, iters_local, 0, 4, 8, flags=flags, codes=False, local=True,
                                      X_local=Xl)
    Dln = Dl.cpu().numpy()
    xi, xc, xn = to_np(Xl)
    ao = np.concatenate([[0], np.cumsum(w.K_local)])
    for t in range(w.L):
        rows = np.arange(w.offsets[t], w.offsets[t + 1])
        if sample is not None and len(rows) > sample:
            rows = np.sort(np.random.default_rng(t).choice(rows, sample, replace=False))
        Dt = Dln[ao[t]:ao[t + 1]]
        Yt = w.Y[w.perm[rows]]
        s = int(w.s_local[t])
        ora = oracle.omp(Dt, Yt, s, trace=True)
        assert (xi[rows, s:] == -1).all() and (xc[rows, s:] == 0).all()
        compare((xi[rows, :s], xc[rows, :s], xn[rows]), ora, Dt, Yt,
                label=f"{label} subset {t} n{w.offsets[t + 1] - w.offsets[t]} K{w.K_local[t]} s{s}")
    return Dln


def test_batched_launch_parity_iteration0(h, dev):
    """iters_local = 0: the local codes are the persistent launch's coding of the initial local
    dictionaries (the unit-normalised first K_t signals of each subset, checked too)."""
    w = _uneven()
    n_items16 = int(sum((w.offsets[t + 1] - w.offsets[t] + 15) // 16 for t in range(w.L)))
    print(f"case batched iteration 0: N={w.N}, {n_items16} items of 16 signals", flush=True)
    assert n_items16 > 2 * 256
    Dln = _local_parity(h, dev, w, 0, "batched it0")
    ao = np.concatenate([[0], np.cumsum(w.K_local)])
    for t in range(w.L):
        sub = w.Y[w.perm[w.offsets[t]:w.offsets[t] + w.K_local[t]]].astype(np.float64)
        ref = sub / np.linalg.norm(sub, axis=1, keepdims=True)
        assert np.abs(Dln[ao[t]:ao[t + 1]] - ref).max() <= 1e-6


def test_batched_launch_parity_after_learning(h, dev):
    """Two learning iterations (graph-replayed batched coding and MOD): the final local codes
    against the oracle's OMP with the learned local dictionaries (teacher-forced)."""
    w = _uneven(seed=93)
    print(f"case batched after 2 iterations: N={w.N}", flush=True)
    _local_parity(h, dev, w, 2, "batched it2")


def test_batched_full_shape_sampled(h, dev):
    """The uneven-subset workload at full size (64 subsets of 1000-20000 signals, K_t in
    {64, 128, 192, 256}, s_t in {4, 8, 12}): the persistent launch's codes of the initial local
    dictionaries, 40 sampled signals per subset against the oracle."""
    w = synth.batched_split(iters=0)
    print(f"case batched full shape: N={w.N}, L={w.L}", flush=True)
    _local_parity(h, dev, w, 0, "batched full", sample=40)


def test_seeded_merge_start(h, dev):
    """merge_seed: the merge starts from the first K pooled columns in the order of a seeded
    permutation (splitmix64 Fisher-Yates); with no iterations the merged dictionary is those
    columns unit-normalised, as in the oracle (whose permutation is its own implementation of
    the published generator)."""
    w = synth.patch_scale(N=3000, L=3, iters=0)
    Kl = np.array([64, 64, 64], np.int32)
    sl = np.array([4, 4, 4], np.int32)
    print("case seeded merge start", flush=True)
    for seed in (0, 12345):
        D, _, Dl, _ = h.split_merge_learn(_t(w.Y, dev), torch.from_numpy(w.perm).to(dev), w.offsets, Kl, sl, 48,
                                          0, 0, 4, 4, codes=False, local=True, merge_seed=seed)
        Do, _, _, _ = oracle.split_merge(w.Y, w.perm, w.offsets, Kl, sl, 48, 0, 0, 4, 4, codes=False,
                                         merge_seed=seed)
        err = np.abs(D.cpu().numpy() - Do).max()
        print(f"  seed {seed}: max difference {err:.2e}", flush=True)
        assert err <= 1e-6
    assert not np.allclose(oracle.seeded_permutation(192, 12345)[:48], np.arange(48))


def test_deterministic_mode_repeats_bitwise(h, dev):
    """SMDL_DETERMINISTIC: two runs of Algorithm 1 (uneven batched subsets, several iterations,
    merge, final coding) give the same bits; and the same dictionaries as the default mode up to
    rounding."""
    import paper_1403_4781_amd as smdl
    w = _uneven(seed=95, L=4)
    perm = torch.from_numpy(w.perm).to(dev)
    Yt = _t(w.Y, dev)
    runs = []
    for rep in range(2):
        print(f"case deterministic run {rep}", flush=True)
        D, X, Dl, sc = h.split_merge_learn(Yt, perm, w.offsets, w.K_local, w.s_local, w.K, 3, 3, 4, 8,
                                           flags=smdl.SMDL_DETERMINISTIC, local=True)
        runs.append((D.cpu().numpy(), Dl.cpu().numpy(), sc, *to_np(X)))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    print("case deterministic vs default, one MOD update", flush=True)
    D, Y, _ = synth.small_problem(96, 64, 256, 8, 0.02, 6000)
    codes = h.omp_code(_t(D, dev), _t(Y, dev), 8)
    Da, Db = _t(D, dev), _t(D, dev)
    h.set_flags(smdl.SMDL_DETERMINISTIC)
    h.mod_update(_t(Y, dev), codes, Da)
    h.set_flags(0)
    h.mod_update(_t(Y, dev), codes, Db)
    gi, gc, gn = to_np(codes)
    Dref, _, _ = oracle.mod_update(Y, oracle.Codes(gi, gc, gn), D)
    for Dx in (Da, Db):
        assert np.linalg.norm(Dx.cpu().numpy() - Dref, axis=1).max() <= 1e-4


def test_check_finite(h, dev):
    """SMDL_CHECK_FINITE turns a NaN or infinity in the signals into SMDL_E_NUMERIC before any
    work; without the flag the call proceeds."""
    import paper_1403_4781_amd as smdl
    w = synth.patch_scale(N=2000, L=2, iters=0)
    Y = w.Y.copy()
    Y[1234, 5] = np.nan
    Yt = _t(Y, dev)
    perm = torch.from_numpy(w.perm).to(dev)
    print("case check finite", flush=True)
    with pytest.raises(smdl.SmdlError, match="E_NUMERIC"):
        h.split_merge_learn(Yt, perm, w.offsets, np.array([64, 64], np.int32), np.array([4, 4], np.int32), 32, 1, 1,
                            4, 4, flags=smdl.SMDL_CHECK_FINITE)
    D = _t(synth.gaussian_dictionary(np.random.default_rng(3), 64, 128), dev)
    h.set_flags(smdl.SMDL_CHECK_FINITE)
    try:
        with pytest.raises(smdl.SmdlError, match="E_NUMERIC"):
            h.omp_code(D, Yt, 4)
        Y2 = w.Y.copy()
        Y2[7, 0] = np.inf
        with pytest.raises(smdl.SmdlError, match="E_NUMERIC"):
            h.omp_code(D, _t(Y2, dev), 4)
        h.omp_code(D, _t(w.Y, dev), 4)                     # finite data passes
    finally:
        h.set_flags(0)
    h.omp_code(D, Yt, 4)                                   # no check: the call runs
    with pytest.raises(smdl.SmdlError, match="E_ARG"):
        h.set_flags(1)
