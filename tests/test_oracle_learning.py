"""Pins of the oracle's learning loop and of Algorithm 1 (Section 2).

Algorithm 1 is an iteration with no closed form, so its pins are structural: the L = 1
reduction to the standard alternation, the pooled data set and its scales, and
Proposition 1 (Section 1, proof in Appendix A) checked on the composed codes the
algorithm produces.  The 10-20 iteration trajectory itself is parity unpinned: the paper
prints no values for it.
"""
import numpy as np
import pytest

import oracle
from paper_1403_4781_amd import synth


def test_alternation_decreases_fit_error():
    """Each MOD step minimises ||Y - D X|| for the current X, so the representation error
    of the codes after the last iteration is below that of the first iteration."""
    D0, Y, _ = synth.small_problem(20, 16, 32, 3, 0.01, 800)
    Yd = Y.astype(np.float64)
    errs = []
    for iters in (0, 1, 5):
        D, c = oracle.learn(Y, 32, 3, iters)
        errs.append(np.linalg.norm(Yd - c.dense(32) @ D))
    assert errs[2] < errs[1] < errs[0]


def test_initialisation_is_first_columns():
    D0, Y, _ = synth.small_problem(21, 16, 32, 3, 0.01, 100)
    D, _ = oracle.learn(Y, 10, 3, 0, codes=False)
    Yd = Y.astype(np.float64)[:10]
    np.testing.assert_allclose(D, Yd / np.linalg.norm(Yd, axis=1, keepdims=True), rtol=1e-13)


def test_single_subset_reduces_to_standard_learning():
    """L = 1: the local dictionary of Algorithm 1 is the standard alternation on the
    (permuted) data, and its scale is the Frobenius norm of that run's final codes."""
    w = synth.oracle_scale(N=600)
    perm = w.perm
    Dsm, _, Dl, sc = oracle.split_merge(w.Y, perm, [0, 600], [64], [5], 64, 3, 2, 3, 5, codes=False)
    Dstd, cstd = oracle.learn(w.Y[perm], 64, 5, 3)
    np.testing.assert_allclose(Dl, Dstd, rtol=1e-12, atol=1e-13)
    assert sc[0] == pytest.approx(np.sqrt((cstd.coef ** 2).sum()), rel=1e-12)


def test_pooled_data_and_merge():
    """Step 3: the pooled set has sum K_t columns, one block per subset; each subset's
    dictionary equals the standard alternation on that subset alone; the merge learns on
    the scaled blocks, initialised with the first K pooled columns."""
    w = synth.oracle_scale(N=900)
    offs = [0, 300, 600, 900]
    Kl, sl = [40, 40, 40], [3, 3, 3]
    D, c, Dl, sc = oracle.split_merge(w.Y, w.perm, offs, Kl, sl, 48, 2, 2, 2, 5)
    assert Dl.shape == (120, 64) and sc.shape == (3,)
    pooled = []
    for t in range(3):
        sub = w.Y[w.perm[offs[t]:offs[t + 1]]]
        Dt, ct = oracle.learn(sub, 40, 3, 2)
        np.testing.assert_allclose(Dl[40 * t:40 * (t + 1)], Dt, rtol=1e-12, atol=1e-13)
        assert sc[t] == pytest.approx(np.sqrt((ct.coef ** 2).sum()), rel=1e-12)
        pooled.append(sc[t] * Dt)
    Dm, _ = oracle.learn(np.vstack(pooled), 48, 2, 2, codes=False)
    np.testing.assert_allclose(D, Dm, rtol=1e-12, atol=1e-13)
    # the final codes are plain OMP of all N signals with the merged dictionary
    cf = oracle.omp(D, w.Y, 5)
    np.testing.assert_array_equal(c.idx, cf.idx)


def test_proposition_1_on_composed_codes():
    """Proposition 1: if y = D~ x1 + e1 (||x1||_0 <= s1) and every used column of D~ is
    D z_j + e_j (||z_j||_0 <= s2), then y = D (Z x1) + E x1 + e1 exactly, ||Z x1||_0 <= s1 s2
    and ||y - D Z x1|| <= K eps2 + eps1 with eps2 = ||x1|| max_j ||e_j|| (K = columns of D~);
    also the sharper ||E x1|| <= sqrt(s1) max_j ||e_j|| ||x1||."""
    w = synth.oracle_scale(N=800)
    offs = [0, 400, 800]
    s1, s2 = 3, 2
    D, _, Dl, sc = oracle.split_merge(w.Y, w.perm, offs, [40, 40], [s1, s1], 48, 3, 3, s2, 6,
                                      codes=False)
    Dt = np.vstack([sc[0] * Dl[:40], sc[1] * Dl[40:]])        # D~ = pooled scaled atoms
    Zc = oracle.omp(D, Dt, s2)                                 # z_j: merge codes of the atoms
    Z = Zc.dense(48).T                                         # (K, 80)
    E = Dt.T - D.T @ Z                                         # e_j as columns
    enorm = np.linalg.norm(E, axis=0)
    Yd = w.Y.astype(np.float64)
    # r from the oracle's composition of the local codes over the unscaled D^(t) (x1 * c_t)
    loc = [oracle.omp(Dt[40 * t:40 * (t + 1)], Yd[w.perm[offs[t]:offs[t + 1]]], s1) for t in range(2)]
    X1u = oracle.Codes(np.vstack([c.idx for c in loc]),
                       np.vstack([loc[t].coef * sc[t] for t in range(2)]),
                       np.concatenate([c.nnz for c in loc]))
    R = oracle.compose_codes(X1u, offs, [40, 40], Zc, sc, 48, perm=w.perm)
    for t in range(2):
        sub = Yd[w.perm[offs[t]:offs[t + 1]]]
        c1 = loc[t]                                            # x1 against D~ (block t)
        X1 = np.zeros((len(sub), 80))
        X1[:, 40 * t:40 * (t + 1)] = c1.dense(40)
        for n in range(len(sub)):
            x1 = X1[n]
            e1 = sub[n] - Dt.T @ x1
            r = R[w.perm[offs[t] + n]]
            np.testing.assert_allclose(sub[n], D.T @ r + E @ x1 + e1, rtol=0, atol=1e-10)
            assert np.count_nonzero(np.abs(r) > 0) <= s1 * s2
            used = np.nonzero(x1)[0]
            if len(used) == 0:
                continue
            eps1 = np.linalg.norm(e1)
            eps2 = np.linalg.norm(x1) * enorm[used].max()
            err = np.linalg.norm(sub[n] - D.T @ r)
            assert err <= Dt.shape[0] * eps2 + eps1 + 1e-12
            assert np.linalg.norm(E @ x1) <= np.sqrt(len(used)) * enorm[used].max() * np.linalg.norm(x1) + 1e-12


def test_splitmix64_published_vectors():
    """The generator of the seeded merge start against the published splitmix64 outputs for
    seed 1234567 (the reference test vector of the generator)."""
    g = oracle.splitmix64(1234567)
    assert [next(g) for _ in range(5)] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                           4593380528125082431, 16408922859458223821]
    p = oracle.seeded_permutation(1000, 99)
    assert sorted(p.tolist()) == list(range(1000))
    assert not np.array_equal(p, np.arange(1000))


def test_seeded_merge_start():
    """With a seeded merge order and no merge iterations, the merged dictionary is the first K
    pooled columns in that order, unit-normalised: the local atoms at those positions (the
    subset scales cancel in the normalisation)."""
    w = synth.patch_scale(N=1200, L=3, iters=0)
    K_local = np.array([64, 64, 64], np.int32)
    s_local = np.array([4, 4, 4], np.int32)
    D, _, Dl, sc = oracle.split_merge(w.Y, w.perm, w.offsets, K_local, s_local, 48, 0, 0, 4, 4, codes=False,
                                      merge_seed=77)
    cols = oracle.seeded_permutation(192, 77)[:48]
    ref = Dl[cols] / np.linalg.norm(Dl[cols], axis=1, keepdims=True)
    np.testing.assert_allclose(D, ref, atol=1e-12)
    D0, _, _, _ = oracle.split_merge(w.Y, w.perm, w.offsets, K_local, s_local, 48, 0, 0, 4, 4, codes=False)
    np.testing.assert_allclose(D0, Dl[:48] / np.linalg.norm(Dl[:48], axis=1, keepdims=True), atol=1e-12)
