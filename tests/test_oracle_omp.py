"""Pins of the FP64 oracle's OMP against facts fixed outside the oracle itself.

OMP is the sparse coder of the standard alternation (Section 1); its error-constrained
form is the one used for denoising (Section 3.2.2); Definition 1 is the contract its
output must satisfy.  Each pin below is chosen so that a plausible slip in the oracle
(a wrong argmax, a dropped re-projection, a transposed operand, a wrong stop) fails it.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1403_4781_amd import synth


def _unit_cols(rng, m, K):
    D = rng.standard_normal((K, m))
    return D / np.linalg.norm(D, axis=1, keepdims=True)


def test_s1_is_brute_force_best_single_atom():
    """s = 1: the best 1-sparse approximation is found by trying every atom with
    numpy's least squares; OMP's first pick must be that atom with that weight."""
    rng = np.random.default_rng(0)
    D = _unit_cols(rng, 12, 40)
    Y = rng.standard_normal((200, 12))
    c = oracle.omp(D, Y, 1)
    for n in range(200):
        res = []
        for j in range(40):
            z, *_ = np.linalg.lstsq(D[j][:, None], Y[n], rcond=None)
            res.append(np.linalg.norm(Y[n] - D[j] * z[0]))
        jb = int(np.argmin(res))
        assert c.idx[n, 0] == jb
        assert c.coef[n, 0] == pytest.approx(D[jb] @ Y[n], rel=1e-12, abs=1e-14)


def test_never_better_than_best_subset_and_exact_when_recoverable():
    """Brute force over all C(K, s) supports (m=6, K=10): OMP's residual is never below
    the best-subset residual.  For signals built from a 1-sparse or, with the
    orthonormal part of the dictionary, any s-sparse code, OMP finds the exact support."""
    rng = np.random.default_rng(1)
    m, K = 6, 10
    D = _unit_cols(rng, m, K)
    Y = rng.standard_normal((60, m))
    for s in (1, 2, 3):
        c = oracle.omp(D, Y, s)
        for n in range(60):
            best = np.inf
            for sup in itertools.combinations(range(K), s):
                A = D[list(sup)].T
                z, *_ = np.linalg.lstsq(A, Y[n], rcond=None)
                best = min(best, np.linalg.norm(Y[n] - A @ z))
            assert c.res_norm[n] >= best - 1e-12
    # exact recovery regime: y = a * d_j is recovered by a single pick
    for j in range(K):
        c = oracle.omp(D, 1.7 * D[j][None, :], 3)
        assert c.nnz[0] == 1 and c.idx[0, 0] == j
        assert c.coef[0, 0] == pytest.approx(1.7, rel=1e-12)


def test_orthonormal_dictionary_closed_form():
    """K = m, D orthonormal: OMP picks the s largest |D^T y| in decreasing order and the
    coefficients are exactly those inner products."""
    rng = np.random.default_rng(2)
    m = 16
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    D = Q.T                      # rows are orthonormal atoms
    Y = rng.standard_normal((100, m))
    s = 5
    c = oracle.omp(D, Y, s)
    for n in range(100):
        a = D @ Y[n]
        order = np.argsort(-np.abs(a), kind="stable")[:s]
        assert list(c.idx[n]) == list(order)
        np.testing.assert_allclose(c.coef[n], a[order], rtol=1e-12, atol=1e-13)


def _hadamard(n):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def test_identity_union_hadamard_exact_recovery():
    """Identity plus normalised Hadamard basis at m=64 (mutual coherence 1/8).  Tropp's
    condition mu < 1/(2s-1) holds for s <= 4, so OMP recovers every noise-free s-sparse
    signal exactly (support and coefficients)."""
    m = 64
    D = np.vstack([np.eye(m), _hadamard(m).T / np.sqrt(m)])
    G = np.abs(D @ D.T - np.eye(2 * m))
    assert G.max() == pytest.approx(1 / 8)
    rng = np.random.default_rng(3)
    for s in (1, 2, 3, 4):
        N = 300
        sup = np.argsort(rng.random((N, 2 * m)), axis=1)[:, :s]
        val = rng.standard_normal((N, s)) + np.sign(rng.standard_normal((N, s)))
        Y = np.einsum('ns,nsm->nm', val, D[sup])
        c = oracle.omp(D, Y, s)
        for n in range(N):
            got = dict(zip(c.idx[n], c.coef[n]))
            want = dict(zip(sup[n], val[n]))
            assert set(got) == set(want)
            for k in want:
                assert got[k] == pytest.approx(want[k], rel=1e-10, abs=1e-12)


def test_invariants_on_random_data():
    """Residual orthogonal to the chosen atoms; coefficients equal numpy lstsq on the
    support; residual norm non-increasing over the steps; Definition 1 predicate."""
    D, Y, _ = synth.small_problem(7, 64, 128, 5, 0.01, 400)
    Dd, Yd = D.astype(np.float64), Y.astype(np.float64)
    c = oracle.omp(D, Y, 8, trace=True)
    for n in range(400):
        I = c.idx[n, :c.nnz[n]]
        assert len(set(I)) == len(I)
        z, *_ = np.linalg.lstsq(Dd[I].T, Yd[n], rcond=None)
        np.testing.assert_allclose(c.coef[n, :c.nnz[n]], z, rtol=1e-9, atol=1e-12)
        r = Yd[n] - Dd[I].T @ c.coef[n, :c.nnz[n]]
        assert np.abs(Dd[I] @ r).max() <= 1e-12 * max(1.0, np.linalg.norm(Yd[n]))
        rn = c.rn[n][~np.isnan(c.rn[n])]
        assert np.all(np.diff(rn) <= 1e-12)
        # Definition 1: ||x||_0 <= s and ||y - D x|| <= eps with eps = the returned residual
        assert c.nnz[n] <= 8
        assert np.linalg.norm(r) == pytest.approx(c.res_norm[n], rel=1e-9, abs=1e-12)
    assert (c.idx[c.nnz[:, None] <= np.arange(8)[None, :]] == -1).all()


def test_scale_and_permutation_equivariance():
    """OMP(c y) = c OMP(y); permuting the atoms permutes the chosen indices."""
    D, Y, _ = synth.small_problem(8, 32, 64, 4, 0.01, 200)
    c1 = oracle.omp(D, Y, 4)
    c2 = oracle.omp(D, -3.5 * Y.astype(np.float64), 4)
    np.testing.assert_array_equal(c1.idx, c2.idx)
    np.testing.assert_allclose(c2.coef, -3.5 * c1.coef, rtol=1e-10, atol=1e-12)
    p = np.random.default_rng(4).permutation(64)
    c3 = oracle.omp(D[p], Y, 4)
    inv = np.argsort(p)
    np.testing.assert_array_equal(np.where(c3.idx >= 0, p[np.maximum(c3.idx, 0)], -1), c1.idx)
    np.testing.assert_allclose(c3.coef, c1.coef, rtol=1e-10, atol=1e-12)
    assert inv.shape == p.shape


def test_error_constrained_form():
    """Section 3.2.2 form: stop as soon as ||r|| <= eps; so either ||r|| <= eps at the end
    or the cap was reached, and one pick fewer would have left ||r|| > eps."""
    D, Y, _ = synth.small_problem(9, 64, 128, 6, 0.05, 300)
    eps = 0.6
    c = oracle.omp(D, Y, 20, eps=eps, trace=True)
    for n in range(300):
        k = c.nnz[n]
        assert c.res_norm[n] <= eps or k == 20
        if k > 0:
            assert c.rn[n, k - 1] > eps
    # a signal already inside the eps ball gets the empty code
    z = oracle.omp(D, 0.01 * Y[:5], 20, eps=10.0)
    assert (z.nnz == 0).all() and (z.idx == -1).all()


def test_degenerate_inputs():
    """Zero signals give empty codes; duplicate atoms are never both chosen."""
    D, Y, _ = synth.small_problem(10, 16, 32, 3, 0.0, 10)
    c = oracle.omp(D, np.zeros((3, 16)), 4)
    assert (c.nnz == 0).all()
    Ddup = np.vstack([D, D[:4]])       # atoms 32..35 duplicate atoms 0..3
    c = oracle.omp(Ddup, Y, 6)
    for n in range(10):
        I = set(c.idx[n, :c.nnz[n]])
        for j in range(4):
            assert not ({j, 32 + j} <= I)
