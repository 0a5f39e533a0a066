"""Pins of the oracle's MOD update (Section 1: least-squares dictionary update for a
fixed code matrix) against numpy's least squares, closed forms and exact recovery."""
import numpy as np
import pytest

import oracle
from paper_1403_4781_amd import synth


def _codes_from_dense(X):
    """ELL codes from a dense (N, K) matrix, atoms in increasing order."""
    N, K = X.shape
    s = max(1, int((X != 0).sum(axis=1).max()))
    idx = -np.ones((N, s), np.int32)
    coef = np.zeros((N, s))
    nnz = np.zeros(N, np.int32)
    for n in range(N):
        nz = np.nonzero(X[n])[0]
        idx[n, :len(nz)] = nz
        coef[n, :len(nz)] = X[n, nz]
        nnz[n] = len(nz)
    return oracle.Codes(idx, coef, nnz)


def _normalise(D):
    n = np.linalg.norm(D, axis=1, keepdims=True)
    return np.where(n > 0, D / np.where(n > 0, n, 1), D)


def test_matches_numpy_lstsq_on_active_atoms():
    D, Y, _ = synth.small_problem(11, 64, 128, 5, 0.01, 1500)
    c = oracle.omp(D, Y, 5)
    Dn, nu, ru = oracle.mod_update(Y, c, D)
    X = c.dense(128)
    act = np.abs(X).sum(axis=0) > 0
    # min_D ||Y - D X||_F  <=>  X^T D^T ~ Y^T  (rows = signals)
    Z, *_ = np.linalg.lstsq(X[:, act], Y.astype(np.float64), rcond=None)
    np.testing.assert_allclose(Dn[act], _normalise(Z), rtol=1e-8, atol=1e-10)
    np.testing.assert_array_equal(Dn[~act], D.astype(np.float64)[~act])
    assert nu == int((~act).sum()) and ru == 0


def test_identity_codes_give_normalised_signals():
    """N = K and X = I: the least-squares dictionary is Y itself, then unit-normalised."""
    rng = np.random.default_rng(12)
    Y = rng.standard_normal((20, 8))
    Dn, nu, _ = oracle.mod_update(Y, _codes_from_dense(np.eye(20)), np.zeros((20, 8)))
    np.testing.assert_allclose(Dn, _normalise(Y), rtol=1e-13, atol=1e-14)
    assert nu == 0


def test_noise_free_data_recovers_generating_dictionary():
    """Y = D0 X exactly with X of full row rank: the update returns D0 (unit atoms)."""
    rng = np.random.default_rng(13)
    m, K, N = 16, 24, 400
    D0 = rng.standard_normal((K, m))
    D0 /= np.linalg.norm(D0, axis=1, keepdims=True)
    X = np.zeros((N, K))
    for n in range(N):
        X[n, rng.choice(K, 3, replace=False)] = rng.standard_normal(3)
    Y = X @ D0
    Dn, nu, _ = oracle.mod_update(Y, _codes_from_dense(X), rng.standard_normal((K, m)))
    np.testing.assert_allclose(Dn, D0, rtol=1e-10, atol=1e-11)
    assert nu == 0


def test_optimality_against_perturbations():
    """Before normalisation the update minimises ||Y - D X||_F; the normalised atoms with
    the code rows rescaled accordingly give the same fit, and random perturbations of
    the dictionary never fit better."""
    D, Y, _ = synth.small_problem(14, 32, 48, 4, 0.05, 600)
    c = oracle.omp(D, Y, 4)
    X = c.dense(48)
    Dn, _, _ = oracle.mod_update(Y, c, D)
    Yd = Y.astype(np.float64)
    # optimal scale per atom for the normalised atoms = the unnormalised solution
    Z, *_ = np.linalg.lstsq(X, Yd, rcond=None)
    scale = np.linalg.norm(Z, axis=1)
    fit = np.linalg.norm(Yd - X @ (Dn * scale[:, None]))
    rng = np.random.default_rng(15)
    for _ in range(20):
        P = Dn * scale[:, None] + 1e-3 * rng.standard_normal(Dn.shape)
        assert np.linalg.norm(Yd - X @ P) >= fit - 1e-12


def test_unused_atoms_and_ridge_path():
    """Atoms no signal uses keep their previous value; two atoms used identically make
    X X^T singular, which forces the ridge retry and still returns finite unit atoms."""
    rng = np.random.default_rng(16)
    m, K, N = 8, 6, 50
    Y = rng.standard_normal((N, m))
    X = np.zeros((N, K))
    X[:, 0] = rng.standard_normal(N)
    X[:, 1] = X[:, 0]                 # atoms 0 and 1 always used together with equal weight
    X[:, 2] = rng.standard_normal(N)
    Dprev = _normalise(rng.standard_normal((K, m)))
    Dn, nu, ru = oracle.mod_update(Y, _codes_from_dense(X), Dprev)
    assert nu == 3 and ru == 1
    np.testing.assert_array_equal(Dn[3:], Dprev[3:])
    assert np.all(np.isfinite(Dn))
    np.testing.assert_allclose(np.linalg.norm(Dn, axis=1), 1.0, rtol=1e-12)
    # with the ridge, the two tied atoms get the same direction
    np.testing.assert_allclose(Dn[0], Dn[1], rtol=1e-4, atol=1e-5)
