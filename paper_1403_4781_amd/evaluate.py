"""Figures of merit of the paper's experiments (Section 3.1, Table 1), in FP64 NumPy.

These measure a learned dictionary and its codes; they are not part of the learning path and
run on the host after it.
"""
from __future__ import annotations

import numpy as np


def residual(Y, D, idx, coef, nnz) -> np.ndarray:
    """Y - X D for ELL codes (row n of Y is signal n, row k of D is atom k), FP64."""
    Y = np.asarray(Y, np.float64)
    D = np.asarray(D, np.float64)
    idx = np.asarray(idx)
    coef = np.asarray(coef, np.float64)
    nnz = np.asarray(nnz)
    s = idx.shape[1]
    live = np.arange(s)[None, :] < nnz[:, None]
    safe = np.where(live, idx, 0)
    w = np.where(live, coef, 0.0)
    return Y - np.einsum("ns,nsm->nm", w, D[safe])


def mse_db(Y, D, idx, coef, nnz) -> float:
    """Training error of Table 1 in dB: 20 log10(||Y - D X||_F / ||Y||_F) (the table defines the
    error as the ratio of Frobenius norms and reports it in dB)."""
    R = residual(Y, D, idx, coef, nnz)
    with np.errstate(divide="ignore"):      # an exact representation is -inf dB
        return float(20.0 * np.log10(np.linalg.norm(R) / np.linalg.norm(np.asarray(Y, np.float64))))


def atom_recovery(D_true, D_hat, thr: float = 0.98) -> float:
    """Fraction of the true atoms d_i recovered: some estimated atom d^_j has |d_i . d^_j| >= thr
    (both taken at unit length)."""
    A = np.asarray(D_true, np.float64)
    B = np.asarray(D_hat, np.float64)
    A = A / np.linalg.norm(A, axis=1, keepdims=True)
    nb = np.linalg.norm(B, axis=1, keepdims=True)
    B = B / np.where(nb > 0, nb, 1.0)
    return float(np.mean(np.abs(A @ B.T).max(axis=1) >= thr))


def psnr(clean, est, peak: float = 255.0) -> float:
    """Peak signal-to-noise ratio of an image estimate, 20 log10(peak / RMSE) in dB (Section 3.2)."""
    d = np.asarray(clean, np.float64) - np.asarray(est, np.float64)
    return float(20.0 * np.log10(peak / np.sqrt(np.mean(d * d))))
