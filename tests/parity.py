"""Comparison helpers for GPU-vs-oracle parity (shared by the GPU tests).

Bar (the tolerances are those of the project's target statement, with the tie rule of
``oracle.tie_mask`` deciding which signals have a unique answer):
  - support agreement >= 99.9 % on signals away from decision boundaries (exact set equality,
    and identical selection order),
  - coefficients within 1e-4 relative (per signal, l2) on agreeing signals,
  - representation RMSE within 1e-5 absolute.
"""
import numpy as np

import oracle

SUPPORT_FRAC = 0.999
COEF_REL = 1e-4
RMSE_ABS = 1e-5


def to_np(codes):
    """GPU Codes -> (idx, coef float64, nnz) numpy."""
    return (codes.idx.cpu().numpy(), codes.coef.cpu().numpy().astype(np.float64), codes.nnz.cpu().numpy())


def rmse(D, Y, idx, coef, nnz):
    """sqrt(||Y - D X||_F^2 / (m N)) in FP64."""
    D = np.asarray(D, np.float64)
    Y = np.asarray(Y, np.float64)
    N, m = Y.shape
    R = Y.copy()
    s = idx.shape[1]
    for i in range(s):
        ok = i < nnz
        R[ok] -= coef[ok, i][:, None] * D[idx[ok, i]]
    return float(np.sqrt((R ** 2).sum() / (m * max(N, 1))))


def compare(gpu, ora, D, Y, eps=0.0, label=""):
    """Compare GPU codes with oracle codes (oracle run with trace=True).  Returns a dict of
    measured quantities; asserts the parity bar."""
    gi, gc, gn = gpu
    oi, oc, on = ora.idx, ora.coef, ora.nnz
    N = len(on)
    ties = oracle.tie_mask(ora, eps=eps)
    same_nnz = gn == on
    s = oi.shape[1]
    cols = np.arange(s)[None, :]
    gi_m = np.where(cols < gn[:, None], gi[:, :s], -1)
    oi_m = np.where(cols < on[:, None], oi, -1)
    same_order = same_nnz & (gi_m == oi_m).all(axis=1)
    same_set = same_nnz & (np.sort(gi_m, axis=1) == np.sort(oi_m, axis=1)).all(axis=1)
    nt = ~ties
    frac = float(same_set[nt].mean()) if nt.any() else 1.0
    frac_order = float(same_order[nt].mean()) if nt.any() else 1.0
    # coefficients of agreeing signals (aligned by selection order)
    agree = same_order
    if agree.any():
        gca = np.where(cols < gn[:, None], gc[:, :s], 0.0)[agree]
        oca = np.where(cols < on[:, None], oc, 0.0)[agree]
        num = np.linalg.norm(gca - oca, axis=1)
        den = np.maximum(np.linalg.norm(oca, axis=1), 1e-30)
        rel = num / den
        rel = np.where(np.linalg.norm(oca, axis=1) == 0, num, rel)
        coef_max = float(rel.max())
    else:
        coef_max = 0.0
    r_g = rmse(D, Y, gi, gc, gn)
    r_o = rmse(D, Y, oi, oc, on)
    out = dict(N=N, ties=int(ties.sum()), support=frac, order=frac_order, coef_rel_max=coef_max,
               rmse_gpu=r_g, rmse_ora=r_o, rmse_diff=abs(r_g - r_o))
    print(f"[parity {label}] {out}", flush=True)
    assert frac >= SUPPORT_FRAC, out
    assert frac_order >= SUPPORT_FRAC, out
    assert coef_max <= COEF_REL, out
    assert abs(r_g - r_o) <= RMSE_ABS, out
    # unused slots
    assert ((gi[:, :s] == -1) | (cols < gn[:, None])).all()
    assert (np.where(cols < gn[:, None], 0.0, gc[:, :s]) == 0).all()
    return out
