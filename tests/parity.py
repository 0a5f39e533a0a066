"""Comparison helpers for GPU-vs-oracle parity (shared by the GPU tests).

Bar (the tolerances are those of the project's target statement, with the tie rule of
``oracle.tie_mask`` deciding which signals have a unique answer):
  - support agreement >= 99.9 % on signals away from decision boundaries (exact set equality,
    and identical selection order),
  - coefficients within 1e-4 relative (per signal, l2) on agreeing signals,
  - representation RMSE within 1e-5 absolute.
The signals the tie rule excludes are counted and capped (at most 1 %, or 2 signals on small
sets): an over-eager rule could otherwise make the support check vacuous.
"""
import numpy as np
import torch

import oracle

SUPPORT_FRAC = 0.999
COEF_REL = 1e-4
RMSE_ABS = 1e-5
TIE_FRAC_MAX = 0.01


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


def compare(gpu, ora, D, Y, eps=0.0, label="", ties=None):
    """Compare GPU codes with oracle codes (oracle run with trace=True).  Returns a dict of
    measured quantities; asserts the parity bar.  `ties` (optional bool[N]) replaces the
    oracle's tie rule, for codes assembled from several oracle runs."""
    gi, gc, gn = gpu
    oi, oc, on = ora.idx, ora.coef, ora.nnz
    N = len(on)
    if ties is None:
        ties = oracle.tie_mask(ora, eps=eps)
    assert ties.sum() <= max(2, TIE_FRAC_MAX * N), f"[parity {label}] {int(ties.sum())} of {N} signals excluded as ties"
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


def proposed_oracle(D, Y, cand, s_max, eps_fb, margin=1e-5):
    """The oracle's proposer path with the candidate sets given (teacher-forced on the GPU's
    candidates, so that the comparison of the codes does not depend on logit rounding):
    per signal, OMP restricted to the atoms cand[n] (traced), the fallback decision on the
    restricted code's FP64 residual, and a traced full OMP where it falls back.
    Returns (codes with traces and atom ids of D, fell_back bool[N], decision_tie bool[N]);
    decision_tie marks signals whose restricted residual lies within margin*||y|| of eps_fb,
    where either decision is correct."""
    D = np.asarray(D, np.float64)
    Y = np.asarray(Y, np.float64)
    N = Y.shape[0]
    idx = np.full((N, s_max), -1, np.int32)
    coef = np.zeros((N, s_max))
    nnz = np.zeros(N, np.int32)
    gap, cmax, l2 = (np.full((N, s_max), np.nan) for _ in range(3))
    rn = np.full((N, s_max + 1), np.nan)
    res = np.zeros(N)
    fell = np.zeros(N, bool)
    dtie = np.zeros(N, bool)
    for n in range(N):
        c = np.asarray(cand[n], np.int64)
        r = oracle.omp(D[c], Y[n:n + 1], s_max, trace=True)
        yn = float(np.linalg.norm(Y[n]))
        rr = float(r.res_norm[0])
        dtie[n] = abs(rr - eps_fb) < margin * yn
        if rr > eps_fb:
            fell[n] = True
            continue
        k = int(r.nnz[0])
        idx[n, :k] = c[r.idx[0, :k]]
        coef[n] = r.coef[0]
        nnz[n] = k
        gap[n], cmax[n], l2[n], rn[n] = r.gap[0], r.cmax[0], r.l2[0], r.rn[0]
        res[n] = rr
    if fell.any():
        f = oracle.omp(D, Y[fell], s_max, trace=True)
        idx[fell], coef[fell], nnz[fell] = f.idx, f.coef, f.nnz
        gap[fell], cmax[fell], l2[fell], rn[fell] = f.gap, f.cmax, f.l2, f.rn
        res[fell] = f.res_norm
    out = oracle.Codes(idx, coef, nnz)
    out.gap, out.cmax, out.l2, out.rn, out.res_norm = gap, cmax, l2, rn, res
    return out, fell, dtie


def proposer_parity(h, dev, p, D, Y, s, n_cand, eps_fb, Ws, bs, label):
    """The proposer path against the oracle: the candidate sets against the oracle's own FP64
    network (away from a top-n_c boundary of the logits), then every signal's code, fallback
    decision, coefficients and the RMSE against the oracle's proposer path teacher-forced on
    the GPU's candidate sets, at the parity bar."""
    Dt = torch.from_numpy(np.ascontiguousarray(D, np.float32)).to(dev)
    Yt = torch.from_numpy(np.ascontiguousarray(Y, np.float32)).to(dev)
    X, fb, nfb, cand = h.omp_code_proposed(p, Dt, Yt, s, n_cand, eps_fb, want_cand=True)
    cn = cand.cpu().numpy()
    lg = oracle.mlp_forward(Ws, bs, Y)
    ora_c = oracle.propose_code(D, Y, lg, n_cand, s, eps_fb)
    srt = -np.sort(-lg, axis=1)
    boundary = (srt[:, n_cand - 1] - srt[:, n_cand]) < 1e-3 * np.maximum(np.abs(srt[:, n_cand - 1]), 1.0)
    same_c = (cn == ora_c.cand).all(axis=1)
    print(f"  [{label}] candidates agree {same_c[~boundary].mean():.5f} (logit-boundary signals {boundary.sum()})",
          flush=True)
    assert same_c[~boundary].mean() >= 0.999
    ora, fell, dtie = proposed_oracle(D, Y, cn, s, eps_fb)
    fbg = fb.cpu().numpy().astype(bool)
    print(f"  [{label}] fallbacks gpu {nfb} oracle {int(fell.sum())}, decision ties {int(dtie.sum())}", flush=True)
    assert (fbg == fell)[~dtie].all()
    assert nfb == int(fbg.sum())
    ties = oracle.tie_mask(ora) | dtie
    out = compare(to_np(X), ora, D, Y, label=label, ties=ties)
    out["restricted"] = int((~fbg).sum())
    return out


def correlation_network(D):
    """A two-layer network whose logits are the correlation magnitudes |d_k^T y| / ||y||:
    the first layer holds +D and -D (ReLU keeps the positive part of each), the second adds the
    two.  Its candidates hold the whole support for a good share of signals, so that the
    restricted codes (not only the fallback) reach the parity comparison."""
    K, m = D.shape
    W1 = np.vstack([D, -D]).astype(np.float32)
    W2 = np.hstack([np.eye(K), np.eye(K)]).astype(np.float32)
    return [W1, W2], [np.zeros(2 * K, np.float32), np.zeros(K, np.float32)]
