"""GPU composition of Algorithm 1's codes by Proposition 1 (proof in Appendix A): teacher-forced
against the oracle's dense composition, and end to end through smdl_split_merge_learn with
SMDL_COMPOSE_CODES."""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth
from tests.parity import rmse, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


def _t(a, dev, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def _codes_t(c, dev):
    import paper_1403_4781_amd as smdl
    return smdl.Codes(_t(c.idx, dev, np.int32), _t(c.coef, dev), _t(c.nnz, dev, np.int32))


def _dense(idx, coef, nnz, K):
    X = np.zeros((len(nnz), K))
    for n in range(len(nnz)):
        for i in range(nnz[n]):
            X[n, idx[n, i]] += coef[n, i]
    return X


def _check_structure(idx, coef, nnz, K, smax):
    assert nnz.min() >= 0 and nnz.max() <= smax
    for n in range(len(nnz)):
        a = idx[n, :nnz[n]]
        assert (a >= 0).all() and (a < K).all() and len(set(a.tolist())) == nnz[n]
        assert (idx[n, nnz[n]:] == -1).all() and (coef[n, nnz[n]:] == 0).all()


def _problem():
    w = synth.oracle_scale(N=800)
    offs, Kl, s1, s2, K = [0, 430, 800], [40, 40], 3, 2, 48
    D, _, Dl, sc = oracle.split_merge(w.Y, w.perm, offs, Kl, [s1, s1], K, 3, 3, s2, 6, codes=False)
    Yp = w.Y[w.perm]
    loc = [oracle.omp(Dl[40 * t:40 * (t + 1)], Yp[offs[t]:offs[t + 1]], s1) for t in range(2)]
    X1 = oracle.Codes(np.vstack([c.idx for c in loc]), np.vstack([c.coef for c in loc]),
                      np.concatenate([c.nnz for c in loc]))
    Dt = np.vstack([sc[0] * Dl[:40], sc[1] * Dl[40:]])
    Z = oracle.omp(D, Dt, s2)
    return w, offs, Kl, s1, s2, K, D, sc, X1, Z


def test_compose_teacher_forced(h, dev):
    """The oracle's local and merge codes composed on the GPU equal the dense composition
    R = Z X1 / c_t (FP32 output of an FP64 sum), with distinct atoms in order of first
    occurrence (local entry, then merge entry)."""
    w, offs, Kl, s1, s2, K, D, sc, X1, Z = _problem()
    print("case compose teacher-forced", flush=True)
    X1f = oracle.Codes(X1.idx, X1.coef.astype(np.float32).astype(np.float64), X1.nnz)
    Zf = oracle.Codes(Z.idx, Z.coef.astype(np.float32).astype(np.float64), Z.nnz)
    R = oracle.compose_codes(X1f, offs, Kl, Zf, sc, K, perm=w.perm)
    X = h.compose_codes(_codes_t(X1f, dev), _codes_t(Zf, dev), offs, Kl, K, sc, torch.from_numpy(w.perm).to(dev))
    gi, gc, gn = to_np(X)
    _check_structure(gi, gc, gn, K, s1 * s2)
    G = _dense(gi, gc.astype(np.float64), gn, K)
    assert np.abs(G - R).max() <= 1e-6 * max(1.0, np.abs(R).max())
    # order of first occurrence, rebuilt by hand for every signal
    aoff = [0, 40]
    for p in range(800):
        t = 0 if p < 430 else 1
        order = []
        for i in range(X1.nnz[p]):
            a = aoff[t] + X1.idx[p, i]
            for k in range(Z.nnz[a]):
                if Z.idx[a, k] not in order:
                    order.append(Z.idx[a, k])
        n = w.perm[p]
        assert gi[n, :gn[n]].tolist() == order


def test_compose_argument_errors(h, dev):
    import paper_1403_4781_amd as smdl
    w, offs, Kl, s1, s2, K, D, sc, X1, Z = _problem()
    with pytest.raises(smdl.SmdlError):
        h.compose_codes(_codes_t(X1, dev), _codes_t(Z, dev), [0, 900, 800], Kl, K, sc)     # decreasing offsets
    with pytest.raises(smdl.SmdlError):
        h.compose_codes(_codes_t(X1, dev), _codes_t(Z, dev), offs, Kl, K, [sc[0], -1.0])  # negative scale
    bad = torch.from_numpy(np.where(np.arange(800) == 5, 800, w.perm)).to(dev)           # entry outside [0, N)
    with pytest.raises(smdl.SmdlError):
        h.compose_codes(_codes_t(X1, dev), _codes_t(Z, dev), offs, Kl, K, sc, bad)


def test_split_merge_composed_codes(h, dev):
    """SMDL_COMPOSE_CODES: the same dictionary as the run with a fresh final coding, and codes that
    are the composition of the run's local codes (a fresh OMP of every subset with its local
    dictionary) with the merge codes (OMP of the pooled scaled atoms with D)."""
    import paper_1403_4781_amd as smdl
    w = synth.oracle_scale(N=2000)
    offs, Kl, sl, K = np.array([0, 700, 1300, 2000]), np.array([64, 48, 64], np.int32), np.array([4, 3, 4], np.int32), 96
    Yt = _t(w.Y, dev)
    perm = torch.from_numpy(w.perm).to(dev)
    print("case split-merge composed", flush=True)
    D0, X0, _, _ = h.split_merge_learn(Yt, perm, offs, Kl, sl, K, 4, 4, 3, 8)
    D1, X1, Dl, sc = h.split_merge_learn(Yt, perm, offs, Kl, sl, K, 4, 4, 3, 8, flags=smdl.SMDL_COMPOSE_CODES,
                                         local=True)
    assert torch.equal(D0, D1)
    gi, gc, gn = to_np(X1)
    _check_structure(gi, gc, gn, K, 4 * 3)
    # rebuild the composition from the run's own dictionaries
    Dln = Dl.cpu().numpy()
    aoff = np.concatenate([[0], np.cumsum(Kl)])
    Yp = _t(w.Y[w.perm], dev)
    parts = [h.omp_code(_t(Dln[aoff[t]:aoff[t + 1]], dev), Yp[offs[t]:offs[t + 1]].contiguous(), int(sl[t]))
             for t in range(3)]
    import paper_1403_4781_amd as smdl2
    loc = smdl2.Codes(torch.cat([torch.nn.functional.pad(p.idx, (0, 4 - p.idx.shape[1]), value=-1) for p in parts]),
                      torch.cat([torch.nn.functional.pad(p.coef, (0, 4 - p.coef.shape[1])) for p in parts]),
                      torch.cat([p.nnz for p in parts]))
    pooled = np.vstack([sc[t] * Dln[aoff[t]:aoff[t + 1]] for t in range(3)]).astype(np.float32)
    Zc = h.omp_code(D1, _t(pooled, dev), 3)
    Xr = h.compose_codes(loc, Zc, offs, Kl, K, sc, perm)
    ri, rc, rn = to_np(Xr)
    same = np.array([gn[n] == rn[n] and (gi[n, :gn[n]] == ri[n, :rn[n]]).all() for n in range(2000)])
    print(f"  rows identical {same.mean():.4f}", flush=True)
    assert same.mean() >= 0.99
    assert np.abs(gc[same] - rc[same]).max() <= 1e-6 * max(1.0, np.abs(rc).max())
    Dn = D1.cpu().numpy()
    r_comp, r_fresh = rmse(Dn, w.Y, gi, gc, gn), rmse(Dn, w.Y, *to_np(X0))
    print(f"  rmse composed {r_comp:.5f} (<= {int(gn.max())} atoms), fresh OMP s=8 {r_fresh:.5f}", flush=True)
    assert np.isfinite(r_comp)
