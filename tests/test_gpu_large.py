"""GPU parity at the shapes of the large-scale workload: m=256 (16x16 patches), local K=512 and
merged K=1024, s=16, the proposer 256-1024-1024-1024 with 48 candidates.  Sizes are reduced so
that the FP64 oracle finishes in seconds; the kernels run the same code paths as at full size
(the MOD panel no longer fits in LDS at K=1024, top-k takes 64 logits per lane, the restricted
OMP runs its 16-step variant).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth
from tests.parity import compare, correlation_network, proposer_parity, rmse, to_np

pytestmark = pytest.mark.gpu

D_TOL = 1e-4
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


def _random_codes(sup, seed):
    """Codes on the generating supports with random FP32 coefficients (MOD needs no OMP)."""
    rng = np.random.default_rng(seed)
    N, s = sup.shape
    coef = rng.standard_normal((N, s)).astype(np.float32).astype(np.float64)
    return oracle.Codes(sup.astype(np.int32).copy(), coef, np.full(N, s, np.int32))


def test_mod_teacher_forced_large(h, dev):
    """K=1024, m=256, s=16: the FP64 factorisation of the augmented 1280 x 1024 system with the
    first panels read from global memory."""
    m, K, s, N = 256, 1024, 16, 8000
    print(f"case mod large m={m} K={K} s={s} N={N}", flush=True)
    D, Y, sup = synth.small_problem(5000, m, K, s, 0.02, N)
    codes = _random_codes(sup, 5001)
    Dref, nu_ref, _ = oracle.mod_update(Y, codes, D)
    Dg = _t(D, dev)
    nu = h.mod_update(_t(Y, dev), _codes_t(codes, dev), Dg)
    err = np.linalg.norm(Dg.cpu().numpy() - Dref, axis=1).max()
    print(f"  max atom error {err:.3e} unused {nu}/{nu_ref}", flush=True)
    assert nu == nu_ref
    assert err <= D_TOL


def test_proposer_large_logits_and_gradients(h, dev):
    widths = [256, 1024, 1024, 1024]
    Ws, bs = synth.mlp_init(widths, seed=21)
    D, Y, sup = synth.small_problem(5002, 256, 1024, 16, 0.02, 96)     # batch padded to 128
    labels = _random_codes(sup, 5003)
    print("case proposer large", flush=True)
    p = h.proposer(Ws, bs)
    lg = p.logits(_t(Y, dev)).cpu().numpy()
    ref = oracle.mlp_forward(Ws, bs, Y)
    e = _relfro(lg, ref)
    print(f"  logits rel {e:.2e}", flush=True)
    assert e <= REL
    loss, dW, db = p.grad(_t(Y, dev), _codes_t(labels, dev))
    lref, dWr, dbr = oracle.mlp_grad(Ws, bs, Y, oracle.multi_hot(labels, 1024))
    print(f"  loss gpu {loss:.6f} oracle {lref:.6f}", flush=True)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    for l in range(3):
        ew, eb = _relfro(dW[l].cpu().numpy(), dWr[l]), _relfro(db[l].cpu().numpy(), dbr[l])
        print(f"  layer {l}: dW rel {ew:.2e} db rel {eb:.2e}", flush=True)
        assert ew <= REL and eb <= REL
    p.close()


def test_proposed_coding_large(h, dev):
    """48 candidates out of 1024 atoms, s=16: the restricted invariants and parity with the
    oracle's proposer path."""
    widths = [256, 512, 1024]
    Ws, bs = synth.mlp_init(widths, seed=22)
    D, Y, _ = synth.small_problem(5004, 256, 1024, 16, 0.02, 400)
    Dt, Yt = _t(D, dev), _t(Y, dev)
    p = h.proposer(Ws, bs)
    print("case proposed large eps=0 / inf", flush=True)
    X0, fb0, n0, _ = h.omp_code_proposed(p, Dt, Yt, 16, 48, 0.0)
    Xp = h.omp_code(Dt, Yt, 16)
    assert n0 == 400
    for a, b in zip(to_np(X0), to_np(Xp)):
        np.testing.assert_array_equal(a, b)
    Xi, fbi, ni, cand = h.omp_code_proposed(p, Dt, Yt, 16, 48, float("inf"), want_cand=True)
    assert ni == 0
    gi, gc, gn = to_np(Xi)
    cn = cand.cpu().numpy()
    assert (np.diff(cn, axis=1) > 0).all() and cn.min() >= 0 and cn.max() < 1024
    for n in range(400):
        assert set(gi[n, :gn[n]]) <= set(cn[n])
    print("case proposed large parity, random network", flush=True)
    plain = oracle.omp(D, Y, 16)
    eps_fb = 1.1 * float(np.sqrt(np.mean(plain.res_norm ** 2)))
    proposer_parity(h, dev, p, D, Y, 16, 48, eps_fb, Ws, bs, "proposed K1024 random net")
    p.close()
    # the correlation network (logits |d_k^T y| / ||y||): restricted codes survive for a share
    Wc, bc = correlation_network(D)
    p = h.proposer(Wc, bc)
    kept = []
    for mult in (1.1, 5.0):
        print(f"case proposed large parity, correlation network, threshold x{mult}", flush=True)
        out = proposer_parity(h, dev, p, D, Y, 16, 48, mult * eps_fb, Wc, bc, f"proposed K1024 corr x{mult}")
        kept.append(out["restricted"])
    p.close()
    print(f"  restricted codes kept: {kept}", flush=True)
    assert max(kept) >= 40


def test_split_merge_large_reduced(h, dev):
    """Algorithm 1 at the large shapes (m=256, 4 uneven subsets, local K=512 s=16, merge to
    K=1024 with s=8, final s=16, 2 + 2 iterations): unit atoms, pooled-atom count, a final RMSE
    below the initial dictionary's, and the final codes against the oracle's OMP with the
    merged dictionary on a sample."""
    g = synth.rng_streams(5005)
    sizes = synth.uneven_sizes(g[0], 4, 1500, 2500)
    w = synth.make_workload("large_reduced", seed=5006, m=256, K0=1024, s0=16, sigma=0.02, N=int(sizes.sum()),
                            sizes=sizes, K_local=512, s_local=16, K=1024, iters_local=2, iters_merge=2,
                            s_merge=8, s_final=16)
    print(f"case split-merge large N={w.N}", flush=True)
    perm = torch.from_numpy(w.perm).to(dev)
    Yt = _t(w.Y, dev)
    D, X, Dl, sc = h.split_merge_learn(Yt, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local,
                                       w.iters_merge, w.s_merge, w.s_final, local=True)
    Dn = D.cpu().numpy()
    assert Dn.shape == (1024, 256) and Dl.shape[0] == 4 * 512
    np.testing.assert_allclose(np.linalg.norm(Dn, axis=1), 1.0, atol=1e-5)
    assert np.all(np.asarray(sc) > 0)
    r_final = rmse(Dn, w.Y, *to_np(X))
    Yp = w.Y[w.perm]
    D0 = Yp[:1024] / np.linalg.norm(Yp[:1024].astype(np.float64), axis=1, keepdims=True)
    X0 = h.omp_code(_t(D0, dev), Yt, 16)
    r_init = rmse(D0, w.Y, *to_np(X0))
    print(f"  rmse final {r_final:.5f} initial dictionary {r_init:.5f}", flush=True)
    assert r_final < r_init
    ora = oracle.omp(Dn, w.Y[:200], 16, trace=True)
    xi, xc, xn = to_np(X)
    compare((xi[:200], xc[:200], xn[:200]), ora, Dn, w.Y[:200], label="large final")
