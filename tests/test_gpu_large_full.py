"""The large workload at its full size (m=256, N=10^6 signals in 100 uneven subsets), in the launch
configurations its benchmark runs: the persistent batched launch coding every subset against its
initial local dictionary (K=512, s=16), the batched MOD update of all 100 local dictionaries, and
the coding of all 10^6 signals against a K=1024 dictionary at s=16.  Sampled signals are compared with the FP64 oracle one by one (which codes
them individually in milliseconds); every code is checked for the invariants that hold at any
size."""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import synth
from tests.parity import compare, to_np
from tests.test_gpu_batched import _local_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


@pytest.fixture(scope="module")
def w():
    print("generating the large workload (10^6 signals of 256)", flush=True)
    return synth.large_scale(iters=0)


def _t(a, dev, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def test_large_batched_local_coding_sampled(h, dev, w):
    """100 subsets of 5000-15000 signals, each coded by the persistent launch against its initial
    local dictionary (K=512, s=16); 3 sampled signals per subset against the oracle."""
    print(f"case large batched local coding: N={w.N}, L={w.L}", flush=True)
    _local_parity(h, dev, w, 0, "large local", sample=3)


def test_large_final_coding_sampled(h, dev, w):
    """All 10^6 signals against a K=1024 dictionary at s=16; 300 sampled signals against the
    oracle, every code checked for its size and distinct atoms."""
    D = synth.gaussian_dictionary(np.random.default_rng(77), 256, 1024).astype(np.float32)
    print("case large final coding: N=1000000, K=1024, s=16", flush=True)
    X = h.omp_code(_t(D, dev), _t(w.Y, dev), 16)
    gi, gc, gn = to_np(X)
    assert (gn == 16).mean() > 0.999
    assert ((gi >= -1) & (gi < 1024)).all()
    srt = np.sort(np.where(gi >= 0, gi, 10 ** 6), axis=1)
    assert not ((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] < 10 ** 6)).any()
    rs = np.sort(np.random.default_rng(78).choice(w.N, 300, replace=False))
    ora = oracle.omp(D, w.Y[rs], 16, trace=True)
    compare((gi[rs], gc[rs], gn[rs]), ora, D, w.Y[rs], label="large final N=1e6 sampled")


def test_large_batched_mod_sampled(h, dev, w):
    """One MOD update of all 100 local dictionaries (K=512, m=256, s=16) at full size in the
    batched launches, teacher-forced: the split phase run with no iteration gives the codes of the
    initial dictionaries, which are the codes the update of a one-iteration run uses; five sampled
    subsets' updated dictionaries against the oracle's MOD of those codes."""
    import paper_1403_4781_amd as smdl
    Yt = _t(w.Y, dev)
    perm = torch.from_numpy(w.perm).to(dev)
    print("case large batched MOD: codes of the initial local dictionaries", flush=True)
    X0 = smdl.Codes.empty(w.N, 16, dev)
    _, _, Dl0, _ = h.split_merge_learn(Yt, perm, w.offsets, w.K_local, w.s_local, w.K, 0, 0, 8, 16, codes=False,
                                       local=True, X_local=X0)
    print("case large batched MOD: one iteration", flush=True)
    _, _, Dl1, _ = h.split_merge_learn(Yt, perm, w.offsets, w.K_local, w.s_local, w.K, 1, 0, 8, 16, codes=False,
                                       local=True)
    xi, xc, xn = to_np(X0)
    D0n, D1n = Dl0.cpu().numpy(), Dl1.cpu().numpy()
    ao = np.concatenate([[0], np.cumsum(w.K_local)])
    for t in np.sort(np.random.default_rng(79).choice(w.L, 5, replace=False)):
        rows = np.arange(w.offsets[t], w.offsets[t + 1])
        codes = oracle.Codes(xi[rows].copy(), xc[rows].astype(np.float64), xn[rows].copy())
        Dref, nu, _ = oracle.mod_update(w.Y[w.perm[rows]], codes, D0n[ao[t]:ao[t + 1]])
        err = np.linalg.norm(D1n[ao[t]:ao[t + 1]] - Dref, axis=1).max()
        print(f"  subset {t} (n={len(rows)}): max atom error {err:.3e}, unused {nu}", flush=True)
        assert err <= 1e-4
