"""Learning from a given initial dictionary (the overcomplete DCT start of Section 3.2.1):
smdl_learn_init and the D_local_init / D_merge_init options of Algorithm 1, against the oracle's
coding and MOD from the same start."""
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


def test_learn_from_given_dictionary(h, dev):
    rng = np.random.default_rng(801)
    Dg = synth.gaussian_dictionary(rng, 64, 256)
    Y, _, _ = synth.sparse_signals(rng, Dg, 6, 0.01, 3000)
    D0 = (3.0 * synth.odct(8, 16, 16)).astype(np.float32)         # not unit length on purpose
    D0n = D0.astype(np.float64) / np.linalg.norm(D0.astype(np.float64), axis=1, keepdims=True)
    print("case learn_init iters=0", flush=True)
    D, X = h.learn(_t(Y, dev), 256, 6, 0, D_init=_t(D0, dev))
    np.testing.assert_allclose(D.cpu().numpy(), D0n, atol=1e-6)
    ora = oracle.omp(D.cpu().numpy(), Y, 6, trace=True)
    compare(to_np(X), ora, D.cpu().numpy(), Y, label="learn_init codes")
    print("case learn_init iters=1", flush=True)
    D1, _ = h.learn(_t(Y, dev), 256, 6, 1, D_init=_t(D0, dev))
    gi, gc, gn = to_np(X)
    Dref, _, _ = oracle.mod_update(Y, oracle.Codes(gi, gc, gn), D.cpu().numpy())
    err = np.linalg.norm(D1.cpu().numpy() - Dref, axis=1).max()
    print(f"  max atom error after one iteration {err:.2e}", flush=True)
    assert err <= 1e-4


def test_split_merge_from_given_dictionaries(h, dev):
    w = synth.patch_scale(N=4000, L=4, iters=0)
    Dl0 = synth.odct(8, 16, 8).astype(np.float32)                  # 128 local atoms
    Dm0 = synth.odct(8, 16, 16).astype(np.float32)
    Kl = np.full(4, 128, np.int32)
    print("case split-merge init iters=0", flush=True)
    D, X, Dl, sc = h.split_merge_learn(_t(w.Y, dev), torch.from_numpy(w.perm).to(dev), w.offsets, Kl, w.s_local,
                                       256, 0, 0, 4, 8, local=True, D_local_init=_t(Dl0, dev),
                                       D_merge_init=_t(Dm0, dev))
    np.testing.assert_allclose(D.cpu().numpy(), Dm0, atol=1e-6)
    Dln = Dl.cpu().numpy()
    for t in range(4):
        np.testing.assert_allclose(Dln[128 * t:128 * (t + 1)], Dl0, atol=1e-6)
    assert np.all(sc > 0)
    print("case split-merge init iters=2", flush=True)
    D2, X2, _, _ = h.split_merge_learn(_t(w.Y, dev), torch.from_numpy(w.perm).to(dev), w.offsets, Kl, w.s_local,
                                       256, 2, 2, 4, 8, D_local_init=_t(Dl0, dev), D_merge_init=_t(Dm0, dev))
    np.testing.assert_allclose(np.linalg.norm(D2.cpu().numpy(), axis=1), 1.0, atol=1e-5)
