"""The large workload at its full size (m=256, N=10^6 signals in 100 uneven subsets), in the launch
configurations its benchmark runs: the persistent batched launch coding every subset against its
initial local dictionary (K=512, s=16), and the coding of all 10^6 signals against a K=1024
dictionary at s=16.  Sampled signals are compared with the FP64 oracle one by one (which codes
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
