"""The allocation-free coding entry point (smdl_omp_code_noalloc), called through the C ABI,
against smdl_omp_code on the same inputs: two calls in a row, the second with fewer signals and a
narrower dictionary (the fixed scratch memory keeps the first call's contents), each compared
with smdl_omp_code at the parity bar (identical supports and counts, coefficients within 1e-4
relative; with the same tile the two give the same bits).  Also: a shape the scratch memory
cannot hold is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1403_4781_amd import synth
from tests.parity import COEF_REL, to_np

pytestmark = pytest.mark.gpu


def _t(a, dev, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def _noalloc(h, D, Y, s, eps=0.0, res=False):
    import paper_1403_4781_amd as smdl
    K, m = D.shape
    N = Y.shape[0]
    X = smdl.Codes.empty(N, s, Y.device)
    r = torch.empty((N,), dtype=torch.float32, device=Y.device) if res else None
    st = smdl.lib().smdl_omp_code_noalloc(h._h, C.c_void_p(D.data_ptr()), m, K, C.c_void_p(Y.data_ptr()), N, s,
                                          float(eps), X._c(), C.c_void_p(r.data_ptr() if r is not None else 0))
    h._check(st)
    return X, r


def _same(a, b, label):
    ai, ac, an = to_np(a)
    bi, bc, bn = to_np(b)
    assert np.array_equal(an, bn), label
    assert np.array_equal(ai, bi), label
    den = np.maximum(np.linalg.norm(bc, axis=1), 1e-30)
    rel = np.linalg.norm(ac - bc, axis=1) / den
    print(f"  [{label}] coef rel max {rel.max():.2e}, bitwise {np.array_equal(ac, bc)}", flush=True)
    assert rel.max() <= COEF_REL


def test_noalloc_matches_omp_code(dev):
    import paper_1403_4781_amd as smdl
    h = smdl.Handle(0)
    cases = [(64, 256, 8, 20000, 0.0), (32, 96, 5, 3001, 0.0)]
    for m, K, s, N, eps in cases:
        D, Y, _ = synth.small_problem(7100 + K, m, K, s, 0.02, N)
        Dt, Yt = _t(D, dev), _t(Y, dev)
        print(f"case noalloc m={m} K={K} s={s} N={N}", flush=True)
        ref, rr = h.omp_code(Dt, Yt, s, eps=eps, res_norm=True)
        got, rg = _noalloc(h, Dt, Yt, s, eps, res=True)
        _same(got, ref, f"m{m} K{K} s{s} N{N}")
        assert torch.allclose(rg, rr, rtol=1e-5, atol=1e-6)
    # error-constrained form on a third, smaller call
    D, Y, _ = synth.small_problem(7200, 64, 128, 4, 0.01, 500)
    Dt, Yt = _t(D, dev), _t(Y, dev)
    print("case noalloc eps form", flush=True)
    _same(_noalloc(h, Dt, Yt, 8, 0.05)[0], h.omp_code(Dt, Yt, 8, eps=0.05), "eps")
    h.close()


def test_noalloc_rejects_bad_arguments(dev):
    import paper_1403_4781_amd as smdl
    h = smdl.Handle(0)
    D = _t(synth.gaussian_dictionary(np.random.default_rng(1), 64, 128), dev)
    Y = _t(np.zeros((10, 64)), dev)
    with pytest.raises(smdl.SmdlError, match="E_SHAPE"):
        _noalloc(h, _t(np.zeros((1100, 64)), dev), Y, 4)          # K > 1024
    with pytest.raises(smdl.SmdlError, match="E_ARG"):
        _noalloc(h, D, Y, 4, eps=-1.0)
    X, _ = _noalloc(h, D, Y, 4)                                    # zero signals: empty codes
    assert int(X.nnz.abs().sum()) == 0
    h.close()
