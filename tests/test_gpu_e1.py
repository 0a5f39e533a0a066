"""The paper's synthetic experiment (Section 3.1, Table 1) through the library, against the FP64
oracle on the same inputs.  Learning over 100 iterations is chaotic: one near-tie decided the
other way changes every later dictionary, so a trial either follows the oracle's trajectory
(then its figures agree to rounding) or lands on another solution of similar quality.  The
test asks for both: at least one of three trials on the oracle's trajectory, and three-trial
means that agree within the trial-to-trial spread (about 2.5 dB and 8 recovery points at one
standard deviation)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1403_4781_amd import evaluate, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(dev):
    import paper_1403_4781_amd as smdl
    return smdl.Handle(0)


def test_e1_against_oracle(h, dev):
    oracle.build()
    res = {"gpu": {"std": [], "sm": []}, "ora": {"std": [], "sm": []}}
    for t in range(3):
        print(f"case e1 trial {t}", flush=True)
        w = synth.synthetic_e1(t, iters=100)
        Y = torch.from_numpy(w.Y).to(dev)
        perm = torch.from_numpy(w.perm).to(dev)
        D, X = h.learn(Y, w.K, 6, 100)
        Xn = [a.cpu().numpy() for a in (X.idx, X.coef, X.nnz)]
        res["gpu"]["std"].append((evaluate.mse_db(w.Y, D.cpu().numpy(), *Xn), evaluate.atom_recovery(w.D0, D.cpu().numpy())))
        D, X, _, _ = h.split_merge_learn(Y, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local, w.iters_merge,
                                         w.s_merge, w.s_final)
        Xn = [a.cpu().numpy() for a in (X.idx, X.coef, X.nnz)]
        res["gpu"]["sm"].append((evaluate.mse_db(w.Y, D.cpu().numpy(), *Xn), evaluate.atom_recovery(w.D0, D.cpu().numpy())))
        Do, Xo = oracle.learn(w.Y, w.K, 6, 100)
        res["ora"]["std"].append((evaluate.mse_db(w.Y, Do, Xo.idx, Xo.coef, Xo.nnz), evaluate.atom_recovery(w.D0, Do)))
        Do, Xo, _, _ = oracle.split_merge(w.Y, w.perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local,
                                          w.iters_merge, w.s_merge, w.s_final)
        res["ora"]["sm"].append((evaluate.mse_db(w.Y, Do, Xo.idx, Xo.coef, Xo.nnz), evaluate.atom_recovery(w.D0, Do)))
        for k in ("std", "sm"):
            g, o = res["gpu"][k][-1], res["ora"][k][-1]
            print(f"  {k}: gpu {g[0]:.2f} dB {g[1]:.3f}  oracle {o[0]:.2f} dB {o[1]:.3f}", flush=True)
    for k in ("std", "sm"):
        g, o = np.array(res["gpu"][k]), np.array(res["ora"][k])
        same = (np.abs(g[:, 0] - o[:, 0]) <= 0.1) & (np.abs(g[:, 1] - o[:, 1]) <= 1.5 / 60)
        assert same.any(), (k, g, o)
        assert abs(g[:, 0].mean() - o[:, 0].mean()) <= 3.0
        assert abs(g[:, 1].mean() - o[:, 1].mean()) <= 0.12
    # the finding of Table 1 on the GPU: the standard approach is better on both figures
    gs, gm = np.array(res["gpu"]["std"]), np.array(res["gpu"]["sm"])
    assert gs[:, 0].mean() < gm[:, 0].mean() - 3.0
    assert gs[:, 1].mean() > gm[:, 1].mean()
