"""The paper's synthetic experiment (Section 3.1, Table 1) on the CPU: the figures of merit
pinned to closed forms, and the FP64 oracle reproducing the table's qualitative finding on one
trial (the standard alternation represents the data better and recovers more atoms than
split-and-merge).  Table 1 averages 20 trials of an unstated iteration count on unstated
hardware, so its printed values are context, not pins."""
import numpy as np

import oracle
from paper_1403_4781_amd import evaluate, synth


def _table1():
    """Table 1's printed values (Section 3.1), from tests/golden/table1_synthetic.txt."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_synthetic.txt")
    out = {}
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, a, b = line.split()
                out[key] = (float(a), float(b))
    return out


def test_atom_recovery_closed_forms():
    rng = np.random.default_rng(501)
    D = synth.gaussian_dictionary(rng, 30, 60)
    assert evaluate.atom_recovery(D, D) == 1.0
    perm = rng.permutation(60)
    sign = rng.choice([-1.0, 1.0], 60)
    assert evaluate.atom_recovery(D, 3.0 * sign[:, None] * D[perm]) == 1.0
    # atom 0 turned away by an angle of cosine c inside the plane of a unit vector orthogonal to it
    v = rng.standard_normal(30)
    v -= (v @ D[0]) * D[0]
    v /= np.linalg.norm(v)
    for c, expect in ((0.985, 1.0), (0.975, 59 / 60)):
        Dh = D.copy()
        Dh[0] = c * D[0] + np.sqrt(1 - c * c) * v
        # the other atoms must not stand in for atom 0
        assert np.abs(D[1:] @ D[0]).max() < 0.98
        assert evaluate.atom_recovery(D, Dh) == expect


def test_mse_db_closed_forms():
    rng = np.random.default_rng(502)
    D = synth.gaussian_dictionary(rng, 30, 60)
    Y, sup, val = synth.sparse_signals(rng, D, 6, 0.0, 500)
    Yd = Y.astype(np.float64)
    # no codes: the residual is Y itself, 0 dB
    z = np.zeros((500, 6), np.int32)
    assert evaluate.mse_db(Yd, D, z, np.zeros((500, 6)), np.zeros(500, np.int32)) == 0.0
    # the generating codes: only the FP32 rounding of Y remains
    Yx = np.einsum("ns,nsm->nm", val, D[sup])
    assert evaluate.mse_db(Yx, D, sup, val, np.full(500, 6, np.int32)) < -250.0
    # half of every coefficient: the residual is Y / 2, 20 log10(1/2) dB
    r = evaluate.mse_db(Yx, D, sup, 0.5 * val, np.full(500, 6, np.int32))
    assert abs(r - 20 * np.log10(0.5)) < 1e-9
    # entries beyond nnz are ignored
    bad = sup.copy()
    bad[:, 5] = -7
    nnz5 = np.full(500, 5, np.int32)
    a = evaluate.mse_db(Yx, D, bad, val, nnz5)
    b = evaluate.mse_db(Yx, D, sup[:, :5], val[:, :5], nnz5)
    assert a == b


def test_e1_oracle_table1_ordering():
    """One full-size trial (N = 4 x 10^4, 100 iterations per stage): the standard approach ends
    several dB below split-and-merge and recovers more atoms; both recover most of them."""
    oracle.build()
    w = synth.synthetic_e1(1, iters=100)
    D, X = oracle.learn(w.Y, w.K, 6, 100)
    std_db = evaluate.mse_db(w.Y, D, X.idx, X.coef, X.nnz)
    std_rec = evaluate.atom_recovery(w.D0, D)
    D2, X2, _, sc = oracle.split_merge(w.Y, w.perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local,
                                       w.iters_merge, w.s_merge, w.s_final)
    sm_db = evaluate.mse_db(w.Y, D2, X2.idx, X2.coef, X2.nnz)
    sm_rec = evaluate.atom_recovery(w.D0, D2)
    print(f"standard {std_db:.2f} dB {std_rec:.3f}; split-and-merge {sm_db:.2f} dB {sm_rec:.3f}")
    assert len(sc) == 40 and np.all(sc > 0)
    assert X2.nnz.max() <= 6
    assert std_db < sm_db - 3.0
    assert std_rec > sm_rec
    assert std_rec >= 0.9 and sm_rec >= 0.6
    # against the averages Table 1 prints (tests/golden/table1_synthetic.txt): one seeded trial
    # has the table's gap in the training error (same sign, within a factor of 2) and lies within
    # the trial-to-trial spread of its averages: 4 dB and 20 points of recovery, about 2.5
    # standard deviations of 20 trials of this experiment (2.6 dB, 8 points)
    tab = _table1()
    gap, gap_paper = std_db - sm_db, tab["mse_train_db"][0] - tab["mse_train_db"][1]
    assert gap_paper < 0 and 0.5 * gap_paper >= gap >= 2.0 * gap_paper
    assert abs(std_db - tab["mse_train_db"][0]) <= 4.0 and abs(sm_db - tab["mse_train_db"][1]) <= 4.0
    assert abs(100 * std_rec - tab["atom_recovery_percent"][0]) <= 20
    assert abs(100 * sm_rec - tab["atom_recovery_percent"][1]) <= 20
