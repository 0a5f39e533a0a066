"""Pins of the decision-boundary rule (``oracle.tie_mask``) that decides which signals have a
unique OMP answer.  Each case plants one boundary on an orthonormal dictionary, where the FP64
correlations, residuals and dependence ratios are known in closed form, once just inside the
margin (must be flagged) and once just outside it (must not be): a top-2 correlation gap, a best
correlation near the tau stop, a residual near eps (error-constrained form) and a nearly
dependent atom.  Clear random cases must not be flagged."""
import numpy as np

import oracle

M = 1e-5          # the relative margin of the parity definition


def _eye(m):
    return np.eye(m)


def _flag(D, y, s, eps=0.0):
    c = oracle.omp(D, y[None, :], s, eps=eps, trace=True)
    return bool(oracle.tie_mask(c, eps=eps)[0]), c


def test_top2_gap_inside_and_outside_margin():
    D = _eye(8)
    for delta, want in ((0.5 * M, True), (2.0 * M, False)):
        y = np.zeros(8)
        y[3], y[5] = 1.0, 1.0 - delta          # |c|_(1) = 1, |c|_(2) = 1 - delta: gap = delta
        f, c = _flag(D, y, 1)
        assert abs(c.gap[0, 0] - delta) < 1e-12
        assert c.idx[0, 0] == 3
        assert f is want, (delta, f)


def test_gap_below_tau_stop_is_not_a_tie():
    """A step whose best correlation is far below the tau stop ends the loop whatever the gap:
    the zero signal and a signal equal to one atom (its second step sees only rounding noise)."""
    D = _eye(8)
    f0, c0 = _flag(D, np.zeros(8), 3)
    assert c0.nnz[0] == 0 and not f0
    y = np.zeros(8)
    y[2] = 2.5
    f1, c1 = _flag(D, y, 3)
    assert c1.nnz[0] == 1 and not f1


def test_best_correlation_near_tau():
    D = _eye(8)
    for t, want in ((1.5 * oracle.TAU, True), (0.3 * oracle.TAU, False), (3.0 * oracle.TAU, False)):
        y = np.zeros(8)
        y[0] = 1.0
        y[1] = t                               # step 2 sees |c| = t = t / ||y|| (to 1e-10)
        f, c = _flag(D, y, 2)
        assert abs(c.cmax[0, 1] - t / np.linalg.norm(y)) < 1e-15
        assert f is want, (t, f)


def test_residual_near_eps():
    D = _eye(8)
    y = np.zeros(8)
    y[0], y[1] = 3.0, 0.4                      # residuals: ||y|| = 3.0265..., then 0.4, then 0
    yn = np.linalg.norm(y)
    for off, want in ((0.5 * M * yn, True), (2.0 * M * yn, False), (-0.5 * M * yn, True), (-2.0 * M * yn, False)):
        f, c = _flag(D, y, 4, eps=0.4 + off)
        assert f is want, (off, f)
        assert c.nnz[0] == (1 if off > 0 else 2)


def test_nearly_dependent_atom():
    """d1 = normalize(e0 + h e1): once e0 is chosen, d1's squared distance to span{e0} is
    h^2 / (1 + h^2); the signal makes d1 the second pick."""
    for ratio, want in ((2.0, True), (0.1, False), (20.0, False)):
        q = ratio * oracle.DEP_TOL             # the dependence ratio planted
        h = np.sqrt(q / (1.0 - q))
        D = np.zeros((2, 8))
        D[0, 0] = 1.0
        D[1, 0], D[1, 1] = 1.0, h
        D[1] /= np.linalg.norm(D[1])
        y = 2.0 * D[0] + 1.0 * np.array([0, 1.0, 0, 0, 0, 0, 0, 0])
        f, c = _flag(D, y, 2)
        assert abs(c.l2[0, 1] - q) < 1e-9 * q + 1e-15
        assert f is want, (ratio, f)


def test_clear_random_signals_are_not_flagged():
    rng = np.random.default_rng(7)
    D = rng.standard_normal((128, 64))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    Y = rng.standard_normal((400, 64))
    c = oracle.omp(D, Y, 8, trace=True)
    t = oracle.tie_mask(c)
    # a random gap below 1e-5 at one of 8 steps has probability ~1e-3 per signal
    assert t.mean() <= 0.01
    # the flagged ones (if any) really have a planted-size gap
    assert (np.nanmin(np.where(c.cmax > oracle.TAU, c.gap, np.inf), axis=1)[t] < M).all() or not t.any()
