"""Python access to the FP64 CPU oracle (``smdl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke`` and by
the CPU-baseline leg of ``bench.py``.  The product package never imports it.

Arrays follow the column-major convention of the C code: Y (m x N) is a NumPy array of
shape (N, m), D (m x K) has shape (K, m).  Everything is converted to float64 here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smdl_oracle.c")
LIB = os.path.join(HERE, "libsmdl_oracle.so")

# Numerical constants of the reading of the paper shared (by value, not by code) with the
# GPU path: the greedy loop stops when the best correlation is below TAU * ||y|| or when
# the chosen atom is numerically dependent on those already chosen.
TAU = 1e-5
DEP_TOL = 1e-5

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over signals)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp, ip, i64p, u8p = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int64), C.POINTER(C.c_uint8))
        L.ora_omp.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int64, C.c_int, C.c_double, C.c_double,
                              C.c_double, ip, dp, ip, dp, dp, dp, dp, dp]
        L.ora_mod_update.argtypes = [dp, C.c_int, C.c_int64, ip, dp, ip, C.c_int, C.c_int, dp, ip, ip]
        L.ora_learn.argtypes = [dp, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_double,
                                C.c_double, dp, ip, dp, ip]
        L.ora_split_merge.argtypes = [dp, C.c_int, C.c_int64, i64p, C.c_int, i64p, ip, ip, C.c_int,
                                      C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                      dp, ip, dp, ip, dp, dp, i64p]
        L.ora_set_bf16.argtypes = [C.c_int]
        L.ora_threads.restype = C.c_int
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_bf16.argtypes = [C.c_double]
        L.ora_bf16.restype = C.c_double
        L.ora_mlp_forward.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(dp), C.POINTER(dp), dp,
                                      C.c_int64, dp]
        L.ora_mlp_grad.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(dp), C.POINTER(dp), dp, dp,
                                   C.c_int64, dp, C.POINTER(dp), C.POINTER(dp)]
        L.ora_adam.argtypes = [dp, dp, dp, dp, C.c_int64, C.c_int, C.c_double, C.c_double,
                               C.c_double, C.c_double]
        L.ora_propose_code.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int64, dp, C.c_int, C.c_int,
                                       C.c_double, C.c_double, C.c_double, ip, dp, ip, u8p, ip]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


class Codes:
    """ELL sparse codes: idx (N, s) int32, coef (N, s) float64, nnz (N,) int32."""

    def __init__(self, idx, coef, nnz):
        self.idx, self.coef, self.nnz = idx, coef, nnz

    def dense(self, K: int) -> np.ndarray:
        """X as a dense (N, K) array (row n = code of signal n)."""
        N, s = self.idx.shape
        X = np.zeros((N, K))
        for i in range(s):
            ok = i < self.nnz
            X[np.nonzero(ok)[0], self.idx[ok, i]] = self.coef[ok, i]
        return X


def omp(D, Y, s_max, eps=0.0, tau=TAU, dep_tol=DEP_TOL, trace=False):
    """OMP of every signal (rows of Y, shape (N, m)) against D (shape (K, m))."""
    D, Y = _d(D), _d(Y)
    K, m = D.shape
    N = Y.shape[0]
    assert Y.shape[1] == m
    idx = np.empty((N, s_max), np.int32)
    coef = np.empty((N, s_max))
    nnz = np.empty(N, np.int32)
    res = np.empty(N)
    tr = [np.empty((N, s_max)) for _ in range(3)] + [np.empty((N, s_max + 1))] if trace else [None] * 4
    rc = lib().ora_omp(_p(D, C.c_double), m, K, _p(Y, C.c_double), N, s_max, eps, tau, dep_tol,
                       _p(idx, C.c_int32), _p(coef, C.c_double), _p(nnz, C.c_int32), _p(res, C.c_double),
                       *[_p(t, C.c_double) for t in tr])
    assert rc == 0, rc
    out = Codes(idx, coef, nnz)
    out.res_norm = res
    if trace:
        out.gap, out.cmax, out.l2, out.rn = tr
    return out


def mod_update(Y, codes: Codes, D):
    """MOD update; returns (D_new (K, m), n_unused, ridge_used) or raises on failure."""
    Y = _d(Y)
    Dn = _d(D).copy()
    K, m = Dn.shape
    N, s = codes.idx.shape
    nu, ru = C.c_int32(0), C.c_int32(0)
    idx = np.ascontiguousarray(codes.idx, np.int32)
    coef = _d(codes.coef)
    nnz = np.ascontiguousarray(codes.nnz, np.int32)
    rc = lib().ora_mod_update(_p(Y, C.c_double), m, N, _p(idx, C.c_int32), _p(coef, C.c_double),
                              _p(nnz, C.c_int32), s, K, _p(Dn, C.c_double), C.byref(nu), C.byref(ru))
    if rc != 0:
        raise FloatingPointError(f"oracle MOD failed ({rc})")
    return Dn, nu.value, ru.value


def learn(Y, K, s, iters, tau=TAU, dep_tol=DEP_TOL, codes=True):
    Y = _d(Y)
    N, m = Y.shape
    D = np.empty((K, m))
    idx = np.empty((N, s), np.int32) if codes else None
    coef = np.empty((N, s)) if codes else None
    nnz = np.empty(N, np.int32) if codes else None
    rc = lib().ora_learn(_p(Y, C.c_double), m, N, K, s, iters, tau, dep_tol, _p(D, C.c_double),
                         _p(idx, C.c_int32), _p(coef, C.c_double), _p(nnz, C.c_int32))
    if rc != 0:
        raise FloatingPointError(f"oracle learn failed ({rc})")
    return D, (Codes(idx, coef, nnz) if codes else None)


_MASK64 = (1 << 64) - 1


def splitmix64(seed: int):
    """The splitmix64 generator (Steele, Lea and Flood, OOPSLA 2014), from its published
    definition: the state advances by the golden-ratio increment 0x9E3779B97F4A7C15 and each
    output is the state passed through the variant-13 finaliser (xor-shift 30, multiply
    0xBF58476D1CE4E5B9, xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31)."""
    state = seed & _MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        yield z ^ (z >> 31)


def seeded_permutation(n: int, seed: int) -> np.ndarray:
    """0..n-1 shuffled by Fisher-Yates from the last position down, position i exchanged with
    position (next splitmix64 output) mod (i + 1)."""
    p = list(range(n))
    g = splitmix64(seed)
    for i in range(n - 1, 0, -1):
        j = next(g) % (i + 1)
        p[i], p[j] = p[j], p[i]
    return np.asarray(p, np.int64)


def split_merge(Y, perm, offsets, K_local, s_local, K, iters_local, iters_merge, s_merge, s_final,
                tau=TAU, dep_tol=DEP_TOL, codes=True, merge_seed=0):
    """Algorithm 1 end to end.  Returns (D, codes, D_local (sumK, m), scales (L,)).  With a
    nonzero merge_seed the merge learns on the pooled columns in the order of
    seeded_permutation(sum K_local, merge_seed), so that it starts from its first K of them."""
    Y = _d(Y)
    N, m = Y.shape
    perm = np.ascontiguousarray(perm, np.int64)
    offsets = np.ascontiguousarray(offsets, np.int64)
    K_local = np.ascontiguousarray(K_local, np.int32)
    s_local = np.ascontiguousarray(s_local, np.int32)
    L = len(K_local)
    D = np.empty((K, m))
    Dl = np.empty((int(K_local.sum()), m))
    sc = np.empty(L)
    idx = np.empty((N, s_final), np.int32) if codes else None
    coef = np.empty((N, s_final)) if codes else None
    nnz = np.empty(N, np.int32) if codes else None
    rc = lib().ora_split_merge(_p(Y, C.c_double), m, N, _p(perm, C.c_int64), L, _p(offsets, C.c_int64),
                               _p(K_local, C.c_int32), _p(s_local, C.c_int32), K, iters_local,
                               iters_merge, s_merge, s_final, tau, dep_tol, _p(D, C.c_double),
                               _p(idx, C.c_int32), _p(coef, C.c_double), _p(nnz, C.c_int32),
                               _p(Dl, C.c_double), _p(sc, C.c_double),
                               _p(mp, C.c_int64) if (mp := (seeded_permutation(int(K_local.sum()), merge_seed)
                                                            if merge_seed else None)) is not None else None)
    if rc != 0:
        raise FloatingPointError(f"oracle split-merge failed ({rc})")
    return D, (Codes(idx, coef, nnz) if codes else None), Dl, sc


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(lib().ora_threads())


def set_threads(n: int) -> None:
    """Run the oracle's loops on n threads (for timing)."""
    lib().ora_set_threads(int(n))


def set_bf16_rounding(enabled: bool) -> None:
    """Switch the oracle's BF16 rounding points on (default) or off (exact FP64 network)."""
    lib().ora_set_bf16(1 if enabled else 0)


def bf16(x):
    x = np.asarray(x, np.float64)
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    r = np.where(special, u & 0xFFFF0000, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _mlp_args(Ws, bs):
    widths = [Ws[0].shape[1]] + [W.shape[0] for W in Ws]
    Wd = [_d(W) for W in Ws]
    bd = [_d(b) for b in bs]
    WP = (C.POINTER(C.c_double) * len(Wd))(*[_p(W, C.c_double) for W in Wd])
    BP = (C.POINTER(C.c_double) * len(bd))(*[_p(b, C.c_double) for b in bd])
    wa = (C.c_int * len(widths))(*widths)
    return widths, Wd, bd, WP, BP, wa


def mlp_forward(Ws, bs, X):
    widths, Wd, bd, WP, BP, wa = _mlp_args(Ws, bs)
    X = _d(X)
    B = X.shape[0]
    out = np.empty((B, widths[-1]))
    rc = lib().ora_mlp_forward(len(Ws), wa, WP, BP, _p(X, C.c_double), B, _p(out, C.c_double))
    assert rc == 0
    return out


def mlp_grad(Ws, bs, X, T):
    """Loss and gradients (dW list, db list) of the mean BCE-with-logits."""
    widths, Wd, bd, WP, BP, wa = _mlp_args(Ws, bs)
    X, T = _d(X), _d(T)
    B = X.shape[0]
    dW = [np.empty_like(W) for W in Wd]
    db = [np.empty_like(b) for b in bd]
    GW = (C.POINTER(C.c_double) * len(dW))(*[_p(g, C.c_double) for g in dW])
    GB = (C.POINTER(C.c_double) * len(db))(*[_p(g, C.c_double) for g in db])
    loss = C.c_double(0)
    rc = lib().ora_mlp_grad(len(Ws), wa, WP, BP, _p(X, C.c_double), _p(T, C.c_double), B,
                            C.byref(loss), GW, GB)
    assert rc == 0
    return loss.value, dW, db


def adam(w, g, mom, vel, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (w, g, mom, vel):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().ora_adam(_p(w, C.c_double), _p(g, C.c_double), _p(mom, C.c_double), _p(vel, C.c_double),
                   w.size, t, lr, beta1, beta2, eps)


def propose_code(D, Y, logits, n_cand, s_max, eps_fallback, tau=TAU, dep_tol=DEP_TOL):
    D, Y, lg = _d(D), _d(Y), _d(logits)
    K, m = D.shape
    N = Y.shape[0]
    idx = np.empty((N, s_max), np.int32)
    coef = np.empty((N, s_max))
    nnz = np.empty(N, np.int32)
    fb = np.empty(N, np.uint8)
    cand = np.empty((N, n_cand), np.int32)
    rc = lib().ora_propose_code(_p(D, C.c_double), m, K, _p(Y, C.c_double), N, _p(lg, C.c_double),
                                n_cand, s_max, eps_fallback, tau, dep_tol, _p(idx, C.c_int32),
                                _p(coef, C.c_double), _p(nnz, C.c_int32), _p(fb, C.c_uint8),
                                _p(cand, C.c_int32))
    assert rc == 0
    out = Codes(idx, coef, nnz)
    out.fell_back = fb
    out.cand = cand
    return out


def multi_hot(codes: Codes, K: int) -> np.ndarray:
    """Training targets of the proposer: t[n, k] = 1 iff atom k is in the support of signal n."""
    N, s = codes.idx.shape
    T = np.zeros((N, K))
    for i in range(s):
        ok = i < codes.nnz
        T[np.nonzero(ok)[0], codes.idx[ok, i]] = 1.0
    return T


def compose_codes(X1: Codes, offsets, K_local, Z: Codes, scales, K: int, perm=None) -> np.ndarray:
    """Proposition 1 (proof in Appendix A) on Algorithm 1's codes, written out densely in FP64:
    y ~ Dtilde x1 with Dtilde = [c_1 D^(1), ..., c_L D^(L)] and Dtilde ~ D Z give y ~ D (Z x1).
    X1 holds each signal's code over its unscaled local dictionary D^(t) (rows in split order,
    local atom ids), so over Dtilde the code is x1 / c_t.  Z holds the codes of the pooled
    columns over D.  Returns R (N x K): row perm[p] = Z (x1_p / c_t) for position p of subset t."""
    offsets = np.asarray(offsets, np.int64)
    K_local = np.asarray(K_local, np.int64)
    aoff = np.concatenate([[0], np.cumsum(K_local)])
    N = int(offsets[-1])
    Zd = Z.dense(K)                                   # (sum K_local, K): row a = z_a
    R = np.zeros((N, K))
    for t in range(len(K_local)):
        if not scales[t] > 0:
            continue
        for p in range(int(offsets[t]), int(offsets[t + 1])):
            x = np.zeros(int(K_local[t]))
            for i in range(int(X1.nnz[p])):
                x[X1.idx[p, i]] += X1.coef[p, i]
            r = (x / scales[t]) @ Zd[aoff[t]:aoff[t + 1]]
            R[perm[p] if perm is not None else p] = r
    return R


def denoise(img, D, p: int, eps: float, s_max: int):
    """Section 3.2.2 written out: every p x p patch of the image (stride 1 in both directions) is
    coded by the error-constrained OMP (||y - D x||_2 <= eps) against D, and every pixel of the
    output is the mean of the estimates D x of the patches that cover it.  FP64 throughout.
    Returns (image, codes of the patches in row-major patch order)."""
    img = np.asarray(img, np.float64)
    D = _d(D)
    H, W = img.shape
    PH, PW = H - p + 1, W - p + 1
    patches = np.empty((PH * PW, p * p))
    for pi in range(PH):
        for pj in range(PW):
            patches[pi * PW + pj] = img[pi:pi + p, pj:pj + p].ravel()
    codes = omp(D, patches, s_max, eps)
    est = codes.dense(D.shape[0]) @ D
    acc = np.zeros((H, W))
    cnt = np.zeros((H, W))
    for pi in range(PH):
        for pj in range(PW):
            acc[pi:pi + p, pj:pj + p] += est[pi * PW + pj].reshape(p, p)
            cnt[pi:pi + p, pj:pj + p] += 1.0
    return acc / cnt, codes


def tie_mask(codes: Codes, eps: float = 0.0, margin: float = 1e-5, tau: float = TAU,
             dep_tol: float = DEP_TOL) -> np.ndarray:
    """Signals whose FP64 trace comes close to a decision boundary (excluded from
    support comparisons): a correlation near-tie (relative top-2 gap < margin) at a step that
    goes on to pick an atom (best correlation above tau: below it the loop stops whatever the
    gap), a best correlation within a factor 2 of the tau stop, a dependence ratio within a
    factor 5 of dep_tol, or (error-constrained form) a residual within margin*||y|| of eps."""
    gap, cmax, l2, rn = codes.gap, codes.cmax, codes.l2, codes.rn
    with np.errstate(invalid="ignore"):
        t = np.nan_to_num((gap < margin) & (cmax > tau), nan=False).any(axis=1)
        t |= np.nan_to_num((cmax > 0.5 * tau) & (cmax < 2 * tau), nan=False).any(axis=1)
        t |= np.nan_to_num((l2 > 0.2 * dep_tol) & (l2 < 5 * dep_tol), nan=False).any(axis=1)
        if eps > 0:
            yn = rn[:, 0]
            t |= np.nan_to_num(np.abs(rn - eps) < margin * np.maximum(yn, 1e-30)[:, None], nan=False).any(axis=1)
    return t
