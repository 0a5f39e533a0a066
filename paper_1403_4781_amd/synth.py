"""Seeded synthetic inputs for the split-and-merge dictionary-learning workloads.

This module only draws random numbers: generating dictionaries, sparse codes,
noise, the random split of the training set and the seeded orders that the
method consumes.  It contains none of the method's arithmetic (no sparse
coding, no dictionary update), so the FP64 oracle and the HIP path can both
take their inputs from it without sharing any computation.

Memory convention (shared with the C ABI): a matrix with ``r`` rows stored
column-major is a NumPy array of shape ``(cols, r)``, C-contiguous.  So the
training matrix Y (m x N, one signal per column, as in the problem statement of
Section 2) is an array of shape ``(N, m)`` whose row ``n`` is signal ``y_n``, and a
dictionary D (m x K) is an array of shape ``(K, m)`` whose row ``k`` is atom ``d_k``.

The generative model follows the synthetic experiment of Section 3.1: Gaussian
atoms normalised to unit length, signals formed from ``s0`` atoms drawn uniformly
without replacement with N(0, 1) weights, plus white Gaussian noise of standard
deviation ``sigma`` (the noise term is stated by the workload definitions, the
paper's own synthetic experiment is noise-free).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 14034780

# Named sub-streams spawned from one SeedSequence per workload.
STREAM_D0, STREAM_SIGNALS, STREAM_SPLIT, STREAM_SUBSET_INIT, STREAM_MERGE_INIT, \
    STREAM_MLP_INIT, STREAM_TRAIN, STREAM_EVAL = range(8)


def rng_streams(seed: int, n: int = 8) -> list[np.random.Generator]:
    """``n`` independent generators spawned from ``SeedSequence(seed)``."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def gaussian_dictionary(rng: np.random.Generator, m: int, K: int) -> np.ndarray:
    """K atoms of dimension m with i.i.d. N(0,1) entries, scaled to unit l2 norm.

    Returned as shape (K, m), float64 (atom k is row k).
    """
    A = rng.standard_normal((K, m))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A


def sparse_signals(rng: np.random.Generator, D0: np.ndarray, s0: int, sigma: float,
                   N: int, block: int = 65536):
    """Draw N signals y = D0 x + n with ||x||_0 = s0.

    The support of each signal is a uniform random s0-subset of the K0 atoms
    (the first s0 entries of a random ordering), the nonzero weights are N(0,1)
    and the noise is N(0, sigma^2) per entry.  Returns ``(Y, support, weights)``
    with Y of shape (N, m) float32 and support/weights of shape (N, s0).
    """
    K0, m = D0.shape
    Y = np.empty((N, m), dtype=np.float32)
    sup = np.empty((N, s0), dtype=np.int32)
    val = np.empty((N, s0), dtype=np.float64)
    for b0 in range(0, N, block):
        B = min(block, N - b0)
        # the first s0 of a random ordering: the s0 smallest of K0 uniforms, in increasing order
        # (selected by a partition, then sorted among themselves)
        r = rng.random((B, K0))
        part = np.argpartition(r, s0 - 1, axis=1)[:, :s0] if s0 < K0 else np.argsort(r, axis=1)
        order = np.take_along_axis(part, np.argsort(np.take_along_axis(r, part, axis=1), axis=1), axis=1)
        w = rng.standard_normal((B, s0))
        noise = rng.standard_normal((B, m))
        # y_n = sum_i w_i d_{order_i} + sigma * noise  (generation only)
        y = np.einsum('bi,bim->bm', w, D0[order]) + sigma * noise
        Y[b0:b0 + B] = y.astype(np.float32)
        sup[b0:b0 + B] = order
        val[b0:b0 + B] = w
    return Y, sup, val


def random_partition(rng: np.random.Generator, N: int, sizes) -> tuple[np.ndarray, np.ndarray]:
    """Random disjoint split of N signals into subsets of the given sizes.

    Returns ``(perm, offsets)``: subset t holds signals ``perm[offsets[t]:offsets[t+1]]``.
    This is the random draw of step 1 of Algorithm 1; the method receives it as input.
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    assert sizes.sum() == N
    perm = rng.permutation(N).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return perm, offsets


def equal_sizes(N: int, L: int) -> np.ndarray:
    base = N // L
    sizes = np.full(L, base, dtype=np.int64)
    sizes[: N - base * L] += 1
    return sizes


def uneven_sizes(rng: np.random.Generator, L: int, lo: int, hi: int, total: int | None = None) -> np.ndarray:
    """L subset sizes uniform in [lo, hi]; optionally rescaled to sum exactly to ``total``."""
    sizes = rng.integers(lo, hi + 1, size=L).astype(np.int64)
    if total is not None:
        scaled = np.floor(sizes * (total / sizes.sum())).astype(np.int64)
        scaled[: total - scaled.sum()] += 1
        sizes = scaled
    return sizes


@dataclass
class Workload:
    """A fully drawn synthetic workload (all arrays are NumPy)."""
    name: str
    m: int
    K: int
    Y: np.ndarray                 # (N, m) float32
    D0: np.ndarray                # (K0, m) float64 generating dictionary
    support: np.ndarray
    perm: np.ndarray              # int64[N]
    offsets: np.ndarray           # int64[L+1]
    K_local: np.ndarray           # int32[L]
    s_local: np.ndarray           # int32[L]
    iters_local: int
    iters_merge: int
    s_merge: int
    s_final: int
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.Y.shape[0]

    @property
    def L(self) -> int:
        return len(self.offsets) - 1


def make_workload(name: str, *, seed: int, m: int, K0: int, s0: int, sigma: float, N: int,
                  sizes, K_local, s_local, K: int, iters_local: int, iters_merge: int,
                  s_merge: int, s_final: int) -> Workload:
    g = rng_streams(seed)
    D0 = gaussian_dictionary(g[STREAM_D0], m, K0)
    Y, sup, _ = sparse_signals(g[STREAM_SIGNALS], D0, s0, sigma, N)
    perm, offsets = random_partition(g[STREAM_SPLIT], N, sizes)
    L = len(sizes)
    K_local = np.broadcast_to(np.asarray(K_local, dtype=np.int32), (L,)).copy()
    s_local = np.broadcast_to(np.asarray(s_local, dtype=np.int32), (L,)).copy()
    return Workload(name, m, K, Y, D0, sup, perm, offsets, K_local, s_local,
                    iters_local, iters_merge, s_merge, s_final)


# --- the five workload definitions -------------------------------------------------------

def oracle_scale(N: int = 2000) -> Workload:
    """m=64, K=128, s=5, sigma=0.01, N=2000, one dictionary (L=1), 10 iterations.

    The initial dictionary is 128 signals in a seeded random order (the split
    permutation with L=1 doubles as that order)."""
    return make_workload("oracle_scale_m64_K128_s5", seed=SEED_BASE + 1, m=64, K0=128, s0=5,
                         sigma=0.01, N=N, sizes=[N], K_local=128, s_local=5, K=128,
                         iters_local=10, iters_merge=0, s_merge=5, s_final=5)


def patch_scale(N: int = 100000, L: int = 20, iters: int = 20) -> Workload:
    """Split-and-merge at 8x8-patch scale: m=64, K=256, s=8, sigma=0.02, N=1e5,
    20 equal subsets of 5000 with local K=256, s=8; merge 5120 pooled atoms to
    K=256 with s=4; final coding of all N at s=8."""
    return make_workload("split_merge_m64_K256_s8_N100000", seed=SEED_BASE + 2, m=64, K0=256, s0=8,
                         sigma=0.02, N=N, sizes=equal_sizes(N, L), K_local=256, s_local=8, K=256,
                         iters_local=iters, iters_merge=iters, s_merge=4, s_final=8)


def batched_split(L: int = 64, lo: int = 1000, hi: int = 20000, iters: int = 20) -> Workload:
    """64 subsets, sizes uniform in [1000, 20000], local K in {64,128,192,256},
    s in {4,8,12}, m=64; data from the patch-scale generative model."""
    g = rng_streams(SEED_BASE + 3)
    sizes = uneven_sizes(g[STREAM_SPLIT], L, lo, hi)
    K_local = g[STREAM_SPLIT].choice([64, 128, 192, 256], size=L).astype(np.int32)
    s_local = g[STREAM_SPLIT].choice([4, 8, 12], size=L).astype(np.int32)
    N = int(sizes.sum())
    return make_workload("batched_split_m64_L64", seed=SEED_BASE + 3, m=64, K0=256, s0=8, sigma=0.02,
                         N=N, sizes=sizes, K_local=K_local, s_local=s_local, K=256,
                         iters_local=iters, iters_merge=iters, s_merge=4, s_final=8)


def large_scale(N: int = 1000000, L: int = 100, iters: int = 20) -> Workload:
    """m=256 (16x16 patches), K=1024, s=16, sigma=0.02, N=1e6 in 100 uneven subsets
    (sizes uniform in [5000, 15000], rescaled to sum to N); local K=512, s=16;
    merge to K=1024 with s=8; final s=16."""
    g = rng_streams(SEED_BASE + 5)
    sizes = uneven_sizes(g[STREAM_SPLIT], L, 5000, 15000, total=N)
    return make_workload("large_m256_K1024_s16", seed=SEED_BASE + 5, m=256, K0=1024, s0=16,
                         sigma=0.02, N=N, sizes=sizes, K_local=512, s_local=16, K=1024,
                         iters_local=iters, iters_merge=iters, s_merge=8, s_final=16)


def synthetic_e1(trial: int, iters: int = 100, N: int = 40000) -> Workload:
    """The paper's synthetic experiment (Section 3.1, Table 1), trial ``trial``: a 30 x 60 Gaussian
    dictionary with unit atoms, N = 4 x 10^4 noise-free signals of 6 atoms with N(0, 1) weights;
    split-and-merge with L = 40 subsets of 1000, local K_1 = 50 at s_1 = 3, merged to K = 60 at
    s_2 = 2, and the final coding at s = 6.  The standard approach learns K = 60 at s = 6 from the
    first 60 training vectors.  The paper does not state the iteration count; ``iters`` serves
    every learning stage."""
    return make_workload(f"e1_trial{trial}", seed=SEED_BASE + 100 + trial, m=30, K0=60, s0=6, sigma=0.0,
                         N=N, sizes=equal_sizes(N, 40), K_local=50, s_local=3, K=60,
                         iters_local=iters, iters_merge=iters, s_merge=2, s_final=6)


def odct(p: int, kh: int, kw: int) -> np.ndarray:
    """Overcomplete two-dimensional DCT for p x p patches (the initial dictionary of Section
    3.2.1): the Kronecker product of two one-dimensional overcomplete cosine sets of kh and kw
    atoms of length p (atom k: cos(pi n k / k_total), n = 0 .. p-1; the mean removed from every
    atom but the first; unit length).  Shape (kh * kw, p * p), float64; atom u kw + v has pixel
    (r, c) at index r p + c equal to C_kh[r, u] C_kw[c, v]."""
    def one(k):
        C = np.cos(np.outer(np.arange(p), np.arange(k)) * np.pi / k)
        C[:, 1:] -= C[:, 1:].mean(axis=0)
        return C / np.linalg.norm(C, axis=0)
    return np.kron(one(kh), one(kw)).T.copy()


def synthetic_image(rng: np.random.Generator, H: int = 256, W: int = 256) -> np.ndarray:
    """A seeded piecewise-smooth grey-level image in [0, 255] (a stand-in for the natural images
    of Section 3.2, which are not available): a smooth background of a few low-frequency cosines,
    ellipses and rectangles of constant offsets (sharp edges) and one striped texture patch."""
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((H, W), 110.0)
    for _ in range(4):
        fy, fx = rng.uniform(0.2, 2.0, 2) * np.pi / np.array([H, W])
        img += rng.uniform(10, 30) * np.cos(fy * y + fx * x + rng.uniform(0, 2 * np.pi))
    for _ in range(8):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        ry, rx = rng.uniform(H / 16, H / 4), rng.uniform(W / 16, W / 4)
        img[((y - cy) / ry) ** 2 + ((x - cx) / rx) ** 2 <= 1.0] += rng.uniform(-60, 60)
    for _ in range(6):
        y0, x0 = rng.integers(0, H - 8), rng.integers(0, W - 8)
        y1, x1 = y0 + rng.integers(8, H // 3), x0 + rng.integers(8, W // 3)
        img[y0:y1, x0:x1] += rng.uniform(-50, 50)
    y0, x0 = rng.integers(0, H // 2), rng.integers(0, W // 2)
    per = rng.uniform(4, 12)
    img[y0:y0 + H // 4, x0:x0 + W // 4] += 25 * np.sign(np.sin(2 * np.pi * x[y0:y0 + H // 4, x0:x0 + W // 4] / per))
    return np.clip(img, 0.0, 255.0)


def image_patches(rng: np.random.Generator, images, n: int, p: int) -> np.ndarray:
    """n random p x p patches (rows, pixel (r, c) at r p + c) of the given images, float32."""
    out = np.empty((n, p * p), dtype=np.float32)
    which = rng.integers(0, len(images), n)
    for i in range(n):
        im = images[which[i]]
        r, c = rng.integers(0, im.shape[0] - p + 1), rng.integers(0, im.shape[1] - p + 1)
        out[i] = im[r:r + p, c:c + p].ravel()
    return out


def fresh_signals(w: Workload, stream: int, N: int, s0: int, sigma: float) -> np.ndarray:
    """Fresh signals from the same generating dictionary as workload ``w``
    (training pairs use STREAM_TRAIN, evaluation signals STREAM_EVAL)."""
    seed = {"oracle_scale_m64_K128_s5": 1, "split_merge_m64_K256_s8_N100000": 2,
            "batched_split_m64_L64": 3, "large_m256_K1024_s16": 5}.get(w.name, 9)
    g = rng_streams(SEED_BASE + seed)
    Y, _, _ = sparse_signals(g[stream], w.D0, s0, sigma, N)
    return Y


def mlp_init(widths, seed: int = SEED_BASE + 4):
    """Kaiming-uniform weights (out x in, row-major) and uniform biases for an MLP,
    as float32 arrays: the seeded initial state of the support proposer."""
    g = rng_streams(seed)[STREAM_MLP_INIT]
    Ws, bs = [], []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        bound = np.sqrt(6.0 / fan_in)
        Ws.append(g.uniform(-bound, bound, size=(fan_out, fan_in)).astype(np.float32))
        bb = 1.0 / np.sqrt(fan_in)
        bs.append(g.uniform(-bb, bb, size=(fan_out,)).astype(np.float32))
    return Ws, bs


def small_problem(seed: int, m: int, K: int, s0: int, sigma: float, N: int):
    """A small random instance: (D (K, m) float32 unit atoms, Y (N, m) float32)."""
    g = rng_streams(seed)
    D0 = gaussian_dictionary(g[STREAM_D0], m, K)
    Y, sup, val = sparse_signals(g[STREAM_SIGNALS], D0, s0, sigma, N)
    return D0.astype(np.float32), Y, sup
