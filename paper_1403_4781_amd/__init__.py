"""Split-and-merge dictionary learning on MI355X (gfx950): Python binding of libsmdl.

Thin ctypes layer over the C ABI declared in ``include/smdl.h``: it checks tensor
shapes/devices, marshals pointers and sizes, and returns torch tensors.  Every step of
the computation runs in the library's HIP kernels; there is no fallback.  The library is
loaded on first use (``lib()``, or creating a :class:`Handle`), which raises if
``libsmdl.so`` is missing.

Conventions: signals ``Y`` are a CUDA float32 tensor of shape (N, m) (row n = signal n,
i.e. the column-major m x N matrix of the paper's problem statement), a dictionary ``D``
has shape (K, m) (row k = atom k).  Sparse codes are :class:`Codes` (ELL layout).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

__all__ = ["Handle", "Codes", "Proposer", "SmdlError", "LIB_PATH", "lib"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsmdl.so")

SMDL_PER_SUBSET_LAUNCH = 1
SMDL_NO_GRAPH = 2
SMDL_COMPOSE_CODES = 4
SMDL_DETERMINISTIC = 8
SMDL_CHECK_FINITE = 16
SMDL_ASYNC = 32

_STATUS = {0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_UNSUPPORTED", -4: "E_NOMEM", -5: "E_HIP",
           -6: "E_NUMERIC", -7: "E_STATE"}


class SmdlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"smdl {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Codes(C.Structure):
    _fields_ = [("idx", C.c_void_p), ("coef", C.c_void_p), ("nnz", C.c_void_p), ("s_max", C.c_int32)]


class _Subsets(C.Structure):
    _fields_ = [("L", C.c_int), ("perm", C.c_void_p), ("offsets", C.POINTER(C.c_int64)),
                ("K_local", C.POINTER(C.c_int32)), ("s_local", C.POINTER(C.c_int32))]


class _LearnOpts(C.Structure):
    _fields_ = [("iters_local", C.c_int), ("iters_merge", C.c_int), ("s_merge", C.c_int),
                ("s_final", C.c_int), ("flags", C.c_uint32), ("D_local_init", C.c_void_p),
                ("D_merge_init", C.c_void_p), ("merge_seed", C.c_uint64), ("X_local", _Codes)]


class _TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("shuffle_seed", C.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1403_4781_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32 = C.c_void_p, C.c_int, C.c_int64, C.c_float
    sigs = {
        "smdl_create": [C.POINTER(vp), i32, vp],
        "smdl_destroy": [vp],
        "smdl_last_error": [vp],
        "smdl_version": [],
        "smdl_gram": [vp, vp, i32, i32, vp],
        "smdl_omp_code": [vp, vp, i32, i32, vp, i64, i32, f32, _Codes, vp],
        "smdl_omp_code_noalloc": [vp, vp, i32, i32, vp, i64, i32, f32, _Codes, vp],
        "smdl_mod_update": [vp, vp, i32, i64, _Codes, i32, vp, C.POINTER(C.c_int32)],
        "smdl_learn": [vp, vp, i32, i64, i32, i32, i32, vp, _Codes],
        "smdl_learn_init": [vp, vp, i32, i64, i32, i32, i32, vp, vp, _Codes],
        "smdl_split_merge_learn": [vp, vp, i32, i64, C.POINTER(_Subsets), i32, C.POINTER(_LearnOpts), vp,
                                   _Codes, vp, C.POINTER(C.c_double)],
        "smdl_compose_codes": [vp, i64, C.POINTER(_Subsets), _Codes, _Codes, i32, C.POINTER(C.c_double), _Codes],
        "smdl_denoise": [vp, vp, i32, i32, i32, vp, i32, f32, i32, vp],
        "smdl_prop_create": [vp, i32, C.POINTER(C.c_int), C.POINTER(C.POINTER(C.c_float)),
                             C.POINTER(C.POINTER(C.c_float)), C.POINTER(vp)],
        "smdl_prop_destroy": [vp],
        "smdl_prop_get": [vp, vp, C.POINTER(C.POINTER(C.c_float)), C.POINTER(C.POINTER(C.c_float))],
        "smdl_prop_create_seeded": [vp, i32, C.POINTER(C.c_int), C.c_uint64, C.POINTER(vp)],
        "smdl_prop_set": [vp, vp, C.POINTER(C.POINTER(C.c_float)), C.POINTER(C.POINTER(C.c_float))],
        "smdl_prop_logits": [vp, vp, vp, i64, vp],
        "smdl_prop_grad": [vp, vp, vp, i64, _Codes, C.POINTER(C.c_float), C.POINTER(vp), C.POINTER(vp)],
        "smdl_prop_train": [vp, vp, vp, i64, _Codes, C.POINTER(_TrainOpts), C.POINTER(C.c_float)],
        "smdl_omp_code_proposed": [vp, vp, vp, i32, i32, vp, i64, i32, i32, f32, _Codes, vp,
                                   C.POINTER(C.c_int64), vp],
        "smdl_prop_phase_ms": [vp, C.POINTER(C.c_float)],
        "smdl_tune": [vp, vp, i32, i32, vp, i64, i32],
        "smdl_get_tile": [vp, i32, i32, i32, C.POINTER(C.c_int), C.POINTER(C.c_int)],
        "smdl_set_tile": [vp, i32, i32, i32, i32],
        "smdl_set_mod_solver": [vp, i32],
        "smdl_set_autotune": [vp, i32],
        "smdl_set_flags": [vp, C.c_uint32],
        "smdl_phase_ms": [vp, C.POINTER(C.c_float)],
        "smdl_last_kernel_ms": [vp, C.POINTER(C.c_float)],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.smdl_last_error.restype = C.c_char_p
    L.smdl_destroy.restype = None
    return L


_LIB = None


def lib():
    """The loaded libsmdl (ctypes.CDLL); raises ImportError if it is not built."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev_tensor(t, dtype, name, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


@dataclass
class Codes:
    """ELL sparse codes: idx (N, s) int32, coef (N, s) float32, nnz (N,) int32 (device)."""
    idx: torch.Tensor
    coef: torch.Tensor
    nnz: torch.Tensor

    @staticmethod
    def empty(N: int, s: int, device) -> "Codes":
        return Codes(torch.empty((N, s), dtype=torch.int32, device=device),
                     torch.empty((N, s), dtype=torch.float32, device=device),
                     torch.empty((N,), dtype=torch.int32, device=device))

    @property
    def s_max(self) -> int:
        return self.idx.shape[1]

    def _c(self) -> _Codes:
        return _Codes(self.idx.data_ptr(), self.coef.data_ptr(), self.nnz.data_ptr(), self.s_max)

    def dense(self, K: int) -> torch.Tensor:
        """Dense (N, K) code matrix (row n = x_n)."""
        N, s = self.idx.shape
        X = torch.zeros((N, K), dtype=torch.float32, device=self.idx.device)
        ok = torch.arange(s, device=self.idx.device)[None, :] < self.nnz[:, None]
        rows = torch.arange(N, device=self.idx.device)[:, None].expand(N, s)
        X[rows[ok], self.idx[ok].long()] = self.coef[ok]
        return X


class Handle:
    """A library handle bound to one GPU (its own HIP stream)."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p(0)
        self.device = torch.device("cuda", device)
        L = lib()
        torch.cuda.init()
        st = L.smdl_create(C.byref(self._h), device, None)
        if st != 0:
            raise SmdlError(st, "smdl_create failed")

    def close(self):
        if self._h:
            lib().smdl_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise SmdlError(st, lib().smdl_last_error(self._h).decode())

    # ---- coding ---------------------------------------------------------------------
    def gram(self, D: torch.Tensor) -> torch.Tensor:
        K, m = D.shape
        _dev_tensor(D, torch.float32, "D")
        G = torch.empty((K, K), dtype=torch.float32, device=D.device)
        self._check(lib().smdl_gram(self._h, _ptr(D), m, K, _ptr(G)))
        return G

    def omp_code(self, D: torch.Tensor, Y: torch.Tensor, s_max: int, eps: float = 0.0,
                 out: Codes | None = None, res_norm: bool = False):
        K, m = D.shape
        _dev_tensor(D, torch.float32, "D")
        _dev_tensor(Y, torch.float32, "Y")
        if Y.dim() != 2 or Y.shape[1] != m:
            raise ValueError("Y must have shape (N, m)")
        N = Y.shape[0]
        X = out if out is not None else Codes.empty(N, s_max, Y.device)
        r = torch.empty((N,), dtype=torch.float32, device=Y.device) if res_norm else None
        self._check(lib().smdl_omp_code(self._h, _ptr(D), m, K, _ptr(Y), N, s_max, float(eps), X._c(), _ptr(r)))
        return (X, r) if res_norm else X

    def last_kernel_ms(self) -> float:
        v = C.c_float(0)
        self._check(lib().smdl_last_kernel_ms(self._h, C.byref(v)))
        return v.value

    # ---- dictionary update ------------------------------------------------------------
    def mod_update(self, Y: torch.Tensor, X: Codes, D: torch.Tensor) -> int:
        """MOD update of D in place; returns the number of unused atoms."""
        K, m = D.shape
        _dev_tensor(D, torch.float32, "D")
        _dev_tensor(Y, torch.float32, "Y")
        N = Y.shape[0]
        nu = C.c_int32(0)
        self._check(lib().smdl_mod_update(self._h, _ptr(Y), m, N, X._c(), K, _ptr(D), C.byref(nu)))
        return nu.value

    # ---- learning -------------------------------------------------------------------
    def learn(self, Y: torch.Tensor, K: int, s: int, iters: int, codes: bool = True,
              D_init: torch.Tensor | None = None):
        """The standard alternation; from the first K signals, or from D_init (K, m) when given."""
        _dev_tensor(Y, torch.float32, "Y")
        N, m = Y.shape
        D = torch.empty((K, m), dtype=torch.float32, device=Y.device)
        X = Codes.empty(N, s, Y.device) if codes else None
        xc = X._c() if X is not None else _Codes(None, None, None, s)
        if D_init is None:
            self._check(lib().smdl_learn(self._h, _ptr(Y), m, N, K, s, iters, _ptr(D), xc))
        else:
            _dev_tensor(D_init, torch.float32, "D_init", (K, m))
            self._check(lib().smdl_learn_init(self._h, _ptr(Y), m, N, K, s, iters, _ptr(D_init), _ptr(D), xc))
        return D, X

    def split_merge_learn(self, Y: torch.Tensor, perm: torch.Tensor | None, offsets, K_local, s_local,
                          K: int, iters_local: int, iters_merge: int, s_merge: int, s_final: int,
                          flags: int = 0, codes: bool = True, local: bool = False,
                          D_local_init: torch.Tensor | None = None, D_merge_init: torch.Tensor | None = None,
                          merge_seed: int = 0, X_local: "Codes | None" = None):
        """Algorithm 1.  Returns (D, codes or None, D_local or None, scales (np.float64[L])).
        D_local_init (max K_local, m) and D_merge_init (K, m) replace the first-columns starts;
        merge_seed != 0 starts the merge from a seeded permutation of the pooled columns;
        X_local (N rows, s >= max s_local) receives the final local codes in split order."""
        _dev_tensor(Y, torch.float32, "Y")
        N, m = Y.shape
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        K_local = np.ascontiguousarray(K_local, dtype=np.int32)
        s_local = np.ascontiguousarray(s_local, dtype=np.int32)
        L = len(K_local)
        if perm is not None:
            _dev_tensor(perm, torch.int64, "perm", (N,))
        sub = _Subsets(L, _ptr(perm).value if perm is not None else None,
                       offsets.ctypes.data_as(C.POINTER(C.c_int64)),
                       K_local.ctypes.data_as(C.POINTER(C.c_int32)),
                       s_local.ctypes.data_as(C.POINTER(C.c_int32)))
        if D_local_init is not None:
            _dev_tensor(D_local_init, torch.float32, "D_local_init", (int(K_local.max()), m))
        if D_merge_init is not None:
            _dev_tensor(D_merge_init, torch.float32, "D_merge_init", (K, m))
        if X_local is not None:
            for t_, nm in ((X_local.idx, "X_local.idx"), (X_local.coef, "X_local.coef"), (X_local.nnz, "X_local.nnz")):
                _dev_tensor(t_, t_.dtype, nm)
            if X_local.idx.shape[0] != N:
                raise ValueError("X_local must have N rows")
        opts = _LearnOpts(iters_local, iters_merge, s_merge, s_final, flags,
                          _ptr(D_local_init).value if D_local_init is not None else None,
                          _ptr(D_merge_init).value if D_merge_init is not None else None,
                          int(merge_seed), X_local._c() if X_local is not None else _Codes(None, None, None, 0))
        D = torch.empty((K, m), dtype=torch.float32, device=Y.device)
        s_out = int(s_local.max()) * s_merge if flags & SMDL_COMPOSE_CODES else s_final
        X = Codes.empty(N, s_out, Y.device) if codes else None
        xc = X._c() if X is not None else _Codes(None, None, None, s_out)
        Dl = torch.empty((int(K_local.sum()), m), dtype=torch.float32, device=Y.device) if local else None
        scales = np.zeros(L, dtype=np.float64)
        self._check(lib().smdl_split_merge_learn(self._h, _ptr(Y), m, N, C.byref(sub), K, C.byref(opts), _ptr(D),
                                               xc, _ptr(Dl), scales.ctypes.data_as(C.POINTER(C.c_double))))
        return D, X, Dl, scales

    def compose_codes(self, X1: "Codes", Z: "Codes", offsets, K_local, K: int, scales, perm: torch.Tensor | None = None):
        """Proposition 1 composition (see smdl_compose_codes): codes over D with at most
        X1.s * Z.s atoms per signal."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        K_local = np.ascontiguousarray(K_local, dtype=np.int32)
        scales = np.ascontiguousarray(scales, dtype=np.float64)
        L = len(K_local)
        N = int(offsets[-1])
        if perm is not None:
            _dev_tensor(perm, torch.int64, "perm", (N,))
        s_l = np.zeros(L, np.int32)
        sub = _Subsets(L, _ptr(perm).value if perm is not None else None,
                       offsets.ctypes.data_as(C.POINTER(C.c_int64)), K_local.ctypes.data_as(C.POINTER(C.c_int32)),
                       s_l.ctypes.data_as(C.POINTER(C.c_int32)))
        X = Codes.empty(N, X1.idx.shape[1] * Z.idx.shape[1], X1.idx.device)
        self._check(lib().smdl_compose_codes(self._h, N, C.byref(sub), X1._c(), Z._c(), K,
                                             scales.ctypes.data_as(C.POINTER(C.c_double)), X._c()))
        return X

    def denoise(self, img: torch.Tensor, D: torch.Tensor, p: int, eps: float, s_max: int) -> torch.Tensor:
        """Section 3.2.2: error-constrained OMP of every p x p patch, overlapping estimates averaged."""
        _dev_tensor(img, torch.float32, "img")
        H, W = img.shape
        K = D.shape[0]
        _dev_tensor(D, torch.float32, "D", (K, p * p))
        out = torch.empty_like(img)
        self._check(lib().smdl_denoise(self._h, _ptr(img), H, W, p, _ptr(D), K, float(eps), s_max, _ptr(out)))
        return out

    def phase_ms(self):
        v = (C.c_float * 3)()
        self._check(lib().smdl_phase_ms(self._h, v))
        return list(v)

    # ---- tuning ---------------------------------------------------------------------
    def tune(self, D: torch.Tensor, Y: torch.Tensor, s_max: int):
        K, m = D.shape
        self._check(lib().smdl_tune(self._h, _ptr(D), m, K, _ptr(Y), Y.shape[0], s_max))
        return self.get_tile(m, K, s_max)

    def get_tile(self, m: int, K: int, s_max: int):
        a, b = C.c_int(0), C.c_int(0)
        self._check(lib().smdl_get_tile(self._h, m, K, s_max, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_tile(self, K: int, s_max: int, lanes: int, signals_per_item: int):
        self._check(lib().smdl_set_tile(self._h, K, s_max, lanes, signals_per_item))

    def set_mod_solver(self, mode: int):
        """0 automatic, 1 multi-work-group panels, 2 one work group per dictionary."""
        self._check(lib().smdl_set_mod_solver(self._h, mode))

    def set_flags(self, flags: int):
        """Handle-wide options: SMDL_DETERMINISTIC | SMDL_CHECK_FINITE | SMDL_ASYNC (0 clears).
        With SMDL_ASYNC the coding, Gram and logit calls return once queued on the handle's stream:
        synchronise (torch.cuda.synchronize()) before reading their outputs."""
        self._check(lib().smdl_set_flags(self._h, int(flags)))

    def set_autotune(self, enabled: bool):
        self._check(lib().smdl_set_autotune(self._h, 1 if enabled else 0))

    # ---- proposer -------------------------------------------------------------------
    def proposer(self, Ws, bs) -> "Proposer":
        return Proposer(self, Ws, bs)

    def proposer_seeded(self, widths, seed: int) -> "Proposer":
        """A proposer with seeded Kaiming-uniform initial weights drawn on the host by the
        library (splitmix64 uniforms)."""
        return Proposer(self, None, None, widths=widths, seed=seed)

    def omp_code_proposed(self, prop: "Proposer", D: torch.Tensor, Y: torch.Tensor, s_max: int, n_cand: int,
                          eps_fallback: float, want_cand: bool = False):
        K, m = D.shape
        _dev_tensor(D, torch.float32, "D")
        _dev_tensor(Y, torch.float32, "Y")
        N = Y.shape[0]
        X = Codes.empty(N, s_max, Y.device)
        fb = torch.empty((N,), dtype=torch.uint8, device=Y.device)
        cand = torch.empty((N, n_cand), dtype=torch.int32, device=Y.device) if want_cand else None
        nfb = C.c_int64(0)
        self._check(lib().smdl_omp_code_proposed(self._h, prop._p, _ptr(D), m, K, _ptr(Y), N, s_max, n_cand,
                                               float(eps_fallback), X._c(), _ptr(fb), C.byref(nfb), _ptr(cand)))
        return X, fb, nfb.value, cand

    def prop_phase_ms(self):
        v = (C.c_float * 3)()
        self._check(lib().smdl_prop_phase_ms(self._h, v))
        return list(v)


class Proposer:
    """The learned support proposer: an MLP y/||y|| -> one logit per atom (on the GPU)."""

    def __init__(self, h: Handle, Ws, bs, widths=None, seed=None):
        self.h = h
        self._p = C.c_void_p(0)
        if Ws is None:
            self.widths = [int(w) for w in widths]
            n = len(self.widths) - 1
            wa = (C.c_int * (n + 1))(*self.widths)
            h._check(lib().smdl_prop_create_seeded(h._h, n, wa, C.c_uint64(int(seed) & (2**64 - 1)),
                                                   C.byref(self._p)))
            return
        self.widths = [int(Ws[0].shape[1])] + [int(W.shape[0]) for W in Ws]
        n = len(Ws)
        wa = (C.c_int * (n + 1))(*self.widths)
        WP, BP, keep = self._host_ptrs(Ws, bs)
        h._check(lib().smdl_prop_create(h._h, n, wa, WP, BP, C.byref(self._p)))

    def _host_ptrs(self, Ws, bs):
        n = self.n_layers
        if len(Ws) != n or len(bs) != n:
            raise ValueError(f"expected {n} weight matrices and bias vectors")
        Ws = [np.ascontiguousarray(W, dtype=np.float32) for W in Ws]
        bs = [np.ascontiguousarray(b, dtype=np.float32) for b in bs]
        for l, (W, b) in enumerate(zip(Ws, bs)):
            if W.shape != (self.widths[l + 1], self.widths[l]) or b.shape != (self.widths[l + 1],):
                raise ValueError(f"layer {l}: W must be {(self.widths[l + 1], self.widths[l])}, "
                                 f"b {(self.widths[l + 1],)}")
        WP = (C.POINTER(C.c_float) * n)(*[W.ctypes.data_as(C.POINTER(C.c_float)) for W in Ws])
        BP = (C.POINTER(C.c_float) * n)(*[b.ctypes.data_as(C.POINTER(C.c_float)) for b in bs])
        return WP, BP, (Ws, bs)

    def set_weights(self, Ws, bs):
        """New weights and biases; the Adam state restarts from zero."""
        WP, BP, keep = self._host_ptrs(Ws, bs)
        self.h._check(lib().smdl_prop_set(self.h._h, self._p, WP, BP))

    def close(self):
        if self._p:
            lib().smdl_prop_destroy(self._p)
            self._p = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_layers(self):
        return len(self.widths) - 1

    def weights(self):
        Ws = [np.empty((o, i), np.float32) for i, o in zip(self.widths[:-1], self.widths[1:])]
        bs = [np.empty((o,), np.float32) for o in self.widths[1:]]
        n = self.n_layers
        WP = (C.POINTER(C.c_float) * n)(*[W.ctypes.data_as(C.POINTER(C.c_float)) for W in Ws])
        BP = (C.POINTER(C.c_float) * n)(*[b.ctypes.data_as(C.POINTER(C.c_float)) for b in bs])
        self.h._check(lib().smdl_prop_get(self.h._h, self._p, WP, BP))
        return Ws, bs

    def logits(self, Y: torch.Tensor) -> torch.Tensor:
        _dev_tensor(Y, torch.float32, "Y")
        out = torch.empty((Y.shape[0], self.widths[-1]), dtype=torch.float32, device=Y.device)
        self.h._check(lib().smdl_prop_logits(self.h._h, self._p, _ptr(Y), Y.shape[0], _ptr(out)))
        return out

    def grad(self, Y: torch.Tensor, labels: Codes):
        _dev_tensor(Y, torch.float32, "Y")
        dW = [torch.empty((o, i), dtype=torch.float32, device=Y.device)
              for i, o in zip(self.widths[:-1], self.widths[1:])]
        db = [torch.empty((o,), dtype=torch.float32, device=Y.device) for o in self.widths[1:]]
        n = self.n_layers
        GW = (C.c_void_p * n)(*[t.data_ptr() for t in dW])
        GB = (C.c_void_p * n)(*[t.data_ptr() for t in db])
        loss = C.c_float(0)
        self.h._check(lib().smdl_prop_grad(self.h._h, self._p, _ptr(Y), Y.shape[0], labels._c(), C.byref(loss), GW, GB))
        return loss.value, dW, db

    def train(self, Y: torch.Tensor, labels: Codes, epochs: int = 10, batch: int = 1024, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, shuffle_seed: int = 0):
        _dev_tensor(Y, torch.float32, "Y")
        opts = _TrainOpts(epochs, batch, lr, beta1, beta2, eps, shuffle_seed)
        losses = (C.c_float * max(1, epochs))()
        self.h._check(lib().smdl_prop_train(self.h._h, self._p, _ptr(Y), Y.shape[0], labels._c(), C.byref(opts), losses))
        return list(losses)[:epochs]
