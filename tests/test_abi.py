"""The C-ABI library loads and exports every entry point include/smdl.h declares; calls
with a null handle fail with SMDL_E_ARG (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "smdl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smdl_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    import paper_1403_4781_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1403_4781_amd import build
        build.build()
    return C.CDLL(pkg.LIB_PATH)


def test_exports_every_declared_symbol(so):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_1403_4781_amd as pkg
    L = pkg.lib()
    for n in _declared():
        assert getattr(L, n).argtypes is not None or n == "smdl_version", n


def test_null_handle_is_rejected(so):
    so.smdl_omp_code.restype = C.c_int
    assert so.smdl_version() == 10000
    for name in ("smdl_gram", "smdl_omp_code", "smdl_mod_update", "smdl_learn", "smdl_split_merge_learn",
                 "smdl_prop_logits", "smdl_omp_code_proposed", "smdl_tune"):
        fn = getattr(so, name)
        fn.restype = C.c_int
        fn.argtypes = None
    assert so.smdl_gram(None, None, 64, 64, None) == -1
    so.smdl_create.restype = C.c_int
    assert so.smdl_create(None, 0, None) == -1


def test_no_gpu_create_fails_cleanly(so):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p(0)
    so.smdl_create.restype = C.c_int
    assert so.smdl_create(C.byref(h), 0, None) != 0
    assert not h.value
