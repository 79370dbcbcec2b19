"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-only entry points (validation, sizes, errors)
behave as documented."""
import ctypes
import os
import re

import pytest

from paper_2404_10631_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "knnf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(knnf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libknnf.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(declared) == _lib.exported_symbols()


def test_struct_layout_matches_header():
    # knnf_frame: 5 int32 + float, then 6 pointers (8-byte aligned) = 24 + 48
    assert ctypes.sizeof(_lib.knnf_frame) == 72
    assert _lib.knnf_frame.pc1.offset == 24
    assert ctypes.sizeof(_lib.knnf_plan) == 28
    assert _lib.knnf_plan.flags.offset == 24


def test_version(lib):
    assert "gfx950" in _lib.knnf_version()


def _frame(**kw):
    f = _lib.knnf_frame()
    f.H, f.W, f.C, f.K, f.R, f.lam = 8, 8, 4, 8, 2, 0.01
    f.pc1 = f.prob = f.out_prob = f.out_class = 0x1000
    for k, v in kw.items():
        setattr(f, k, v)
    return f


@pytest.mark.parametrize("kw", [
    dict(H=0), dict(W=0), dict(C=0), dict(C=17), dict(K=0), dict(K=65), dict(R=-1),
    dict(K=9, R=0),                 # K > smallest window (1 row x 8)
    dict(lam=-1.0), dict(lam=float("nan")), dict(lam=float("inf")), dict(lam=1e18),
    dict(pc1=None), dict(prob=None), dict(out_prob=None), dict(out_class=None),
    dict(H=50000, W=50000),         # H*W > 2^31-1
])
def test_validate_rejects(lib, kw):
    assert _lib.knnf_validate(_frame(**kw)) == _lib.KNNF_EINVAL
    assert _lib.last_error() != ""


@pytest.mark.parametrize("kw", [dict(), dict(K=8, R=0), dict(K=64, H=8, W=8, R=7),
                                dict(lam=0.0), dict(out_nbr=None), dict(H=1, W=1, K=1)])
def test_validate_accepts(lib, kw):
    assert _lib.knnf_validate(_frame(**kw)) == _lib.KNNF_OK


def test_frame_bytes(lib):
    b = _lib.knnf_frame_bytes(380, 480, 4, 40, False)
    px = 380 * 480
    assert b >= px * (4 + 16 + 16 + 4)
    assert b < px * (4 + 16 + 16 + 4) + 4 * 256
    assert _lib.knnf_frame_bytes(380, 480, 4, 40, True) >= b + 2 * px * 40 * 4
    assert _lib.knnf_frame_bytes(0, 4, 4, 4, False) == 0


def test_null_context_is_einval(lib):
    f = _frame()
    assert lib.knnf_filter(None, ctypes.byref(f), None, None) == _lib.KNNF_EINVAL
    assert lib.knnf_filter_batch(None, ctypes.byref(f), 1, None, None) == _lib.KNNF_EINVAL
    assert lib.knnf_destroy(None) == _lib.KNNF_OK


@pytest.mark.parametrize("kw,word", [
    (dict(npix=0), "npix"), (dict(npix=(1 << 40) + 1), "npix"),
    (dict(bands=0), "bands"), (dict(bands=4097), "bands"),
    (dict(cube=None), "NULL"), (dict(mean=None), "NULL"), (dict(vec=None), "NULL"),
    (dict(out=None), "NULL"), (dict(), "context"),
])
def test_pc1_validation(lib, kw, word):
    a = dict(cube=0x1000, npix=100, bands=128, mean=0x2000, vec=0x3000, out=0x4000)
    a.update(kw)
    st = lib.knnf_pc1(None, a["cube"], a["npix"], a["bands"], a["mean"], a["vec"], a["out"], 1, None)
    assert st == _lib.KNNF_EINVAL
    assert word in _lib.last_error()


@pytest.mark.parametrize("kw,word", [
    (dict(npix=0), "npix"), (dict(npix=(1 << 31) + 1), "npix"),
    (dict(bands=0), "bands"), (dict(bands=4097), "bands"),
    (dict(classes=1), "classes"), (dict(classes=9), "classes"),
    (dict(cube=None), "NULL"), (dict(w=None), "NULL"), (dict(bias=None), "NULL"),
    (dict(A=None), "NULL"), (dict(B=None), "NULL"), (dict(out=None), "NULL"),
    (dict(), "context"),
])
def test_svm_validation(lib, kw, word):
    a = dict(cube=0x1000, npix=100, bands=128, classes=4, w=0x2000, bias=0x3000, A=0x4000,
             B=0x5000, out=0x6000)
    a.update(kw)
    st = lib.knnf_svm(None, a["cube"], a["npix"], a["bands"], a["classes"], a["w"], a["bias"],
                      a["A"], a["B"], a["out"], None)
    assert st == _lib.KNNF_EINVAL
    assert word in _lib.last_error()


def test_context_calls_reject_null(lib):
    assert lib.knnf_ctx_status(None) == _lib.KNNF_EINVAL
    assert lib.knnf_inject_fault(None) == _lib.KNNF_EINVAL
    f = _frame()
    p = _lib.knnf_plan()
    assert lib.knnf_tune_lookup(None, ctypes.byref(f), 1, ctypes.byref(p)) == _lib.KNNF_EINVAL
    assert lib.knnf_tune(None, ctypes.byref(f), 1, 1, None, None) == _lib.KNNF_EINVAL


def test_create_without_a_gpu_is_a_device_error(lib):
    """No usable HIP device: knnf_create fails with KNNF_EDEVICE (or EINVAL for
    an ordinal beyond the devices present) and leaves *out NULL."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p(0x1234)
    st = lib.knnf_create(ctypes.byref(h), 0)
    assert st in (_lib.KNNF_EDEVICE, _lib.KNNF_EINVAL)
    assert h.value is None
    assert _lib.last_error() != ""
