"""CPU checks of the C ABI: the library loads, exports every symbol include/llp.h declares, and the host-side
validation rejects bad problem descriptions.  No device work is done here."""
import ctypes
import os
import re

import pytest

from paper_2103_09943_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2103_09943_amd import build
        build.build()
    return B.lib()


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(llp_[a-zA-Z_0-9]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "llp_pansharpen" in names and len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert B.status_str(B.OK) == "ok"
    assert "non-finite" in B.status_str(B.E_NONFINITE)
    assert B.status_str(12345) == "unknown status"


def test_null_context_is_rejected(lib):
    shp = B.Shape(4, 16, 16, 4, 9)
    prm = B.Params(1, 1e-2, 1e-3, 10, 0.0, 0)
    st = lib.llp_pansharpen(None, ctypes.byref(shp), ctypes.byref(prm), None, None, None, None, None, None, None)
    assert st == B.E_ARG
    assert lib.llp_apply_A(None, ctypes.byref(shp), ctypes.byref(prm), None, None, None, None, None) == B.E_ARG
    assert lib.llp_create(None, 0) == B.E_ARG
    assert lib.llp_pansharpen_batch(None, 1, ctypes.byref(shp), ctypes.byref(prm), None, None, None, None, None,
                                    None, 0, None) == B.E_ARG
    assert lib.llp_autotune(None, ctypes.byref(shp), ctypes.byref(prm), None, None, None, None, 8, None,
                            None) == B.E_ARG
    assert lib.llp_autotune_batch(None, ctypes.byref(shp), ctypes.byref(prm), None, None, None, 0, 8, None,
                                  None) == B.E_ARG
    assert lib.llp_tune_save(None, b"/tmp/x.json") == B.E_ARG
    assert lib.llp_tune_load(None, b"/tmp/x.json") == B.E_ARG
    assert lib.llp_tune_clear(None) == B.E_ARG
    assert lib.llp_tune_count(None) == 0
    assert lib.llp_cnn_set_weights(None, None, B.CNN_PARAMS) == B.E_ARG
    assert lib.llp_cnn_get_weights(None, None, B.CNN_PARAMS) == B.E_ARG
    assert lib.llp_cnn_warm_start(None, ctypes.byref(shp), None, None, None, None, None) == B.E_ARG
    assert lib.llp_cnn_loss_grad(None, ctypes.byref(shp), None, None, None, None, None, None) == B.E_ARG
    assert lib.llp_cnn_train_step(None, ctypes.byref(shp), None, None, None, 1e-3, None, None) == B.E_ARG


GOOD = dict(N=4, h=64, w=64, c=4, n=9)
GOODP = dict(r=1, lam=1e-2, eps=1e-3, max_iters=50, tol=0.0, init_mode=0)


@pytest.mark.parametrize("shape,params,want", [
    ({}, {}, B.OK),
    ({"n": 8}, {}, B.E_SHAPE),                      # even kernel
    ({"N": 0}, {}, B.E_SHAPE),
    ({"h": 2, "w": 2, "c": 2, "n": 5}, {}, B.E_SHAPE),  # kernel larger than the image
    ({"c": 9}, {}, B.E_UNSUPPORTED),
    ({"n": 35, "h": 64}, {}, B.E_UNSUPPORTED),
    ({}, {"r": -1}, B.E_ARG),
    ({}, {"r": 5}, B.E_UNSUPPORTED),
    ({"h": 1, "w": 1, "c": 2, "n": 1}, {"r": 1}, B.E_SHAPE),  # window larger than the image
    ({}, {"lam": -1.0}, B.E_ARG),
    ({}, {"eps": -1e-3}, B.E_ARG),
    ({}, {"lam": float("nan")}, B.E_ARG),
    ({}, {"max_iters": -1}, B.E_ARG),
    ({}, {"tol": float("inf")}, B.E_ARG),
    ({}, {"init_mode": 3}, B.E_ARG),
    ({"N": 1, "h": 3, "w": 5, "c": 1, "n": 3}, {"r": 1}, B.OK),  # ragged, c = 1
    ({"N": 16, "h": 1024, "w": 1024, "c": 4, "n": 17}, {"r": 2}, B.OK),  # the largest measured scene
    ({"N": 200, "h": 1024, "w": 1024, "c": 4, "n": 17}, {"r": 2}, B.E_UNSUPPORTED),  # > 2^31 pixels
])
def test_validation(lib, shape, params, want):
    s = B.Shape(**{**GOOD, **shape})
    p = dict(GOODP, **params)
    prm = B.Params(p["r"], p["lam"], p["eps"], p["max_iters"], p["tol"], p["init_mode"])
    assert B.validate(s, prm) == want


def test_binding_refuses_cpu_tensors(lib):
    import torch
    with pytest.raises(TypeError):
        B._ptr(torch.zeros(4))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libllp.so"))
    with pytest.raises(RuntimeError, match="not built"):
        B.lib()
