"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before touching the GPU (these run without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_2304_09439_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = ""
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            with open(os.path.join(ROOT, "include", name)) as f:
                text += f.read()
    return sorted(set(re.findall(r"LOCC_API[^;(]*?\b(locc_\w+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = B.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert B.version().startswith("locc ")


def test_no_hip_fallback_or_cpu_symbols_are_exported():
    out = os.popen(f"nm -D --defined-only {B.LIB_PATH}").read()
    exported = sorted(re.findall(r"\bT (\w+)", out))
    assert exported == _declared()


def _cfg(**kw):
    base = dict(K=64, enc_h1=64, enc_h2=128, head_h=256, pad_m=0.01, precision=0, reserved=0)
    base.update(kw)
    return B.Config(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(K=0), B.ERR_INVALID_ARG),
    (dict(K=48), B.ERR_INVALID_ARG),
    (dict(K=512), B.ERR_INVALID_ARG),
    (dict(pad_m=-1.0), B.ERR_INVALID_ARG),
    (dict(pad_m=float("nan")), B.ERR_INVALID_ARG),
    (dict(reserved=1), B.ERR_INVALID_ARG),
    (dict(precision=7), B.ERR_INVALID_ARG),
    (dict(enc_h1=96), B.ERR_UNSUPPORTED),
    (dict(enc_h2=256), B.ERR_UNSUPPORTED),
])
def test_create_rejects_bad_configurations(kw, status):
    L = B.load()
    h = ctypes.c_void_p()
    cfg = _cfg(**kw)
    assert L.locc_create(ctypes.byref(cfg), 0, ctypes.byref(h)) == status
    assert not h.value
    assert L.locc_last_error().decode()


def test_null_arguments_are_rejected():
    L = B.load()
    assert L.locc_create(None, 0, None) == B.ERR_INVALID_ARG
    assert L.locc_detect(None, None, 0, None, 0, None, None, None) == B.ERR_INVALID_ARG
    assert L.locc_debug_crop(None, None, 0, None, 0, None, None, None) == B.ERR_INVALID_ARG
    assert L.locc_debug_forward(None, None, 0, None, 0, None, None, None, None, None) == B.ERR_INVALID_ARG
    assert L.locc_upload_shapes(None, 1, None, None) == B.ERR_INVALID_ARG
    assert L.locc_upload_weights(None, None, 0) == B.ERR_INVALID_ARG
    n = ctypes.c_int64()
    assert L.locc_device_errors(None, None, ctypes.byref(n), 0) == B.ERR_INVALID_ARG
    L.locc_destroy(None)  # no-op


def test_object_and_contact_layouts_are_32_bytes():
    import numpy as np
    objs = B.pack_objects(np.zeros((3, 3)), np.tile([1, 0, 0, 0], (3, 1)), [0, 5, -1])
    assert objs.dtype == np.float32 and objs.shape == (3, 8) and objs.nbytes == 96
    assert list(objs[:, 3].view(np.int32)) == [0, 5, -1]


def test_voxel_weight_count_and_host_argument_checks():
    L = B.load()
    from oracle import voxel_locc as V
    assert L.locc_voxel_weight_count() == V.n_weights()
    out = ctypes.c_void_p()
    assert L.locc_voxel_create(0, None) == B.ERR_INVALID_ARG
    assert L.locc_voxel_upload_weights(None, None, 0) == B.ERR_INVALID_ARG
    assert L.locc_voxel_detect(None, None, 0, None, 0, None, None, None, None) == B.ERR_INVALID_ARG
    del out
