"""The C ABI library loads and exports every function include/perch.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "perch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(perch_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_symbols():
    from paper_1510_05613_amd import perch

    assert set(_declared()) == set(perch.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1510_05613_amd import perch

    if not os.path.exists(perch.LIB_PATH):
        from paper_1510_05613_amd import build

        build.build()
    lib = ctypes.CDLL(perch.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    lib.perch_last_error.restype = ctypes.c_char_p
    assert lib.perch_last_error() == b""


def test_argument_errors_need_no_gpu():
    """Host-side validation runs before any device work."""
    from paper_1510_05613_amd import perch

    L = perch.load()
    out = ctypes.c_void_p()
    assert L.perch_create(None, None, ctypes.byref(out)) == -1
    assert b"null" in L.perch_last_error()
    s = perch._Sensor()
    s.width, s.height, s.fx, s.fy, s.delta = 0, 10, 100.0, 100.0, 0.01
    assert L.perch_create(ctypes.byref(s), None, ctypes.byref(out)) == -1
    assert L.perch_eval_successors(None, None, 0, None, 0, None, None, None) == -1
    assert L.perch_cnn_predict_scene(None, None, None, 0, None, 0, None) == -1
    assert L.perch_cnn_predict(None, None, 0, None, 0, None) == -1


def test_product_path_refuses_without_gpu():
    import torch

    from paper_1510_05613_amd import perch, scenes

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    sensor = scenes.make_sensor(scenes.CONFIGS[1])
    with pytest.raises(perch.PerchError):
        perch.Context(sensor)
