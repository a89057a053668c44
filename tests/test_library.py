"""The C-ABI library loads and exports every symbol include/hgnn.h declares;
host-side argument checks fail cleanly without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hgnn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hgnn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("hgnn_create", "hgnn_forward", "hgnn_backward", "hgnn_adam_step",
              "hgnn_serve_submit", "hgnn_serve_poll", "hgnn_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2207_11333_amd import hgnn
    lib = hgnn.lib()
    for n in _declared():
        assert hasattr(lib, n), n
        assert n in hgnn._SIGS, f"binding lacks a signature for {n}"


@pytest.mark.parametrize("field,value,msg", [
    ("hidden", 17, "hidden"), ("hidden", 0, "hidden"), ("num_layers", 0, "num_layers"),
    ("edge_feat", 5, "edge_feat"), ("max_degree", 256, "max_degree"),
    ("precision", 2, "precision"), ("delta", 0.0, "delta"), ("recompute", 3, "recompute")])
def test_create_rejects_bad_config_before_touching_a_device(field, value, msg):
    from paper_2207_11333_amd import hgnn
    cfg = hgnn.Config(3, 64, 9, 1, 4, 0, 0, 0, 1.0, 1e-5)
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    rc = hgnn.lib().hgnn_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h))
    assert rc == hgnn.EINVAL
    assert msg in hgnn.lib().hgnn_last_error().decode()
    assert not h.value


def test_null_context_calls_fail_cleanly():
    from paper_2207_11333_amd import hgnn
    L = hgnn.lib()
    assert L.hgnn_backward(None, None, None) == hgnn.EINVAL
    assert L.hgnn_serve_poll(None, 1, None, None) == hgnn.EINVAL
    n = ctypes.c_int64()
    assert L.hgnn_num_params(None, ctypes.byref(n)) == hgnn.EINVAL
    L.hgnn_destroy(None)
