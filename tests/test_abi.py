"""The C-ABI library loads on a machine without a GPU and exports every
function include/ckks_hip.h declares; host-only helpers behave (no device
calls are made here)."""
import ctypes
import os
import re

import numpy as np

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckks_hip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("he_ctx_create", "he_keygen", "he_encode", "he_decode", "he_encrypt", "he_decrypt",
                 "he_add", "he_mul_plain", "he_mul_relin", "he_rescale", "he_rotate",
                 "he_enc_conv_im2col", "he_enc_matmul", "he_sum_slots", "he_pack"):
        assert must in names


def test_library_exports_every_symbol():
    import paper_2104_03152_amd as H
    lib = H.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared call under the same name
    assert all(n in H._SIGS for n in declared_functions())


def test_host_im2col_matches_oracle():
    import paper_2104_03152_amd as H
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 1, (28, 28))
    assert np.array_equal(H.he_im2col(img, 7, 3), O.im2col(img, 7, 3))
    img = rng.uniform(0, 1, (10, 13))
    assert np.array_equal(H.he_im2col(img, 3, 2), O.im2col(img, 3, 2))


def test_last_error_is_a_string():
    import paper_2104_03152_amd as H
    assert isinstance(H.he_last_error(), str)


def test_binding_raises_without_library(tmp_path, monkeypatch):
    import paper_2104_03152_amd as H
    monkeypatch.setattr(H, "LIBPATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(H, "_lib", None)
    try:
        H.lib()
    except RuntimeError as e:
        assert "not built" in str(e)
    else:
        raise AssertionError("expected a failure without the HIP library")
