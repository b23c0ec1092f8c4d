"""C-ABI checks that need no GPU: the in-tree library loads, exports every entry point
declared in include/bound.h, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "bound.h")).read()
    return sorted(set(re.findall(r"^\S.*?\b(bound_[a-z_]+)\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2412_09584_amd import binding as B
    return B.lib()


def test_header_declares_the_boundary():
    names = declared()
    for n in ("bound_init", "bound_backward", "bound_concretize", "bound_grad", "bound_adam",
              "bound_dims", "bound_destroy", "bound_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for n in declared():
        assert hasattr(L, n), n


def test_binding_names_match_header():
    from paper_2412_09584_amd import binding as B
    for n in declared():
        assert callable(getattr(B, n)), n


def test_error_paths_without_device(L):
    from paper_2412_09584_amd import binding as B
    assert L.bound_backward(None, None, None, None) == B.BOUND_E_ARG
    assert "null" in B.bound_last_error()
    assert L.bound_grad(None, 0, 0, 0, 0, None, None, None, None) == B.BOUND_E_ARG
    assert L.bound_grad_adam(None, 0, 0, 0, 0, None, None, None, None) == B.BOUND_E_ARG
    st = B.BoundAdamStep(None, None, None, 0, 0.1, 0.9, 0.999, 1e-8, -1.0, 0.0, 1.0)
    assert L.bound_grad_adam(None, 0, 0, 0, 0, None, ctypes.byref(st), None, None) == B.BOUND_E_ARG
    assert L.bound_concretize(-1, 1, 1, None, None, None, None, None, 0, None, None) == B.BOUND_E_ARG
    assert L.bound_adam(10, None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8, 1.0, 0.0, 1.0,
                        None) == B.BOUND_E_ARG
    assert L.bound_adam(0, None, None, None, None, 0, 0.1, 0.9, 0.999, 1e-8, 1.0, 0.0, 1.0,
                        None) == B.BOUND_E_ARG
    out = ctypes.c_void_p()
    assert L.bound_init(None, 1, 1, 1, 0, None, ctypes.byref(out)) == B.BOUND_E_ARG
    layer = B.BoundLayer(B.BOUND_LINEAR, 4, 1, 1, 3, 1, 1, 1, 1, 1, 0, None, None)
    assert L.bound_init(ctypes.byref(layer), 1, 1, 16, 32, None, ctypes.byref(out)) == B.BOUND_E_ARG
    assert "max_save_rows" in B.bound_last_error()
    assert L.bound_set_plan(None, b"R", 1, 1, -1, 0) == B.BOUND_E_ARG
    assert "bound_set_plan" in B.bound_last_error()


def test_bab_error_paths_without_device(L):
    from paper_2412_09584_amd import binding as B
    out = ctypes.c_void_p()
    assert L.bound_bab_init(0, 2, 8, ctypes.byref(out)) == B.BOUND_E_ARG
    assert L.bound_bab_init(4, 2, 4096, ctypes.byref(out)) == B.BOUND_E_ARG   # > 2048 samples
    assert L.bound_bab_pick_out(None, 1, None, None, None, 1, 0.5, 0.05, None, None, None) == B.BOUND_E_ARG
    assert L.bound_bab_split(None, 1, None, None, None, 1, None, None, None, None) == B.BOUND_E_ARG
    assert L.bound_bab_prune(None, 1, None, None, None, None, None) == B.BOUND_E_ARG
    assert "bad arguments" in B.bound_last_error()


def test_shape_validation_without_device(L):
    from paper_2412_09584_amd import binding as B
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    arr = (B.BoundLayer * 2)(
        B.BoundLayer(B.BOUND_CONV2D, 3, 8, 8, 4, 8, 8, 3, 3, 1, 1, fake, fake),
        B.BoundLayer(B.BOUND_LINEAR, 4, 7, 8, 5, 1, 1, 1, 1, 1, 0, fake, fake))
    assert L.bound_init(arr, 2, 1, 16, 0, None, ctypes.byref(out)) == B.BOUND_E_SHAPE
    arr2 = (B.BoundLayer * 1)(B.BoundLayer(B.BOUND_CONV2D, 3, 8, 8, 4, 7, 7, 3, 3, 1, 1, fake, fake))
    assert L.bound_init(arr2, 1, 1, 16, 0, None, ctypes.byref(out)) == B.BOUND_E_SHAPE
    arr3 = (B.BoundLayer * 1)(B.BoundLayer(B.BOUND_CONV2D, 3, 8, 8, 4, 3, 3, 3, 3, 3, 0, fake, fake))
    assert L.bound_init(arr3, 1, 1, 16, 0, None, ctypes.byref(out)) == B.BOUND_E_SHAPE


def test_noalloc_prune_rejects_sizes_without_device(L):
    from paper_2412_09584_amd import binding as B
    assert L.bound_bab_prune_noalloc(4194305, None, None, None, None, None) == B.BOUND_E_ARG
    assert "4194304" in B.bound_last_error()
    assert L.bound_bab_prune_noalloc(-1, None, None, None, None, None) == B.BOUND_E_ARG
