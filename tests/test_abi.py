"""CPU checks of the C ABI: the library loads, exports every symbol the header declares and
rejects bad arguments before touching the GPU."""

from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmb_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2308_14737_amd import _lib
    return _lib.load()


def test_header_symbols_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in fmb.h but not exported"


def test_binding_covers_header():
    from paper_2308_14737_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES), set(_declared()) ^ set(_lib.SIGNATURES)


def test_abi_version(lib):
    assert lib.fmb_abi_version() == 3


def test_invalid_arguments_rejected_without_gpu(lib):
    h = ctypes.c_void_p()
    f = ctypes.c_float
    assert lib.fmb_scene_create(None, 4, None, None, None, None, f(1.0)) == 1
    assert lib.fmb_scene_create(ctypes.byref(h), 0, None, None, None, None, f(1.0)) == 1
    assert b"n must be" in lib.fmb_last_error()
    fake = ctypes.c_void_p(4096)
    assert lib.fmb_scene_create(ctypes.byref(h), 4, fake, fake, fake, None, f(1.0)) == 1
    assert lib.fmb_scene_create(ctypes.byref(h), 4, fake, fake, fake, fake, f(0.0)) == 1
    assert b"eta" in lib.fmb_last_error()
    assert lib.fmb_scene_create(ctypes.byref(h), 4, ctypes.c_void_p(4098), fake, fake, fake, f(1.0)) == 1
    assert lib.fmb_render(None, None, None, None, None, None, None, None) == 1
    assert lib.fmb_backward(None, *([None] * 14)) == 1
    assert lib.fmb_set_colors(None, None, None) == 1
    assert lib.fmb_set_cameras(None, 1, None, None, None, None, None) == 1
    assert lib.fmb_batch_forward(None, None, None, None, None, None, None, None) == 1
    assert lib.fmb_batch_forward_loss(None, *([None] * 8), f(1.0), None, None, None) == 1
    assert lib.fmb_batch_graph_launch(None, 2, None) == 1
    assert lib.fmb_scene_destroy(None) == 0
    assert lib.fmb_batch_destroy(None) == 0
    assert lib.fmb_num_rays(None) == 0
    out = (ctypes.c_double * 6)()
    assert lib.fmb_kernel_times(out, 1) == 0


def test_batch_create_rejects_bad_sizes(lib):
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096)
    n = (ctypes.c_int32 * 2)(3, 0)
    v = (ctypes.c_int32 * 2)(1, 1)
    eta = (ctypes.c_float * 2)(1.0, 1.0)
    hw = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    rc = lib.fmb_batch_create(ctypes.byref(h), 2, n, v, fake, fake, fake, fake, eta, fake, fake, hw, None, None)
    assert rc == 1 and b">= 1 Gaussian" in lib.fmb_last_error()


def test_new_entry_points_reject_bad_arguments(lib):
    """Model, flow-target, configuration, split-statistic and split entry points check their
    arguments on the host."""
    assert lib.fmb_set_model(None, None, 1) == 1
    assert lib.fmb_set_flow_pose2(None, None, None, None) == 1
    assert lib.fmb_set_config(None, None, 0, 0, 1, 1) == 1
    assert lib.fmb_split_statistic(None, None, None, None, None, None) == 1
    assert lib.fmb_prune_mask(0, None, ctypes.c_float(2.0), None) == 1
    assert lib.fmb_split_mask(0, None, ctypes.c_float(1.0), None) == 1
    assert lib.fmb_split_gaussians(-1, *([None] * 10)) == 1
    # a precision factor that is not positive definite is refused
    mean = (ctypes.c_float * 3)(0, 0, 0)
    prec = (ctypes.c_float * 6)(0, 0, 0, 0, 0, 0)
    w = (ctypes.c_float * 1)(1.0)
    nw = (ctypes.c_float * 2)(0, 0)
    om, op, ow = (ctypes.c_float * 6)(), (ctypes.c_float * 12)(), (ctypes.c_float * 2)()
    assert lib.fmb_split_gaussians(1, mean, prec, w, None, nw, None, om, op, ow, None) == 1
    assert lib.fmb_loss_grad(4, *([None] * 8), ctypes.c_float(1), ctypes.c_float(1), 2, 3, ctypes.c_float(1),
                             *([None] * 5), None) == 1


def test_oversized_shapes_rejected_without_gpu(lib):
    """More rays, Gaussians or views than the FMB_MAX_* limits of fmb.h are refused with
    FMB_ERR_SHAPE on the host, before any device work (and before a scene handle is used)."""
    max_rays, max_gauss, max_views = 2130706432, 268435455, 134217727
    h = ctypes.c_void_p()
    f = ctypes.c_float
    fake = ctypes.c_void_p(4096)
    assert lib.fmb_scene_create(ctypes.byref(h), max_gauss + 1, fake, fake, fake, fake, f(1.0)) == 2
    assert b"FMB_MAX_GAUSSIANS" in lib.fmb_last_error()
    one = (ctypes.c_int32 * 1)(1)
    eta = (ctypes.c_float * 1)(1.0)
    # one view of more than FMB_MAX_RAYS rays, then FMB_MAX_RAYS + 1 rays over two views
    big = (ctypes.c_int32 * 2)(max_rays // 65536 + 1, 65536)
    assert lib.fmb_batch_create(ctypes.byref(h), 1, one, one, fake, fake, fake, fake, eta, fake, fake, big,
                                None, None) == 2
    assert b"FMB_MAX_RAYS" in lib.fmb_last_error()
    two = (ctypes.c_int32 * 1)(2)
    hw2 = (ctypes.c_int32 * 4)(max_rays // 2, 1, max_rays // 2 + 1, 1)
    assert lib.fmb_batch_create(ctypes.byref(h), 1, one, two, fake, fake, fake, fake, eta, fake, fake, hw2,
                                None, None) == 2
    n_big = (ctypes.c_int32 * 2)(max_gauss, 1)
    v2 = (ctypes.c_int32 * 2)(1, 1)
    eta2 = (ctypes.c_float * 2)(1.0, 1.0)
    hw_small = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    assert lib.fmb_batch_create(ctypes.byref(h), 2, n_big, v2, fake, fake, fake, fake, eta2, fake, fake,
                                hw_small, None, None) == 2
    vmany = (ctypes.c_int32 * 1)(max_views + 1)
    assert lib.fmb_batch_create(ctypes.byref(h), 1, one, vmany, fake, fake, fake, fake, eta, fake, fake,
                                hw_small, None, None) == 2
    assert b"FMB_MAX_VIEWS" in lib.fmb_last_error()
    # per-scene cameras and explicit rays: the shape checks run before the handle is used
    assert lib.fmb_set_cameras(fake, 1, fake, fake, big, None, None) == 2
    counts = (ctypes.c_int32 * 2)(max_rays // 2, max_rays // 2 + 1)
    assert lib.fmb_set_rays(fake, 2, fake, fake, counts, fake, None, None) == 2
    assert lib.fmb_set_rays(fake, max_views + 1, fake, fake, counts, fake, None, None) == 2
    # the loss gradient over more rays than the limit
    assert lib.fmb_loss_grad(max_rays + 1, *([fake] * 8), f(1), f(1), 2, 2, f(1), fake, fake, None, None,
                             None, None) == 2
