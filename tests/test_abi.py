"""The C ABI without a GPU: the library loads, exports every function the
header declares, and its host-only calls validate and lay out plans."""
import ctypes
import os
import re

import numpy as np
import pytest

import dicgen
import paper_1905_06228_amd as dic
from paper_1905_06228_amd.dic import PairDesc, PlanDesc, Tuning

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dic.h")


@pytest.fixture(scope="module")
def L():
    return dic.load_library()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dic_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(dic.dic.EXPORTS)


def make(L, pairs, precision=0, max_iters=20, tol=1e-3, flags=0):
    arr = (PairDesc * max(1, len(pairs)))()
    for k, q in enumerate(pairs):
        arr[k] = PairDesc(*q)
    d = PlanDesc(len(pairs), arr, precision, max_iters, tol, flags)
    h = ctypes.c_void_p()
    rc = L.dic_plan_create(ctypes.byref(d), ctypes.byref(h))
    return rc, h


def test_plan_create_and_workspace(L):
    rc, h = make(L, [(256, 256, 10, 8, 0, 0, 0, 484)])
    assert rc == 0 and h.value
    nb = ctypes.c_size_t(0)
    assert L.dic_plan_workspace_size(h, ctypes.byref(nb)) == 0
    # gradients 2*H*W floats + 484 templates of 441 floats + 484 records, at least
    assert nb.value >= 2 * 256 * 256 * 4 + 484 * 441 * 4 + 484 * 300
    rc64, h64 = make(L, [(256, 256, 10, 8, 0, 0, 0, 484)], precision=1)
    nb64 = ctypes.c_size_t(0)
    L.dic_plan_workspace_size(h64, ctypes.byref(nb64))
    assert nb64.value < nb.value      # the plain form keeps no gradients or templates
    t = Tuning()
    assert L.dic_plan_get_tuning(h, ctypes.byref(t)) == 0
    # search +-8: the matrix-core search form is the default
    assert (t.search_block, t.search_occupancy) == (32, 0)
    for bad in (Tuning(5, 0, 4, 4), Tuning(8, 17, 4, 4), Tuning(8, 0, 9, 4), Tuning(4, 0, 1, 17),
                Tuning(16, 0, 4, 4)):
        assert L.dic_plan_set_tuning(h, ctypes.byref(bad)) == -1
    for good in (Tuning(4, 2, 2, 6), Tuning(8, 0, 4, 4), Tuning(32, 3, 1, 2)):
        assert L.dic_plan_set_tuning(h, ctypes.byref(good)) == 0
        got = Tuning()
        L.dic_plan_get_tuning(h, ctypes.byref(got))
        assert (got.search_block, got.search_occupancy) == (good.search_block, good.search_occupancy)
    L.dic_plan_destroy(h)
    L.dic_plan_destroy(h64)


def test_search_form_follows_radius(L):
    """Windows up to +-31 default to the matrix-core search form (2 x 2 tiles
    beyond +-16); beyond that the vector-ALU form runs and the matrix-core
    form is refused."""
    t = Tuning()
    for S in (16, 20, 31):
        rc, h = make(L, [(512, 512, 12, S, 0, 0, 0, 100)])
        assert rc == 0
        L.dic_plan_get_tuning(h, ctypes.byref(t))
        assert t.search_block == 32, S
        L.dic_plan_destroy(h)
    rc, h = make(L, [(512, 512, 12, 32, 0, 0, 0, 100)])
    assert rc == 0
    L.dic_plan_get_tuning(h, ctypes.byref(t))
    assert t.search_block == 8
    assert L.dic_plan_set_tuning(h, ctypes.byref(Tuning(32, 0, 4, 4))) == -4
    assert "matrix-core" in L.dic_last_error().decode()
    L.dic_plan_destroy(h)
    rc, h = make(L, [(512, 512, 20, 16, 0, 0, 0, 100)])
    L.dic_plan_get_tuning(h, ctypes.byref(t))
    assert rc == 0 and t.search_block == 32
    L.dic_plan_destroy(h)


@pytest.mark.parametrize("pairs,kw,why", [
    ([(4, 256, 10, 8, 0, 0, 0, 1)], {}, "width"),
    ([(256, 256, 21, 8, 0, 0, 0, 1)], {}, "subset_radius"),
    ([(256, 256, 10, 33, 0, 0, 0, 1)], {}, "search_radius"),
    ([(256, 256, 10, 8, -1, 0, 0, 1)], {}, "offset"),
    ([(256, 256, 10, 8, 0, 0, 5, 1)], {}, "contiguous"),
    ([(256, 256, 10, 8, 0, 0, 0, 3), (64, 64, 5, 4, 0, 0, 2, 3)], {}, "contiguous"),
    ([(256, 256, 10, 8, 0, 0, 0, 1)], {"max_iters": 0}, "max_iters"),
    ([(256, 256, 10, 8, 0, 0, 0, 1)], {"tol": 0.0}, "conv_tol"),
    ([(256, 256, 10, 8, 0, 0, 0, 1)], {"precision": 7}, "precision"),
    ([(256, 256, 10, 8, 0, 0, 0, 1)], {"flags": 128}, "flag"),
    ([(20, 20, 9, 0, 0, 0, 0, 1)], {}, "fit"),
    # deterministic adjoint: a deformed image partly overlapping another pair's
    ([(64, 64, 5, 4, 0, 0, 0, 1), (64, 64, 5, 4, 0, 100, 1, 1)], {"flags": 4}, "disjoint"),
    ([(64, 64, 5, 4, 0, 0, 0, 1), (32, 64, 5, 4, 0, 0, 1, 1)], {"flags": 4}, "disjoint"),
])
def test_plan_create_rejects(L, pairs, kw, why):
    rc, h = make(L, pairs, **kw)
    assert rc == -1 and not h.value
    assert why in L.dic_last_error().decode()


def test_deterministic_adjoint_shared_or_disjoint_images(L):
    """With the deterministic adjoint, pairs on the same deformed image share
    one fixed-point accumulator (no extra workspace); disjoint images each
    get one; without the flag overlaps are allowed (float atomics)."""
    one = (64, 64, 5, 4, 0, 0, 0, 1)
    same = (64, 64, 7, 4, 0, 0, 1, 1)             # same def_offset, width, height
    apart = (64, 64, 7, 4, 0, 64 * 64, 1, 1)      # the next image of the arena
    sizes = {}
    for name, pairs in (("single", [one]), ("same", [one, same]), ("apart", [one, apart])):
        rc, h = make(L, pairs, flags=4)
        assert rc == 0, L.dic_last_error()
        nb = ctypes.c_size_t(0)
        L.dic_plan_workspace_size(h, ctypes.byref(nb))
        sizes[name] = nb.value
        L.dic_plan_destroy(h)
    # a second accumulator (8 bytes per pixel) only for a distinct image
    assert sizes["apart"] - sizes["same"] >= 8 * 64 * 64 - 512
    rc, h = make(L, [one, (64, 64, 5, 4, 0, 100, 1, 1)])
    assert rc == 0
    L.dic_plan_destroy(h)


def test_interpolation_flags(L):
    """Bilinear (16), the bicubic coefficient table (32) and the B-spline (64)
    are FP32-only and exclusive; the table adds 64 bytes of workspace per
    deformed pixel, the spline's coefficient and scratch images 8."""
    pair = [(256, 128, 10, 8, 0, 0, 0, 50)]
    sizes = {}
    for flags in (0, 16, 32, 64):
        rc, h = make(L, pair, flags=flags)
        assert rc == 0
        nb = ctypes.c_size_t(0)
        assert L.dic_plan_workspace_size(h, ctypes.byref(nb)) == 0
        sizes[flags] = nb.value
        L.dic_plan_destroy(h)
    assert sizes[16] == sizes[0]
    assert 256 * 128 * 64 <= sizes[32] - sizes[0] <= 256 * 128 * 64 + 256
    assert 256 * 128 * 8 <= sizes[64] - sizes[0] <= 256 * 128 * 8 + 1024
    for flags in (48, 80, 96, 112):
        rc, h = make(L, pair, flags=flags)
        assert rc == -1 and not h.value and "exclusive" in L.dic_last_error().decode()
    for flags in (16, 32, 64):
        rc, h = make(L, pair, precision=1, flags=flags)
        assert rc == -4 and not h.value and "FP32" in L.dic_last_error().decode()


def test_null_arguments_and_unbound(L):
    assert L.dic_plan_create(None, None) == -1
    rc, h = make(L, [(64, 64, 5, 4, 0, 0, 0, 10)])
    assert rc == 0
    # device calls on an unbound plan fail on the host before touching a GPU
    assert L.dic_integer_search(h, None, None, None, None, None, None, None, None) == -6
    assert L.dic_plan_bind(h, None, 0, None) == -1
    assert L.dic_plan_bind(h, ctypes.c_void_p(256 + 8), 1 << 30, None) == -1   # misaligned
    assert L.dic_plan_bind(h, ctypes.c_void_p(4096), 16, None) == -2           # too small
    L.dic_plan_destroy(h)
    assert L.dic_status_string(-2).decode() == "workspace too small"


def test_empty_plan_is_valid(L):
    rc, h = make(L, [(64, 64, 5, 4, 0, 0, 0, 0)])
    assert rc == 0
    L.dic_plan_destroy(h)


@pytest.mark.parametrize("W,H,M,S,step", [(256, 256, 10, 8, 10), (1024, 1024, 15, 16, 5),
                                          (512, 512, 20, 8, 6), (4096, 3000, 14, 24, 7),
                                          (100, 60, 7, 3, 9), (30, 30, 10, 8, 5)])
def test_library_grid_matches_generator(W, H, M, S, step):
    lib = dic.poi_grid(W, H, M, S, step).numpy()
    np.testing.assert_array_equal(lib, dicgen.poi_grid(W, H, M, S, step))


def test_noalloc_rejects_plans_beyond_its_scratch(L):
    """dic_correlate_noalloc checks the plan's workspace against its 64 MiB
    static scratch before touching the device."""
    rc, h = make(L, [(4096, 3000, 14, 24, 0, 0, 0, 16)])
    assert rc == 0
    nb = ctypes.c_size_t(0)
    L.dic_plan_workspace_size(h, ctypes.byref(nb))
    assert nb.value > 64 << 20
    fake = ctypes.c_void_p(256)
    args = [h, fake, fake, fake, None, None, fake, None, None, fake, fake, fake, fake, None]
    assert L.dic_correlate_noalloc(*args) == -2
    assert b"64" in L.dic_last_error() or b"67108864" in L.dic_last_error()
    # null required pointers are rejected first
    args[1] = None
    assert L.dic_correlate_noalloc(*args) == -1
    L.dic_plan_destroy(h)
