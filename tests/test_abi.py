"""C-ABI checks that need no GPU: the library loads, exports every function
include/vr.h declares, and rejects bad arguments and wrong states with the
documented codes (on a host-only context, device = -1)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1012_2909_amd import vr
    if not os.path.exists(vr.LIB_PATH):
        pytest.skip("library not built")
    return vr, vr.lib()


def header_functions():
    src = open(os.path.join(ROOT, "include", "vr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    vr, L = _lib()
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    # the binding's signature table covers the header exactly
    assert sorted(n for n, _, _ in vr.SIGNATURES) == names


def test_checkpoint_interval_matches_header():
    from paper_1012_2909_amd import vr
    src = open(os.path.join(ROOT, "include", "vr.h")).read()
    assert int(re.search(r"#define VR_CHECKPOINT_INTERVAL (\d+)", src).group(1)) == vr.CHECKPOINT_INTERVAL


def test_version():
    vr, L = _lib()
    assert b"gfx950" in L.vr_version()


def test_volume_bytes_is_pure_and_matches_layout():
    vr, L = _lib()
    # one brick: (n+2) per axis, rows padded to a multiple of 8 elements
    assert L.vr_volume_bytes(64, 64, 64, 0, 0, 1) == 72 * 66 * 66 * 4
    assert L.vr_volume_bytes(64, 64, 64, 1, 0, 1) == 72 * 66 * 66 * 2
    # 2048x2048x4096 in 256^3 bricks: 1024 bricks of 258^3 (rows of 264)
    assert L.vr_volume_bytes(2048, 2048, 4096, 0, 256, 1) == 1024 * 264 * 258 * 258 * 4
    assert L.vr_volume_bytes(2048, 2048, 4096, 2, 256, 1) == 1024 * 264 * 258 * 258 * 2
    # ragged: 100 = 3 bricks of edge 40 along x (last one partial, stored full)
    assert L.vr_volume_bytes(100, 40, 40, 0, 40, 1) == 3 * 48 * 42 * 42 * 4
    for _ in range(3):
        assert L.vr_volume_bytes(1024, 1024, 2048, 0, 0, 1) == 1032 * 1026 * 2050 * 4
    assert L.vr_volume_bytes(0, 4, 4, 0, 0, 1) < 0
    assert L.vr_volume_bytes(4, 4, 4, 7, 0, 1) < 0
    # three orientation copies: x-, y-, z-fastest, each rounded to 256 bytes
    def r8(n):
        return (n + 2 + 7) // 8 * 8
    c0 = r8(64) * 50 * 40
    c1 = r8(48) * 40 * 66
    c2 = r8(38) * 66 * 50
    a = lambda e: (e + 127) // 128 * 128
    # FP32 with three copies adds the line copy: 31-element steps along x in 32-element lines
    lines = 40 * 50 * ((64 + 2 + 30) // 31) * 32
    assert L.vr_volume_bytes(64, 48, 38, 0, 0, 3) == (a(a(c0) + a(c1) + c2) + lines) * 4
    assert L.vr_volume_bytes(64, 48, 38, 1, 0, 3) == (a(c0) + a(c1) + c2) * 2
    assert L.vr_volume_bytes(64, 48, 38, 0, 16, 3) < 0        # copies need one brick
    assert L.vr_volume_bytes(64, 48, 38, 0, 0, 2) < 0


@pytest.fixture()
def hctx():
    vr, L = _lib()
    h = C.c_void_p()
    assert L.vr_create(C.byref(h), -1) == 0
    yield vr, L, h
    L.vr_destroy(h)


def _cam(vr, **kw):
    from paper_1012_2909_amd import synth
    cam = synth.camera_axis_z()
    for k, v in kw.items():
        setattr(cam, k, v)
    return vr.camera_struct(cam)


def test_state_errors(hctx):
    vr, L, h = hctx
    p = vr.params_struct()
    out = C.c_void_p(0x1000)
    assert L.vr_render(h, C.byref(p), out, None, 0, None) == vr.ESTATE
    assert b"volume" in L.vr_last_error(h)
    assert L.vr_load_slab(h, out, 0, 1, None) == vr.ESTATE
    assert L.vr_render_workspace_bytes(h, C.byref(p)) == vr.ESTATE
    assert L.vr_touched_bitmap_bytes(h) == vr.ESTATE


def test_argument_errors(hctx):
    vr, L, h = hctx
    buf = C.c_void_p(0x1000)
    # volume
    assert L.vr_describe_volume(h, 64, 64, 64, 0, 0, 1, None, 1 << 30) == vr.EINVAL
    assert L.vr_describe_volume(h, 64, 64, 64, 0, 0, 1, buf, 100) == vr.ENOMEM
    assert L.vr_describe_volume(h, -1, 64, 64, 0, 0, 1, buf, 1 << 30) == vr.EINVAL
    assert L.vr_describe_volume(h, 64, 64, 64, 3, 0, 1, buf, 1 << 30) == vr.EINVAL
    # a single brick of more than 2^32 voxels is refused
    assert L.vr_describe_volume(h, 2048, 2048, 4096, 0, 0, 1, buf, 1 << 62) == vr.EUNSUPPORTED
    assert L.vr_describe_volume(h, 64, 64, 64, 0, 0, 1, buf, 72 * 66 * 66 * 4) == vr.OK
    assert L.vr_load_slab(h, None, 0, 64, None) == vr.EINVAL
    assert L.vr_load_slab(h, buf, 60, 8, None) == vr.EINVAL
    assert L.vr_load_slab(h, buf, 0, 64, None) == vr.EDEVICE      # host-only context
    # table
    assert L.vr_set_transfer_function(h, buf, 1, 0.0, 1.0) == vr.EINVAL
    assert L.vr_set_transfer_function(h, buf, 2048, 0.0, 1.0) == vr.EINVAL
    assert L.vr_set_transfer_function(h, buf, 256, 1.0, 1.0) == vr.EINVAL
    assert L.vr_set_transfer_function(h, None, 256, 0.0, 1.0) == vr.EINVAL
    assert L.vr_set_transfer_function(h, buf, 256, -3.0, 10.0) == vr.OK
    # camera
    assert L.vr_set_camera(h, None) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr, kind=5))) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr, tile=(0, 0, 300, 10)))) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr, tile=(250, 0, 10, 10)))) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr, up=(0.0, 0.0, 1.0)))) == vr.EINVAL     # up parallel to view
    assert L.vr_set_camera(h, C.byref(_cam(vr, target=(32.0, 32.0, -1.0)))) == vr.EINVAL  # eye == target
    assert L.vr_set_camera(h, C.byref(_cam(vr, half_w=0.0))) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr, kind=1, fovy_deg=180.0))) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr, eye=(float("nan"), 0.0, 0.0)))) == vr.EINVAL
    assert L.vr_set_camera(h, C.byref(_cam(vr))) == vr.OK
    # tuning
    t = vr.Tuning(7, 9, 4, 1, 4, 0, 48, 16, -1, 1)
    assert L.vr_set_tuning(h, C.byref(t)) == vr.EINVAL
    t = vr.Tuning(16, 4, 2, 2, 4, 1, 32, 8, 2, 0)
    assert L.vr_set_tuning(h, C.byref(t)) == vr.OK
    t2 = vr.Tuning()
    assert L.vr_get_tuning(h, C.byref(t2)) == vr.OK and (t2.packet_w, t2.waves_per_group) == (16, 2)
    # LDS budget: 0 (automatic per view) or 8..144 KiB; tile orders 0..3
    for kib, ok in [(0, True), (8, True), (144, True), (4, False), (160, False), (-1, False)]:
        t = vr.Tuning(16, 4, 4, 1, 4, 2, kib, 16, -1, 1)
        assert (L.vr_set_tuning(h, C.byref(t)) == vr.OK) == ok, kib
    for order, ok in [(0, True), (2, True), (3, True), (4, False)]:
        t = vr.Tuning(16, 4, 4, 1, 4, 2, 64, 16, -1, order)
        assert (L.vr_set_tuning(h, C.byref(t)) == vr.OK) == ok, order
    # the LDS-staged path runs 4- or 8-wave groups only
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(16, 4, 2, 1, 4, 2, 64, 16, -1, 1))) == vr.EINVAL
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(16, 4, 8, 1, 4, 2, 64, 16, -1, 1))) == vr.OK
    # the compacting path (3) runs groups of at most 4 waves, shares of 1..32 packets per wave;
    # path 4 is MIP in object order; no path 5
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(16, 4, 4, 2, 8, 3, 0, 16, -1, 1))) == vr.OK
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(8, 8, 1, 4, 32, 3, 0, 16, -1, 1))) == vr.OK
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(16, 4, 8, 2, 4, 3, 0, 16, -1, 1))) == vr.EINVAL
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(16, 4, 4, 2, 4, 4, 0, 16, -1, 1))) == vr.OK
    assert L.vr_set_tuning(h, C.byref(vr.Tuning(16, 4, 4, 2, 4, 5, 0, 16, -1, 1))) == vr.EINVAL


def test_params_errors(hctx):
    vr, L, h = hctx
    buf = C.c_void_p(0x1000)
    assert L.vr_describe_volume(h, 64, 64, 64, 0, 0, 1, buf, 72 * 66 * 66 * 4) == vr.OK
    assert L.vr_set_camera(h, C.byref(_cam(vr))) == vr.OK
    for bad in [dict(step=0.0), dict(step=-1.0), dict(ert=0.0)]:
        p = vr.params_struct(**bad)
        assert L.vr_count_samples(h, C.byref(p), buf, None) in (vr.EINVAL, vr.ESTATE)
    p = vr.params_struct()
    p.mode = 9
    assert L.vr_render(h, C.byref(p), buf, None, 0, None) in (vr.EINVAL, vr.ESTATE)


def test_null_context():
    vr, L = _lib()
    assert L.vr_create(None, 0) == vr.EINVAL
    p = vr.params_struct()
    assert L.vr_render(None, C.byref(p), None, None, 0, None) == vr.EINVAL
    assert L.vr_last_error(None)
