"""FP64 reference ray caster (ctypes wrapper around vr_oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the GPU
renderer.  The C source states every rule it implements; `brute.py` holds an
exact-rational renderer for tiny volumes that pins it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "vr_oracle.c")

FLAG_STOP, FLAG_COUNT, FLAG_CELL, FLAG_BRICK = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE FP64, OpenMP over rays)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Camera(C.Structure):
    _fields_ = [("kind", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("fovy_deg", C.c_double), ("half_w", C.c_double),
                ("half_h", C.c_double), ("full_w", C.c_int32), ("full_h", C.c_int32),
                ("tile_x0", C.c_int32), ("tile_y0", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("filter", C.c_int32), ("step", C.c_double),
                ("tau", C.c_double), ("eps_stop", C.c_double), ("eps_t", C.c_double),
                ("eps_pos", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        P, D, I64, I32 = C.c_void_p, C.c_double, C.c_int64, C.c_int32
        L.orc_render.argtypes = [P, I64, I64, I64, P, I32, D, D, P, P, P, I64, P, P, P, P, P, C.c_int]
        L.orc_render_bricked.argtypes = [P, I64, I64, I64, P, I32, D, D, P, P, I64, I64, P, I64, P, P, P, P,
                                         C.c_int]
        L.orc_backward.argtypes = [P, I64, I64, I64, P, I32, D, D, P, P, P, P, P, C.c_int]
        L.orc_ray.argtypes = [P, I64, I64, P, P]
        L.orc_basis.argtypes = [P, P, P, P]
        L.orc_lut.argtypes = [P, I32, D, D, D, P, P, P, P]
        L.orc_trilinear.argtypes = [P, P, P, P]
        L.orc_trilinear.restype = D
        L.orc_brick_key.argtypes = [P, I64, I64, I64, I64]
        L.orc_brick_key.restype = I64
        L.orc_ray_interval.argtypes = [P, I64, I64, I64, P, P, I64, I64, P, P, P, P, P]
        L.orc_depth.argtypes = [P, I64, I64, I64, P, I32, D, D, P, P, D, D, P, I64, P, P, P, P, C.c_int]
        L.orc_overlay.argtypes = [P, P, I64, D, D, P, D, P, P, C.c_int]
        _lib = L
    return _lib


def _cam(cam) -> _Camera:
    c = _Camera()
    c.kind = cam.kind
    for i in range(3):
        c.eye[i], c.target[i], c.up[i] = cam.eye[i], cam.target[i], cam.up[i]
    c.fovy_deg, c.half_w, c.half_h = cam.fovy_deg, cam.half_w, cam.half_h
    c.full_w, c.full_h = cam.full_w, cam.full_h
    c.tile_x0, c.tile_y0, c.tile_w, c.tile_h = cam.tile
    return c


def _params(mode, filt, step, tau, eps_stop, eps_t, eps_pos) -> _Params:
    p = _Params()
    p.mode = {"composite": 0, "mip": 1}[mode] if isinstance(mode, str) else int(mode)
    p.filter = {"trilinear": 0, "nearest": 1}[filt] if isinstance(filt, str) else int(filt)
    p.step, p.tau, p.eps_stop, p.eps_t, p.eps_pos = step, tau, eps_stop, eps_t, eps_pos
    return p


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _vol(vol):
    v = np.ascontiguousarray(vol, dtype=np.float32)
    nz, ny, nx = v.shape
    return v, nx, ny, nz


def render(vol, lut, cam, mode="composite", filt="trilinear", step=0.5, tau=0.99,
           pixels=None, eps_stop=1e-5, eps_t=1e-9, eps_pos=1e-7, threads=0):
    """Render (tile-local) pixels.  Returns dict with 'out', 'lo', 'hi' of shape
    (h, w, 4) / (h, w) for the full tile, or (n, 4) / (n,) for a pixel list,
    plus 'flags' and 'taken' (samples processed up to the stop)."""
    v, nx, ny, nz = _vol(vol)
    table = np.ascontiguousarray(lut.table, dtype=np.float32)
    c = _cam(cam)
    p = _params(mode, filt, step, tau, eps_stop, eps_t, eps_pos)
    ch = 1 if p.mode == 1 else 4
    if pixels is None:
        n = cam.tile[2] * cam.tile[3]
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pix.shape[0]
    out = np.zeros(n * ch)
    lo = np.zeros(n * ch)
    hi = np.zeros(n * ch)
    flags = np.zeros(n, np.int32)
    taken = np.zeros(n, np.int64)
    lib().orc_render(_ptr(v), nx, ny, nz, _ptr(table), table.shape[0], lut.vmin, lut.vmax,
                     C.byref(c), C.byref(p), _ptr(pix), n, _ptr(out), _ptr(lo), _ptr(hi),
                     _ptr(flags), _ptr(taken), threads)
    shp = (cam.tile[3], cam.tile[2]) if pixels is None else (n,)
    shp_c = shp + ((4,) if ch == 4 else ())
    return {"out": out.reshape(shp_c), "lo": lo.reshape(shp_c), "hi": hi.reshape(shp_c),
            "flags": flags.reshape(shp), "taken": taken.reshape(shp)}


def render_bricked(vol, lut, cam, brick, mode="composite", filt="trilinear", step=0.5, tau=0.99,
                   only_brick=-1, pixels=None, eps_stop=1e-5, eps_t=1e-9, eps_pos=1e-7, threads=0):
    """Bricked render (per-brick partials, "over" in key order), or the partial
    of one brick when only_brick >= 0.  Returns 'out', 'lo', 'hi' (candidate
    interval over flipped stop and count decisions; brick-face ties are
    flagged FLAG_BRICK but not widened) and 'flags'."""
    v, nx, ny, nz = _vol(vol)
    table = np.ascontiguousarray(lut.table, dtype=np.float32)
    c = _cam(cam)
    p = _params(mode, filt, step, tau, eps_stop, eps_t, eps_pos)
    ch = 1 if p.mode == 1 else 4
    if pixels is None:
        n = cam.tile[2] * cam.tile[3]
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pix.shape[0]
    out = np.zeros(n * ch)
    lo = np.zeros(n * ch)
    hi = np.zeros(n * ch)
    flags = np.zeros(n, np.int32)
    lib().orc_render_bricked(_ptr(v), nx, ny, nz, _ptr(table), table.shape[0], lut.vmin, lut.vmax,
                             C.byref(c), C.byref(p), int(brick), int(only_brick), _ptr(pix), n,
                             _ptr(out), _ptr(lo), _ptr(hi), _ptr(flags), threads)
    shp = (cam.tile[3], cam.tile[2]) if pixels is None else (n,)
    shp_c = shp + ((4,) if ch == 4 else ())
    return {"out": out.reshape(shp_c), "lo": lo.reshape(shp_c), "hi": hi.reshape(shp_c),
            "flags": flags.reshape(shp)}


def depth(vol, lut, cam, mode="composite", filt="trilinear", step=0.5, tau=0.99, level=0.5, pixels=None,
          eps_stop=1e-5, eps_t=1e-9, eps_pos=1e-7, eps_val=0.0, threads=0):
    """Per-pixel depth (ray parameter t, +inf for none): composite, the first
    sample after which A reaches `level`; MIP, the first sample equal to the
    maximum.  Returns 'out', 'lo', 'hi' (candidate depths over flipped
    decisions) and 'flags'."""
    v, nx, ny, nz = _vol(vol)
    table = np.ascontiguousarray(lut.table, dtype=np.float32)
    c = _cam(cam)
    p = _params(mode, filt, step, tau, eps_stop, eps_t, eps_pos)
    if pixels is None:
        n = cam.tile[2] * cam.tile[3]
        pix = None
        shp = (cam.tile[3], cam.tile[2])
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        n = pix.shape[0]
        shp = (n,)
    out, lo, hi = np.zeros(n), np.zeros(n), np.zeros(n)
    flags = np.zeros(n, np.int32)
    lib().orc_depth(_ptr(v), nx, ny, nz, _ptr(table), table.shape[0], lut.vmin, lut.vmax, C.byref(c),
                    C.byref(p), float(level), float(eps_val), _ptr(pix), n, _ptr(out), _ptr(lo), _ptr(hi),
                    _ptr(flags), threads)
    return {"out": out.reshape(shp), "lo": lo.reshape(shp), "hi": hi.reshape(shp), "flags": flags.reshape(shp)}


def overlay(cam, boxes, image, half_width=0.75, near=1e-3, depth=None, eps=1e-9, threads=0):
    """Wireframe boxes over a premultiplied RGBA tile.  boxes: (n, 10) =
    lo xyz, hi xyz, straight RGBA; image: (h, w, 4), not modified; depth:
    (h, w) float32 or None.  Returns (image with the overlay (FP64), flags)."""
    c = _cam(cam)
    b = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 10)
    img = np.array(image, dtype=np.float64, copy=True).reshape(cam.tile[3], cam.tile[2], 4)
    d = None if depth is None else np.ascontiguousarray(depth, dtype=np.float32).reshape(cam.tile[3], cam.tile[2])
    flags = np.zeros((cam.tile[3], cam.tile[2]), np.int32)
    lib().orc_overlay(C.byref(c), _ptr(b), b.shape[0], float(half_width), float(near), _ptr(d), float(eps),
                      _ptr(img), _ptr(flags), threads)
    return img, flags


def backward(vol, lut, cam, grad_out, step=0.5, tau=0.99, threads=0):
    """Adjoint of the composite render: (grad_lut (n,4), grad_vol (nz,ny,nx)), FP64."""
    v, nx, ny, nz = _vol(vol)
    table = np.ascontiguousarray(lut.table, dtype=np.float32)
    c = _cam(cam)
    p = _params(0, 0, step, tau, 0.0, 0.0, 0.0)
    g = np.ascontiguousarray(grad_out, dtype=np.float64).reshape(-1)
    assert g.size == cam.tile[2] * cam.tile[3] * 4
    gl = np.zeros(table.shape[0] * 4)
    gv = np.zeros(nx * ny * nz)
    lib().orc_backward(_ptr(v), nx, ny, nz, _ptr(table), table.shape[0], lut.vmin, lut.vmax,
                       C.byref(c), C.byref(p), _ptr(g), _ptr(gl), _ptr(gv), threads)
    return gl.reshape(-1, 4), gv.reshape(nz, ny, nx)


def ray(cam, col, row):
    """(origin, direction) of full-frame pixel (col, row), FP64."""
    o = np.zeros(3)
    d = np.zeros(3)
    lib().orc_ray(C.byref(_cam(cam)), int(col), int(row), _ptr(o), _ptr(d))
    return o, d


def basis(cam):
    f, r, u = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_basis(C.byref(_cam(cam)), _ptr(f), _ptr(r), _ptr(u))
    return f, r, u


def ray_interval(shape, cam, col, row, step=0.5):
    nz, ny, nx = shape
    o, d = np.zeros(3), np.zeros(3)
    t0, t1, n = C.c_double(), C.c_double(), C.c_int64()
    p = _params(0, 0, step, 1.0, 0.0, 0.0, 0.0)
    hit = lib().orc_ray_interval(None, nx, ny, nz, C.byref(_cam(cam)), C.byref(p), int(col), int(row),
                                 _ptr(o), _ptr(d), C.byref(t0), C.byref(t1), C.byref(n))
    return bool(hit), t0.value, t1.value, n.value, o, d


def lut_eval(lut, s):
    table = np.ascontiguousarray(lut.table, dtype=np.float32)
    rgba, dv = np.zeros(4), np.zeros(4)
    j, w = C.c_int32(), C.c_double()
    lib().orc_lut(_ptr(table), table.shape[0], lut.vmin, lut.vmax, float(s), _ptr(rgba),
                  C.byref(j), C.byref(w), _ptr(dv))
    return rgba, j.value, w.value, dv


def trilinear(vol, p):
    v, nx, ny, nz = _vol(vol)

    class _Scene(C.Structure):
        _fields_ = [("vol", C.c_void_p), ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                    ("lut", C.c_void_p), ("nlut", C.c_int32), ("vmin", C.c_double), ("vmax", C.c_double)]

    s = _Scene(v.ctypes.data, nx, ny, nz, None, 0, 0.0, 1.0)
    pos = np.asarray(p, dtype=np.float64)
    idx = np.zeros(8, np.int64)
    wt = np.zeros(8)
    val = lib().orc_trilinear(C.byref(s), _ptr(pos), _ptr(idx), _ptr(wt))
    return val, idx, wt


def brick_key(cam, B, bx, by, bz):
    return lib().orc_brick_key(C.byref(_cam(cam)), int(B), int(bx), int(by), int(bz))


def over(partials, order):
    """Front-to-back "over" of premultiplied RGBA partial images (each (h, w, 4))
    in the given order: C += (1 - A_acc) C_b, A likewise."""
    acc = np.zeros_like(np.asarray(partials[0], dtype=np.float64))
    for b in order:
        pb = np.asarray(partials[b], dtype=np.float64)
        acc = acc + (1.0 - acc[..., 3:4]) * pb
    return acc


def nthreads():
    return os.cpu_count() or 1
