"""Python binding of the HIP ray caster (libvrcube.so, include/vr.h).

Argument marshalling only: every step of rendering runs in the library's HIP
kernels.  PyTorch provides device memory (every buffer is a torch tensor the
binding allocates and keeps alive) and the HIP stream (the current torch
stream).  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; VRCUBE_LIB names another build of the same sources
LIB_PATH = os.environ.get("VRCUBE_LIB") or os.path.join(HERE, "libvrcube.so")

OK, EINVAL, ESTATE, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
MODES = {"composite": 0, "mip": 1}
FILTERS = {"trilinear": 0, "nearest": 1}
TRANS = {"auto": 0, "product": 1, "log": 2}
CHECKPOINT_INTERVAL = 8     # VR_CHECKPOINT_INTERVAL of include/vr.h


class Camera(C.Structure):
    _fields_ = [("kind", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("fovy_deg", C.c_double), ("half_w", C.c_double),
                ("half_h", C.c_double), ("full_w", C.c_int32), ("full_h", C.c_int32),
                ("tile_x0", C.c_int32), ("tile_y0", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("filter", C.c_int32), ("step", C.c_double),
                ("ert_alpha", C.c_float), ("transmittance", C.c_int32),
                ("save_for_backward", C.c_int32)]


class Partial(C.Structure):
    _fields_ = [("data", C.c_void_p), ("x0", C.c_int32), ("y0", C.c_int32), ("w", C.c_int32),
                ("h", C.c_int32), ("brick_id", C.c_int32), ("pad", C.c_int32)]


class View(C.Structure):
    _fields_ = [("cam", Camera), ("lut_index", C.c_int32), ("pad", C.c_int32), ("out", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("packet_w", C.c_int32), ("packet_h", C.c_int32), ("waves_per_group", C.c_int32),
                ("unroll", C.c_int32), ("persistent_groups", C.c_int32), ("path", C.c_int32),
                ("lds_kib", C.c_int32), ("slab_max", C.c_int32), ("copy", C.c_int32),
                ("order", C.c_int32)]


# (name, restype, argtypes) of every exported entry point
P, I32, I64, F32, D = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
SIGNATURES = [
    ("vr_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    ("vr_destroy", C.c_int, [P]),
    ("vr_last_error", C.c_char_p, [P]),
    ("vr_debug_bounds_violations", C.c_int64, [P]),
    ("vr_version", C.c_char_p, []),
    ("vr_volume_bytes", I64, [I64, I64, I64, I32, I32, I32]),
    ("vr_load_volume", C.c_int, [P, P, I64, I64, I64, I32, I32, I32, P, I64, P]),
    ("vr_describe_volume", C.c_int, [P, I64, I64, I64, I32, I32, I32, P, I64]),
    ("vr_load_slab", C.c_int, [P, P, I64, I64, P]),
    ("vr_set_transfer_function", C.c_int, [P, P, I32, F32, F32]),
    ("vr_set_camera", C.c_int, [P, C.POINTER(Camera)]),
    ("vr_render_workspace_bytes", I64, [P, C.POINTER(RenderParams)]),
    ("vr_render", C.c_int, [P, C.POINTER(RenderParams), P, P, I64, P]),
    ("vr_render_depth", C.c_int, [P, C.POINTER(RenderParams), C.c_float, P, P]),
    ("vr_overlay_boxes", C.c_int, [P, P, I32, C.c_float, P, P, P]),
    ("vr_brick_bytes", I64, [I64, I64, I64, I32, I32]),
    ("vr_pack_bricks_host", C.c_int, [P, I64, I64, I64, I32, I32, P, I64, I32]),
    ("vr_describe_streamed_volume", C.c_int, [P, I64, I64, I64, I32, I32, P, I64, P, I64]),
    ("vr_stream_stats", C.c_int, [P, P, P, P]),
    ("vr_pyramid_bytes", I64, [I32, I32, I32, P]),
    ("vr_build_pyramid", C.c_int, [P, P, I32, I32, I32, P, I64, P]),
    ("vr_write_pyramid_tiff", C.c_int, [C.c_char_p, P, I32, I32, I32, I32]),
    ("vr_render_noalloc_max_bytes", I64, []),
    ("vr_render_noalloc", C.c_int, [P, C.POINTER(RenderParams), P, P]),
    ("vr_count_samples", C.c_int, [P, C.POINTER(RenderParams), P, P]),
    ("vr_touched_bitmap_bytes", I64, [P]),
    ("vr_mark_touched_blocks", C.c_int, [P, C.POINTER(RenderParams), P, I64, P]),
    ("vr_bricks_pool_bytes", I64, [P, C.POINTER(RenderParams)]),
    ("vr_render_bricks", C.c_int, [P, C.POINTER(RenderParams), C.POINTER(Partial), I32,
                                   C.POINTER(I32), P, I64, P]),
    ("vr_brick_order", C.c_int, [P, C.POINTER(Partial), I32, C.POINTER(I32)]),
    ("vr_composite_workspace_bytes", I64, [I32]),
    ("vr_composite_bricks", C.c_int, [P, C.POINTER(RenderParams), C.POINTER(Partial),
                                      C.POINTER(I32), I32, P, P, I64, P]),
    ("vr_render_backward", C.c_int, [P, C.POINTER(RenderParams), P, P, I64, P, P, P]),
    ("vr_batch_workspace_bytes", I64, [P, C.POINTER(View), I32]),
    ("vr_render_batch", C.c_int, [P, C.POINTER(RenderParams), C.POINTER(View), I32, P, I32, I32,
                                  F32, F32, P, I64, I32, P]),
    ("vr_batch_graph_captures", C.c_int, [P]),
    ("vr_autotune_batch", C.c_int, [P, C.POINTER(RenderParams), C.POINTER(View), I32, P, I32, I32, F32, F32,
                                    P, I64, C.c_char_p, P]),
    ("vr_get_tuning", C.c_int, [P, C.POINTER(Tuning)]),
    ("vr_set_tuning", C.c_int, [P, C.POINTER(Tuning)]),
    ("vr_autotune", C.c_int, [P, C.POINTER(RenderParams), P, P, I64, C.c_char_p, P]),
]

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class VRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vr error {code}: {msg}")
        self.code = code


def check(rc, ctx=None):
    if rc < 0:
        msg = lib().vr_last_error(ctx)
        raise VRError(int(rc), msg.decode() if msg else "")
    return rc


def camera_struct(cam) -> Camera:
    c = Camera()
    c.kind = int(cam.kind)
    for i in range(3):
        c.eye[i], c.target[i], c.up[i] = cam.eye[i], cam.target[i], cam.up[i]
    c.fovy_deg, c.half_w, c.half_h = cam.fovy_deg, cam.half_w, cam.half_h
    c.full_w, c.full_h = int(cam.full_w), int(cam.full_h)
    c.tile_x0, c.tile_y0, c.tile_w, c.tile_h = (int(v) for v in cam.tile)
    return c


def params_struct(mode="composite", filt="trilinear", step=0.5, ert=0.99, trans="auto",
                  save=False) -> RenderParams:
    p = RenderParams()
    p.mode = MODES[mode]
    p.filter = FILTERS[filt]
    p.step = float(step)
    p.ert_alpha = float(ert)
    p.transmittance = TRANS[trans]
    p.save_for_backward = 1 if save else 0
    return p


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def pack_bricks_host(cube, storage="f32", brick=256, out=None, threads=0):
    """Pack a float32 (nz, ny, nx) host cube (numpy array or memmap) into the
    bricked layout in host memory: `out` (uint8 CPU tensor, pinned for
    asynchronous copies) or a new pinned tensor.  Returns it."""
    src = np.ascontiguousarray(cube, dtype=np.float32)
    nz, ny, nx = src.shape
    nbytes = int(lib().vr_volume_bytes(nx, ny, nz, DTYPES[storage], int(brick), 1))
    if nbytes < 0:
        raise VRError(nbytes, "invalid volume size")
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    assert out.device.type == "cpu" and out.numel() >= nbytes
    rc = lib().vr_pack_bricks_host(src.ctypes.data_as(C.c_void_p), nx, ny, nz, DTYPES[storage], int(brick),
                                   C.c_void_p(out.data_ptr()), out.numel(), int(threads))
    if rc != 0:
        raise VRError(rc, lib().vr_last_error(None).decode())
    return out


def pyramid_levels(pyr, dims):
    """Split a pyramid buffer (host or device uint8) into (h_l, w_l, 4) levels."""
    out, off = [], 0
    for h, w in dims:
        out.append(pyr[off:off + h * w * 4].reshape(h, w, 4))
        off += h * w * 4
    return out


def write_pyramid_tiff(path, pyramid, w, h, tile=256, bigtiff=False):
    """Write a pyramid (uint8, host: numpy array or CPU tensor) as a pyramidal
    tiled TIFF through the library's host writer."""
    buf = pyramid.cpu().numpy() if torch.is_tensor(pyramid) else np.asarray(pyramid)
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    rc = lib().vr_write_pyramid_tiff(os.fsencode(path), buf.ctypes.data_as(C.c_void_p), int(w), int(h), int(tile),
                                     1 if bigtiff else 0)
    if rc != 0:
        raise VRError(rc, lib().vr_last_error(None).decode())


class Renderer:
    """One rendering context on one GPU.  Holds references to every tensor the
    library borrows (volume storage, transfer table)."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        check(lib().vr_create(C.byref(h), device))
        self.ctx = h
        self.storage = None
        self.lut = None
        self.shape = None
        self.cam = None
        # bumped by every call that changes what a render reads (volume,
        # table, camera), so a caller can tell whether its state still holds
        self.generation = 0

    def close(self):
        if self.ctx:
            lib().vr_destroy(self.ctx)
            self.ctx = None

    def debug_bounds_violations(self):
        """Index-range violations counted since the last call (debug library
        only; a release library raises VRError with VR_EUNSUPPORTED)."""
        return int(self._check(lib().vr_debug_bounds_violations(self.ctx)))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        return check(rc, self.ctx)

    # ---- volume --------------------------------------------------------
    @staticmethod
    def default_orientations(shape, brick):
        return 3 if brick <= 0 or all(brick >= d for d in shape) else 1

    def load_volume(self, vol, storage="f32", brick=0, orientations=None):
        """vol: float32 (nz, ny, nx) cuda tensor (or numpy array, uploaded).
        orientations: 3 keeps x-, y- and z-fastest copies (one-brick layouts;
        the default there; with FP32 storage also the line copy the
        object-order MIP reads), 1 the x-fastest copy only."""
        if not torch.is_tensor(vol):
            vol = torch.from_numpy(vol)
        vol = vol.to(self.device, torch.float32).contiguous()
        nz, ny, nx = vol.shape
        if orientations is None:
            orientations = self.default_orientations(vol.shape, int(brick))
        nbytes = int(lib().vr_volume_bytes(nx, ny, nz, DTYPES[storage], int(brick), int(orientations)))
        if nbytes < 0:
            raise VRError(nbytes, "invalid volume size")
        self.storage = None
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(lib().vr_load_volume(self.ctx, _ptr(vol), nx, ny, nz, DTYPES[storage], int(brick),
                                         int(orientations), _ptr(self.storage), nbytes, _stream()))
        self.orientations = int(orientations)
        self.shape = (nz, ny, nx)
        self.brick = int(brick)
        self.storage_dtype = storage
        self.generation += 1
        return self.storage

    def describe_volume(self, shape, storage="f32", brick=0, orientations=None):
        nz, ny, nx = shape
        if orientations is None:
            orientations = self.default_orientations(shape, int(brick))
        nbytes = int(lib().vr_volume_bytes(nx, ny, nz, DTYPES[storage], int(brick), int(orientations)))
        if nbytes < 0:
            raise VRError(nbytes, "invalid volume size")
        self.storage = None
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(lib().vr_describe_volume(self.ctx, nx, ny, nz, DTYPES[storage], int(brick),
                                             int(orientations), _ptr(self.storage), nbytes))
        self.orientations = int(orientations)
        self.shape = tuple(shape)
        self.brick = int(brick)
        self.storage_dtype = storage
        self.generation += 1

    def describe_streamed_volume(self, shape, host_bricks, storage="f32", brick=256, cache_slots=None,
                                 cache=None):
        """Render from bricks packed in host memory (pack_bricks_host)
        through a device cache of `cache_slots` bricks (or the given cache
        tensor)."""
        nz, ny, nx = shape
        bb = int(lib().vr_brick_bytes(nx, ny, nz, DTYPES[storage], int(brick)))
        if bb < 0:
            raise VRError(bb, "invalid volume size")
        if cache is None:
            cache = torch.empty(bb * int(cache_slots), dtype=torch.uint8, device=self.device)
        self.storage = None
        self._check(lib().vr_describe_streamed_volume(self.ctx, nx, ny, nz, DTYPES[storage], int(brick),
                                                      C.c_void_p(host_bricks.data_ptr()), host_bricks.numel(),
                                                      _ptr(cache), cache.numel()))
        self.host_bricks = host_bricks
        self.storage = cache
        self.orientations = 1
        self.shape = tuple(shape)
        self.brick = int(brick)
        self.storage_dtype = storage
        self.generation += 1

    def stream_stats(self):
        """(bricks copied from host, cache hits, cache slots) so far."""
        a, b, n = C.c_int64(), C.c_int64(), C.c_int32()
        self._check(lib().vr_stream_stats(self.ctx, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def load_slab(self, slab, z0):
        slab = slab.to(self.device, torch.float32).contiguous()
        self._check(lib().vr_load_slab(self.ctx, _ptr(slab), int(z0), int(slab.shape[0]), _stream()))
        self.generation += 1

    # ---- table / camera ------------------------------------------------
    def set_transfer_function(self, table, vmin, vmax):
        if not torch.is_tensor(table):
            table = torch.from_numpy(table)
        table = table.to(self.device, torch.float32).contiguous()
        self._check(lib().vr_set_transfer_function(self.ctx, _ptr(table), int(table.shape[0]),
                                                   float(vmin), float(vmax)))
        self.lut = table
        self.lut_range = (float(vmin), float(vmax))
        self.generation += 1

    def set_lut(self, lut):
        self.set_transfer_function(lut.table, lut.vmin, lut.vmax)

    def set_camera(self, cam):
        c = camera_struct(cam)
        self._check(lib().vr_set_camera(self.ctx, C.byref(c)))
        self.cam = cam
        self.generation += 1

    # ---- render --------------------------------------------------------
    def workspace_bytes(self, **kw):
        p = params_struct(**kw)
        return int(self._check(lib().vr_render_workspace_bytes(self.ctx, C.byref(p))))

    def render(self, mode="composite", filt="trilinear", step=0.5, ert=0.99, trans="auto",
               out=None, save=False, workspace=None):
        p = params_struct(mode, filt, step, ert, trans, save)
        w, h = self.cam.tile[2], self.cam.tile[3]
        shape = (h, w, 4) if mode == "composite" else (h, w)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        ws_bytes = int(self._check(lib().vr_render_workspace_bytes(self.ctx, C.byref(p))))
        if ws_bytes > 0 and (workspace is None or workspace.numel() < ws_bytes):
            workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        self._check(lib().vr_render(self.ctx, C.byref(p), _ptr(out),
                                    _ptr(workspace) if ws_bytes > 0 else None, ws_bytes, _stream()))
        if save:
            return out, workspace
        return out

    def render_noalloc(self, mode="composite", filt="trilinear", step=0.5, ert=0.99, trans="auto", out=None):
        """render() through vr_render_noalloc: the library's fixed scratch
        instead of a workspace (no device allocation inside the call)."""
        p = params_struct(mode, filt, step, ert, trans, False)
        w, h = self.cam.tile[2], self.cam.tile[3]
        shape = (h, w, 4) if mode == "composite" else (h, w)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        self._check(lib().vr_render_noalloc(self.ctx, C.byref(p), _ptr(out), _stream()))
        return out

    def render_depth(self, mode="composite", filt="trilinear", step=0.5, ert=0.99, trans="auto", level=0.5,
                     out=None):
        """Per-pixel depth (ray parameter t, +inf for none) of the render
        with these settings: composite, where the opacity first reaches
        `level`; MIP, the first maximum sample."""
        p = params_struct(mode, filt, step, ert, trans, False)
        w, h = self.cam.tile[2], self.cam.tile[3]
        if out is None:
            out = torch.empty((h, w), dtype=torch.float32, device=self.device)
        self._check(lib().vr_render_depth(self.ctx, C.byref(p), float(level), _ptr(out), _stream()))
        return out

    def overlay_boxes(self, boxes, image, half_width=0.75, depth=None):
        """Draw catalogue boxes ((n, 10) float32: lo xyz, hi xyz, straight
        RGBA) as wireframes over `image` (the current view's (h, w, 4)
        premultiplied tile, modified in place), hiding edges behind `depth`."""
        if not torch.is_tensor(boxes):
            boxes = torch.from_numpy(np.ascontiguousarray(boxes, dtype=np.float32))
        b = boxes.to(self.device, torch.float32).contiguous()
        assert b.ndim == 2 and b.shape[1] == 10
        d = None if depth is None else depth.to(self.device, torch.float32).contiguous()
        self._check(lib().vr_overlay_boxes(self.ctx, _ptr(b), int(b.shape[0]), float(half_width), _ptr(d),
                                           _ptr(image), _stream()))
        return image

    def build_pyramid(self, image, tile=256):
        """Display pyramid of a premultiplied RGBA (h, w, 4) float image:
        (uint8 tensor of vr_pyramid_bytes, list of (h_l, w_l) per level)."""
        img = image.to(self.device, torch.float32).contiguous()
        h, w = int(img.shape[0]), int(img.shape[1])
        levels = C.c_int32()
        nbytes = int(lib().vr_pyramid_bytes(w, h, int(tile), C.byref(levels)))
        if nbytes < 0:
            raise VRError(nbytes, lib().vr_last_error(None).decode())
        dst = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(lib().vr_build_pyramid(self.ctx, _ptr(img), w, h, int(tile), _ptr(dst), nbytes, _stream()))
        dims = []
        for _ in range(levels.value):
            dims.append((h, w))
            h, w = (h + 1) // 2, (w + 1) // 2
        return dst, dims

    def render_backward(self, grad_out, workspace, grad_lut=None, grad_vol=None, step=0.5, ert=0.99,
                        trans="auto"):
        """Accumulate dL/d(table) and dL/d(voxels) given dL/d(image) and the
        workspace of a render(save=True) with the same settings."""
        p = params_struct("composite", "trilinear", step, ert, trans, True)
        g = grad_out.to(self.device, torch.float32).contiguous()
        self._check(lib().vr_render_backward(self.ctx, C.byref(p), _ptr(g), _ptr(workspace), workspace.numel(),
                                             _ptr(grad_lut), _ptr(grad_vol), _stream()))
        return grad_lut, grad_vol

    def count_samples(self, mode="composite", filt="trilinear", step=0.5, ert=0.99, trans="auto"):
        p = params_struct(mode, filt, step, ert, trans)
        w, h = self.cam.tile[2], self.cam.tile[3]
        counts = torch.empty((h, w), dtype=torch.int32, device=self.device)
        self._check(lib().vr_count_samples(self.ctx, C.byref(p), _ptr(counts), _stream()))
        return counts

    def touched_blocks(self, mode="composite", filt="trilinear", step=0.5, ert=0.99):
        """Number of 8^3 voxel blocks touched by taken samples' footprints."""
        p = params_struct(mode, filt, step, ert)
        nbytes = int(self._check(lib().vr_touched_bitmap_bytes(self.ctx)))
        bits = torch.zeros(nbytes // 4, dtype=torch.int32, device=self.device)
        self._check(lib().vr_mark_touched_blocks(self.ctx, C.byref(p), _ptr(bits), nbytes, _stream()))
        b = bits.view(torch.uint8).cpu()
        return int(torch.bitwise_and(b.unsqueeze(-1) >> torch.arange(8, dtype=torch.uint8), 1).sum())

    # ---- tuning ----------------------------------------------------------
    def get_tuning(self):
        t = Tuning()
        self._check(lib().vr_get_tuning(self.ctx, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = Tuning(**cur)
        self._check(lib().vr_set_tuning(self.ctx, C.byref(t)))

    # ---- bricks and sort-last compositing ---------------------------------
    def render_bricks(self, mode="composite", filt="trilinear", step=0.5, ert=0.99, pool=None):
        """Per-brick partial images of the current viewport.  Returns (parts,
        pool): parts is a ctypes array of Partial (device pointers into pool)."""
        p = params_struct(mode, filt, step, ert)
        need = int(self._check(lib().vr_bricks_pool_bytes(self.ctx, C.byref(p))))
        if pool is None or pool.numel() < need:
            pool = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        nb = 1
        for d, b in zip(self.shape, [self.brick] * 3):
            nb *= (d + b - 1) // b if b > 0 else 1
        parts = (Partial * max(nb, 1))()
        n = C.c_int32()
        self._check(lib().vr_render_bricks(self.ctx, C.byref(p), parts, len(parts), C.byref(n), _ptr(pool),
                                           pool.numel(), _stream()))
        return parts[:n.value], pool

    def brick_order(self, parts):
        n = len(parts)
        arr = (Partial * max(n, 1))(*parts)
        order = (C.c_int32 * max(n, 1))()
        self._check(lib().vr_brick_order(self.ctx, arr, n, order))
        return list(order[:n])

    def composite_bricks(self, parts, order, mode="composite", out=None, workspace=None):
        p = params_struct(mode)
        n = len(parts)
        w, h = self.cam.tile[2], self.cam.tile[3]
        if out is None:
            out = torch.empty((h, w, 4) if mode == "composite" else (h, w), dtype=torch.float32,
                              device=self.device)
        need = int(lib().vr_composite_workspace_bytes(n))
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        arr = (Partial * max(n, 1))(*parts)
        order_arr = (C.c_int32 * max(n, 1))(*order)
        self._check(lib().vr_composite_bricks(self.ctx, C.byref(p), arr, order_arr, n, _ptr(out),
                                              _ptr(workspace), workspace.numel(), _stream()))
        return out

    def render_bricked(self, mode="composite", filt="trilinear", step=0.5, ert=0.99):
        """Bricked render: per-brick partials, then the sort-last composite."""
        parts, pool = self.render_bricks(mode, filt, step, ert)
        order = self.brick_order(parts)
        out = self.composite_bricks(parts, order, mode)
        self._keep = pool
        return out

    # ---- batches and tuning ----------------------------------------------------
    def _views(self, cams, outs, lut_index):
        arr = (View * len(cams))()
        for i, (c, o) in enumerate(zip(cams, outs)):
            arr[i].cam = camera_struct(c)
            arr[i].lut_index = int(lut_index[i])
            arr[i].out = o.data_ptr()
        return arr

    def render_batch(self, cams, luts=None, lut_index=None, mode="composite", filt="trilinear", step=0.5, ert=0.99,
                     trans="auto", outs=None, use_graph=False, workspace=None, stream=None):
        """Render many views in one persistent launch.  luts: (n_luts, n, 4)
        float32 cuda tensor (all over the range given to set_lut_range) or a
        list of synth.Lut; returns the list of output tensors."""
        p = params_struct(mode, filt, step, ert, trans)
        n = len(cams)
        if outs is None:
            outs = [torch.empty((c.tile[3], c.tile[2], 4) if mode == "composite" else (c.tile[3], c.tile[2]),
                                dtype=torch.float32, device=self.device) for c in cams]
        if luts is None:
            luts_t, vmin, vmax = self.lut.unsqueeze(0), *self.lut_range
        elif isinstance(luts, tuple) and len(luts) == 3 and torch.is_tensor(luts[0]):
            luts_t, vmin, vmax = luts
        else:
            luts_t, vmin, vmax = self.stack_luts(luts)
        if lut_index is None:
            lut_index = list(range(n)) if luts_t.shape[0] == n else [0] * n
        views = self._views(cams, outs, lut_index)
        need = int(self._check(lib().vr_batch_workspace_bytes(self.ctx, views, n)))
        if workspace is None:
            workspace = getattr(self, "_batch_ws", None)   # reused: graphs replay on the same workspace
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1 << 16), dtype=torch.uint8, device=self.device)
            self._batch_ws = workspace
        self._batch_keep = (luts_t, workspace, outs)
        s = C.c_void_p(stream.cuda_stream) if stream is not None else _stream()
        self._check(lib().vr_render_batch(self.ctx, C.byref(p), views, n, _ptr(luts_t), int(luts_t.shape[0]),
                                          int(luts_t.shape[1]), float(vmin), float(vmax), _ptr(workspace),
                                          workspace.numel(), 1 if use_graph else 0, s))
        return outs

    def stack_luts(self, luts):
        """(tensor (n_luts, n, 4) on the device, vmin, vmax) from a list of synth.Lut."""
        t = torch.stack([torch.from_numpy(l.table) for l in luts]).to(self.device).contiguous()
        return t, float(luts[0].vmin), float(luts[0].vmax)

    def graph_captures(self):
        return int(lib().vr_batch_graph_captures(self.ctx))

    def autotune(self, mode="composite", filt="trilinear", step=0.5, ert=0.99, cache_path=None):
        p = params_struct(mode, filt, step, ert)
        w, h = self.cam.tile[2], self.cam.tile[3]
        out = torch.empty((h, w, 4) if mode == "composite" else (h, w), dtype=torch.float32, device=self.device)
        cp = cache_path.encode() if cache_path else None
        self._check(lib().vr_autotune(self.ctx, C.byref(p), _ptr(out), None, 0, cp, _stream()))
        return self.get_tuning()

    def autotune_batch(self, cams, luts, lut_index=None, mode="composite", filt="trilinear", step=0.5, ert=0.99,
                       cache_path=None):
        p = params_struct(mode, filt, step, ert)
        n = len(cams)
        outs = [torch.empty((c.tile[3], c.tile[2], 4) if mode == "composite" else (c.tile[3], c.tile[2]),
                            dtype=torch.float32, device=self.device) for c in cams]
        luts_t = torch.stack([torch.from_numpy(l.table) for l in luts]).to(self.device).contiguous()
        if lut_index is None:
            lut_index = list(range(n))
        views = self._views(cams, outs, lut_index)
        need = int(self._check(lib().vr_batch_workspace_bytes(self.ctx, views, n)))
        ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        cp = cache_path.encode() if cache_path else None
        self._check(lib().vr_autotune_batch(self.ctx, C.byref(p), views, n, _ptr(luts_t), int(luts_t.shape[0]),
                                            int(luts_t.shape[1]), float(luts[0].vmin), float(luts[0].vmax),
                                            _ptr(ws), ws.numel(), cp, _stream()))
        torch.cuda.synchronize()
        return self.get_tuning()
