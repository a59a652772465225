"""Seeded synthetic inputs: spectral cubes, transfer-function tables, cameras.

This module is shared by the GPU path, the tests and the benchmark.  It holds
no rendering arithmetic at all: it only draws numbers.  The paper's own cubes
(HIPASS southern sky, 1721x1721x1025 float32; the Ursa Major HI cube; the
expected WALLABY cube, 6144x6144x16384, section 3) are not available, so these
cubes stand in for them: float32 RA x Dec x frequency volumes of unit Gaussian
noise plus compact Gaussian sources that are broad along the spectral axis.

Array convention: a cube is a C-ordered numpy array of shape (nz, ny, nx) with
x (RA) fastest and z the frequency axis.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, asdict

import numpy as np

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


# --------------------------------------------------------------------------
# cubes
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class CubeSpec:
    """Recipe of one synthetic cube (shape is (nz, ny, nx))."""
    shape: tuple
    n_sources: int
    seed: int
    sigma_xy: tuple = (1.0, 4.0)      # spatial Gaussian sigma range, voxels
    fwhm_z: tuple | None = None       # spectral FWHM range, channels; None = isotropic
    amp: tuple = (3.0, 10.0)          # peak amplitude range, units of noise sigma
    truncate: float = 4.0             # sources are cut at +-truncate sigma


# The five workloads (shape = (nz, ny, nx)).
CUBE_64 = CubeSpec((64, 64, 64), 20, seed=1)
CUBE_8GIB = CubeSpec((2048, 1024, 1024), 500, seed=2, fwhm_z=(5.0, 50.0))
CUBE_64GIB = CubeSpec((4096, 2048, 2048), 4000, seed=3, fwhm_z=(5.0, 50.0))
CUBE_512MIB = CubeSpec((1024, 512, 512), 200, seed=4, fwhm_z=(5.0, 50.0))
CUBE_DIFF = CubeSpec((256, 128, 128), 40, seed=5, fwhm_z=(5.0, 50.0))
CUBE_FD16 = CubeSpec((16, 16, 16), 4, seed=5)


def _noise_chunk(seed_seq, shape, out):
    rng = np.random.default_rng(seed_seq)
    rng.standard_normal(out=out, dtype=np.float32)


def make_cube(spec: CubeSpec, out: np.ndarray | None = None, threads: int | None = None,
              chunk_planes: int = 16) -> np.ndarray:
    """Noise N(0,1) plus Gaussian sources, float32 (nz, ny, nx).

    The noise is drawn per slab of `chunk_planes` z-planes, each slab from its
    own child of SeedSequence(seed), so the result does not depend on the
    number of threads.  Sources are drawn from default_rng(seed + 7919):
    centres uniform in the continuous box, amplitude uniform in spec.amp,
    sigma_xy uniform in spec.sigma_xy, and either the same sigma along z
    (isotropic) or a spectral FWHM uniform in spec.fwhm_z.  A source is
    evaluated at voxel centres (i + 1/2) in float64 and added once per voxel.
    `out` may be a writable memmap of the right shape and dtype.
    """
    nz, ny, nx = spec.shape
    if out is None:
        out = np.empty(spec.shape, dtype=np.float32)
    assert out.shape == spec.shape and out.dtype == np.float32
    n_chunks = (nz + chunk_planes - 1) // chunk_planes
    children = np.random.SeedSequence(spec.seed).spawn(n_chunks)
    threads = threads or min(16, os.cpu_count() or 1)

    def work(c):
        z0 = c * chunk_planes
        z1 = min(nz, z0 + chunk_planes)
        buf = np.empty((z1 - z0, ny, nx), dtype=np.float32)
        _noise_chunk(children[c], buf.shape, buf)
        out[z0:z1] = buf

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(n_chunks)))

    for s in draw_sources(spec):
        add_source(out, s, spec.truncate)
    return out


def draw_sources(spec: CubeSpec):
    """List of (cx, cy, cz, amp, sx, sy, sz) tuples, float64."""
    nz, ny, nx = spec.shape
    rng = np.random.default_rng(spec.seed + 7919)
    src = []
    for _ in range(spec.n_sources):
        cx, cy, cz = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
        amp = rng.uniform(*spec.amp)
        sx = rng.uniform(*spec.sigma_xy)
        sy = rng.uniform(*spec.sigma_xy)
        if spec.fwhm_z is None:
            sz = rng.uniform(*spec.sigma_xy)
        else:
            sz = rng.uniform(*spec.fwhm_z) * FWHM_TO_SIGMA
        src.append((cx, cy, cz, amp, sx, sy, sz))
    return src


def add_source(cube, s, truncate):
    nz, ny, nx = cube.shape
    cx, cy, cz, amp, sx, sy, sz = s

    def axis(c, sig, n):
        lo = max(0, int(math.floor(c - truncate * sig)))
        hi = min(n, int(math.ceil(c + truncate * sig)) + 1)
        x = np.arange(lo, hi, dtype=np.float64) + 0.5
        g = np.exp(-0.5 * ((x - c) / sig) ** 2)
        g[np.abs(x - c) > truncate * sig] = 0.0
        return lo, hi, g

    x0, x1, gx = axis(cx, sx, nx)
    y0, y1, gy = axis(cy, sy, ny)
    z0, z1, gz = axis(cz, sz, nz)
    if x1 <= x0 or y1 <= y0 or z1 <= z0:
        return
    blob = amp * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    sub = cube[z0:z1, y0:y1, x0:x1]
    cube[z0:z1, y0:y1, x0:x1] = (sub.astype(np.float64) + blob).astype(np.float32)


def catalogue_boxes(spec: CubeSpec, seed: int = 0, reach: float = 2.0, n_false: int = 0) -> np.ndarray:
    """A source-finder-style catalogue of the cube: for every source, the
    bounding cube of the voxels within `reach` sigma of its centre, as
    (lo x, lo y, lo z, hi x, hi y, hi z) in voxel coordinates (voxel edges,
    clipped to the cube), plus a straight RGBA colour drawn from
    default_rng(seed); `n_false` extra boxes at random places stand for
    spurious detections.  float32 (n, 10)."""
    nz, ny, nx = spec.shape
    rng = np.random.default_rng(seed)
    rows = []
    for cx, cy, cz, _amp, sx, sy, sz in draw_sources(spec):
        lo = [max(0.0, math.floor(c - reach * sg)) for c, sg in ((cx, sx), (cy, sy), (cz, sz))]
        hi = [min(float(n), math.ceil(c + reach * sg)) for c, sg, n in ((cx, sx, nx), (cy, sy, ny), (cz, sz, nz))]
        rows.append(lo + hi + list(rng.uniform(0.2, 1.0, 3)) + [rng.uniform(0.5, 1.0)])
    for _ in range(n_false):
        c = [rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)]
        h = rng.uniform(1.0, 6.0, 3)
        rows.append([c[0] - h[0], c[1] - h[1], c[2] - h[2], c[0] + h[0], c[1] + h[1], c[2] + h[2]] +
                    list(rng.uniform(0.2, 1.0, 3)) + [rng.uniform(0.5, 1.0)])
    return np.asarray(rows, dtype=np.float32).reshape(-1, 10)


# --------------------------------------------------------------------------
# transfer-function tables (straight RGBA, shape (n, 4), float32)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Lut:
    table: np.ndarray     # (n, 4) float32, straight (not premultiplied) RGBA
    vmin: float
    vmax: float


def lut_ramp(n: int = 256, vmin: float = -3.0, vmax: float = 10.0, alpha_scale: float = 1.0) -> Lut:
    """Grey ramp: entry j = (x, x, x, x * alpha_scale) with x = j / (n - 1).

    alpha_scale = 1 is the 256-entry linear ramp over [-3 sigma, 10 sigma];
    alpha_scale = 1/64 is the deep-traversal variant (rays then run long).
    """
    x = np.arange(n, dtype=np.float64) / (n - 1)
    t = np.stack([x, x, x, x * alpha_scale], axis=1).astype(np.float32)
    return Lut(t, float(vmin), float(vmax))


def lut_random(seed: int, n: int = 256, vmin: float = -3.0, vmax: float = 10.0,
               knots: int = 4, alpha_range=(0.05, 1.0)) -> Lut:
    """Random piecewise-linear table: per channel `knots` interior knots at
    uniform positions with uniform values, plus end points; alpha scaled by a
    uniform factor from alpha_range."""
    rng = np.random.default_rng(seed)
    xs = np.arange(n, dtype=np.float64) / (n - 1)
    chans = []
    for ch in range(4):
        kx = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, knots)), [1.0]])
        ky = rng.uniform(0, 1, knots + 2)
        chans.append(np.interp(xs, kx, ky))
    t = np.stack(chans, axis=1)
    t[:, 3] *= rng.uniform(*alpha_range)
    return Lut(t.astype(np.float32), float(vmin), float(vmax))


def lut_dyadic(values, vmin: float, vmax: float) -> Lut:
    return Lut(np.asarray(values, dtype=np.float32).reshape(-1, 4), float(vmin), float(vmax))


# --------------------------------------------------------------------------
# cameras (plain parameters; the renderer derives rays from them)
# --------------------------------------------------------------------------
ORTHO, PERSPECTIVE = 0, 1


@dataclass
class Camera:
    kind: int
    eye: tuple
    target: tuple
    up: tuple
    fovy_deg: float = 30.0
    half_w: float = 1.0
    half_h: float = 1.0
    full_w: int = 256
    full_h: int = 256
    tile: tuple = field(default=None)   # (x0, y0, w, h); None = full frame

    def __post_init__(self):
        if self.tile is None:
            self.tile = (0, 0, self.full_w, self.full_h)
        self.eye = tuple(float(v) for v in self.eye)
        self.target = tuple(float(v) for v in self.target)
        self.up = tuple(float(v) for v in self.up)
        self.tile = tuple(int(v) for v in self.tile)

    def with_tile(self, x0, y0, w, h) -> "Camera":
        d = asdict(self)
        d["tile"] = (x0, y0, w, h)
        return Camera(**d)

    def as_dict(self):
        return asdict(self)


def camera_axis_z(nx=64, ny=64, nz=64, w=256, h=256) -> Camera:
    """Orthographic view along +z covering the x-y face exactly (64^3 case):
    eye one voxel in front of z = 0, up = -y, so image rows follow +y."""
    return Camera(ORTHO, (nx / 2, ny / 2, -1.0), (nx / 2, ny / 2, 0.0), (0.0, -1.0, 0.0),
                  half_w=nx / 2, half_h=ny / 2, full_w=w, full_h=h)


def orbit_camera(shape, seed: int, w: int, h: int, fovy_deg: float = 30.0,
                 elev_deg=(-60.0, 60.0)) -> Camera:
    """Perspective camera on the bounding sphere's fitting orbit.

    Centre c0 = (nx, ny, nz)/2, radius R = |(nx, ny, nz)|/2, distance
    D = R / sin(fovy/2); azimuth phi ~ U[0, 2 pi), elevation theta ~ U[elev)
    from default_rng(seed); eye = c0 + D (cos th sin ph, sin th, cos th cos ph);
    up = (0, -1, 0)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    th = math.radians(rng.uniform(*elev_deg))
    c0 = np.array([nx, ny, nz], dtype=np.float64) / 2.0
    R = 0.5 * math.sqrt(nx * nx + ny * ny + nz * nz)
    D = R / math.sin(math.radians(fovy_deg) / 2.0)
    eye = c0 + D * np.array([math.cos(th) * math.sin(phi), math.sin(th), math.cos(th) * math.cos(phi)])
    return Camera(PERSPECTIVE, tuple(eye), tuple(c0), (0.0, -1.0, 0.0), fovy_deg=fovy_deg,
                  full_w=w, full_h=h)


def batch_views(shape, seed: int, n_views: int = 64, w_range=(256, 1920), h_range=(256, 1080)):
    """Uneven views: sizes W ~ U{w_range}, H ~ U{h_range}, orbit cameras with
    sub-seeds, one random transfer table per view (seed-derived)."""
    rng = np.random.default_rng(seed)
    views = []
    for v in range(n_views):
        w = int(rng.integers(w_range[0], w_range[1] + 1))
        h = int(rng.integers(h_range[0], h_range[1] + 1))
        sub = int(rng.integers(0, 2**31 - 1))
        views.append((orbit_camera(shape, sub, w, h), sub))
    luts = [lut_random(sub + 1) for (_, sub) in views]
    return [v for (v, _) in views], luts


def tiles_5x5(cam: Camera, tw: int = 1920, th: int = 1080):
    """The 5 x 5 display wall: 25 viewports of one full frame."""
    return [cam.with_tile(c * tw, r * th, tw, th) for r in range(5) for c in range(5)]


def sample_pixels(w: int, h: int, n: int, seed: int) -> np.ndarray:
    """n distinct seeded pixel coordinates (x, y), int32, shape (n, 2)."""
    rng = np.random.default_rng(seed)
    n = min(n, w * h)
    idx = rng.choice(w * h, size=n, replace=False)
    return np.stack([idx % w, idx // w], axis=1).astype(np.int32)
