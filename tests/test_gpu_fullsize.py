"""Full-size parity, on sampled pixels, in the launch configuration the
benchmark times (the library's default tuning: automatic path and LDS
budget, orientation copies on one-brick layouts).

- 8 GiB cube (1024 x 1024 x 2048), 1920x1080 orbit cameras: composite,
  trilinear MIP and nearest MIP at three of the benchmark's angles (the
  first, the most oblique and the most axis-aligned).
- 64 GiB cube (2048 x 2048 x 4096) as 256^3 bricks, 9600x5400 frame as 5x5
  tiles of 1920x1080: per-brick partials + sort-last "over" on three tiles,
  composite with FP32, FP16 and BF16 storage, MIP with FP32 storage.
- 512 MiB cube, FP16 storage: 64 uneven views with random tables in one
  persistent launch replayed from a HIP graph.

Each case draws seeded pixels of the frame (a quarter of them forced onto
pixels whose ray hits the cube) and compares them one by one with the FP64
oracle."""
import numpy as np
import pytest
import torch

import bench
import oracle
from paper_1012_2909_amd import synth
from tests.gpu_util import (TOL_COMPOSITE, TOL_LOWP, assert_accept, assert_bitexact_mip, log,
                            max_neighbour_diff, mip_tol)

pytestmark = [pytest.mark.gpu, pytest.mark.big]


@pytest.fixture(scope="module")
def R():
    from paper_1012_2909_amd import vr
    r = vr.Renderer(0)
    yield r
    r.close()


def _pixels(img, n, seed):
    """n seeded pixels (x, y) of the frame, at least a quarter of them where
    the GPU image shows a hit."""
    h, w = img.shape[:2]
    rng = np.random.default_rng(seed)
    pix = synth.sample_pixels(w, h, n, seed)
    hit = np.argwhere((img[..., 3] if img.ndim == 3 else np.isfinite(img)) != 0)
    if len(hit):
        k = rng.choice(len(hit), size=min(n // 4, len(hit)), replace=False)
        pix = np.concatenate([pix, hit[k][:, ::-1].astype(np.int32)])
    return np.unique(pix, axis=0)


@pytest.fixture(scope="module")
def cube8():
    return synth.make_cube(synth.CUBE_8GIB)


_G = {}


def _grad8(cube8):
    if "g8" not in _G:
        _G["g8"] = max_neighbour_diff(cube8)
    return _G["g8"]


@pytest.mark.parametrize("angle", [0, 8, 10])
def test_8gib_1920x1080_sampled(R, cube8, angle):
    spec = synth.CUBE_8GIB
    if R.shape != spec.shape or R.orientations != 3 or R.storage_dtype != "f32":
        R.load_volume(torch.from_numpy(cube8), orientations=3)
    lut = synth.lut_ramp()
    R.set_lut(lut)
    cam = synth.orbit_camera(spec.shape, seed=bench.angle_seeds()[angle], w=1920, h=1080)
    R.set_camera(cam)
    for mode, filt in [("composite", "trilinear"), ("mip", "trilinear"), ("mip", "nearest")]:
        log(f"case: 8 GiB angle {angle} {mode}/{filt}")
        img = R.render(mode=mode, filt=filt).cpu().numpy()
        pix = _pixels(img, 1200, 100 + angle)
        got = img[pix[:, 1], pix[:, 0]]
        res = oracle.render(cube8, lut, cam, mode=mode, filt=filt, pixels=pix, eps_stop=2e-5)
        what = f"8 GiB angle {angle} {mode}/{filt} ({len(pix)} px)"
        if filt == "nearest":
            assert_bitexact_mip(got, res, what)
        elif mode == "mip":
            assert_accept(got, res, mip_tol(np.abs(cube8).max(), _grad8(cube8), res["taken"]), what=what)
        else:
            assert_accept(got, res, TOL_COMPOSITE, what=what)


def test_8gib_9600x5400_in_one_call_sampled(R, cube8):
    """The largest viewport in one render call (the full 5x5-panel frame)."""
    spec = synth.CUBE_8GIB
    if R.shape != spec.shape or R.orientations != 3 or R.storage_dtype != "f32":
        R.load_volume(torch.from_numpy(cube8), orientations=3)
    lut = synth.lut_ramp()
    R.set_lut(lut)
    cam = synth.orbit_camera(spec.shape, seed=bench.angle_seeds()[3], w=9600, h=5400)
    R.set_camera(cam)
    for mode in ("composite", "mip"):
        log(f"case: 8 GiB 9600x5400 {mode}")
        img = R.render(mode=mode).cpu().numpy()
        pix = _pixels(img, 800, 500)
        res = oracle.render(cube8, lut, cam, mode=mode, pixels=pix, eps_stop=2e-5)
        got = img[pix[:, 1], pix[:, 0]]
        if mode == "mip":
            assert_accept(got, res, mip_tol(np.abs(cube8).max(), _grad8(cube8), res["taken"]),
                          what=f"9600x5400 {mode}")
        else:
            assert_accept(got, res, TOL_COMPOSITE, what=f"9600x5400 {mode}")


@pytest.fixture(scope="module")
def cube64():
    return synth.make_cube(synth.CUBE_64GIB)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_64gib_bricked_9600x5400_sampled(R, cube64, storage):
    spec = synth.CUBE_64GIB
    nz = spec.shape[0]
    log(f"case: 64 GiB bricked {storage}")
    R.describe_volume(spec.shape, storage=storage, brick=256)
    for z0 in range(0, nz, 256):                      # 4 GiB slabs
        R.load_slab(torch.from_numpy(cube64[z0:z0 + 256]), z0)
    torch.cuda.synchronize()
    lut = synth.lut_ramp(alpha_scale=1.0 / 64.0)      # deep traversal: the early stop rarely fires
    R.set_lut(lut)
    vmax = max(float(np.abs(cube64[z0:z0 + 256]).max()) for z0 in range(0, nz, 256))
    frame = synth.orbit_camera(spec.shape, seed=3, w=9600, h=5400)
    tiles = synth.tiles_5x5(frame)
    tol = TOL_COMPOSITE if storage == "f32" else TOL_LOWP
    # tiles that see the cube: 6 holds its silhouette's edge, 12 its centre,
    # 18 a partly covered panel (the frame's corner panels see nothing)
    for t in (6, 12, 18):
        cam = tiles[t]
        R.set_camera(cam)
        # MIP of rounded storage has no stated bar: FP32 storage only
        for mode in (("composite", "mip") if storage == "f32" else ("composite",)):
            img = R.render_bricked(mode=mode).cpu().numpy()
            pix = _pixels(img, 300, 300 + t)
            got = img[pix[:, 1], pix[:, 0]]
            res = oracle.render_bricked(cube64, lut, cam, 256, mode=mode, pixels=pix, eps_stop=2e-5)
            hits = int((got[:, 3] > 0).sum()) if mode == "composite" else int(np.isfinite(got).sum())
            assert hits >= len(pix) // 5, f"tile {t}: only {hits} of {len(pix)} sampled pixels see the cube"
            # brick-face ties (a sample within 1e-7 voxel of a brick face, which
            # the two sides may assign to different bricks) are the only
            # flagged pixels the candidate interval does not cover
            face = (res["flags"] & oracle.FLAG_BRICK) != 0
            assert face.sum() <= 2
            keep = ~face
            sub = {k: v[keep] for k, v in res.items()}
            if mode == "composite":
                bound = tol
            else:
                if "g64" not in _G:
                    _G["g64"] = max_neighbour_diff(cube64)
                n = oracle.render(cube64, lut, cam, mode="mip", pixels=pix)["taken"][keep]
                bound = mip_tol(vmax, _G["g64"], n)
            assert_accept(got[keep], sub, bound,
                          what=f"64 GiB {storage} tile {t} {mode} ({len(pix)} px, {hits} hit)")


def test_64gib_streamed_quarter_cache_equals_resident(R, cube64):
    """The 64 GiB cube, FP16 storage, as 1024 bricks of 256^3: the centre
    panel of the 9600x5400 frame rendered from bricks streamed out of pinned
    host memory through a device cache of 256 bricks (a quarter) equals the
    resident bricked render bit for bit, in both modes."""
    import time
    from paper_1012_2909_amd import vr
    spec = synth.CUBE_64GIB
    log("case: 64 GiB streamed, quarter cache")
    R.describe_volume(spec.shape, storage="f16", brick=256)
    for z0 in range(0, spec.shape[0], 256):
        R.load_slab(torch.from_numpy(cube64[z0:z0 + 256]), z0)
    lut = synth.lut_ramp(alpha_scale=1.0 / 64.0)
    R.set_lut(lut)
    cam = synth.tiles_5x5(synth.orbit_camera(spec.shape, seed=3, w=9600, h=5400))[12]
    R.set_camera(cam)
    ref = {m: R.render_bricked(mode=m).cpu().numpy() for m in ("composite", "mip")}
    t = time.time()
    host = vr.pack_bricks_host(cube64, storage="f16", brick=256)
    log(f"packed {host.numel() / 1e9:.1f} GB of bricks in pinned host memory in {time.time() - t:.1f}s")
    R.describe_streamed_volume(spec.shape, host, storage="f16", brick=256, cache_slots=256)
    R.set_lut(lut)
    R.set_camera(cam)
    for m in ("composite", "mip"):
        torch.cuda.synchronize()
        t = time.time()
        got = R.render_bricked(mode=m).cpu().numpy()
        dt = time.time() - t
        copied, hits, slots = R.stream_stats()
        log(f"streamed {m}: {dt * 1e3:.0f} ms, {copied} bricks copied so far, {hits} hits, {slots} slots")
        assert np.array_equal(got, ref[m]), m
    assert slots == 256 and copied > 256
    R.storage = None
    del host


def test_512mib_f16_batch_of_64_views_graph_sampled(R):
    spec = synth.CUBE_512MIB
    vol = synth.make_cube(spec)
    R.load_volume(torch.from_numpy(vol), storage="f16")
    cams, luts = synth.batch_views(spec.shape, 4, n_views=64)
    packed = R.stack_luts(luts)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        R.render_batch(cams, packed, use_graph=True, stream=s)          # capture
        outs = R.render_batch(cams, packed, use_graph=True, stream=s)   # replay
    s.synchronize()
    worst = 0.0
    for i in range(0, 64, 3):
        img = outs[i].cpu().numpy()
        pix = _pixels(img, 60, 400 + i)
        res = oracle.render(vol, luts[i], cams[i], pixels=pix, eps_stop=2e-5)
        worst = max(worst, assert_accept(img[pix[:, 1], pix[:, 0]], res, TOL_LOWP, what=f"batch view {i}"))
    log(f"batch of 64 views, FP16 storage: worst error {worst:.3e} (bar {TOL_LOWP})")
