"""GPU tests of the batched renderer (one persistent launch over many uneven
views, optionally replayed from a HIP graph) and of the autotuner.  A batch
must reproduce, bit for bit, the images of the same views rendered one by one
(the arithmetic per pixel is the same), and those images are checked against
the FP64 oracle."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1012_2909_amd import synth
from tests.gpu_util import TOL_COMPOSITE, assert_accept, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1012_2909_amd import vr
    r = vr.Renderer(0)
    yield r
    r.close()


SHAPE = (80, 56, 64)


@pytest.fixture(scope="module")
def cube():
    return synth.make_cube(synth.CubeSpec(SHAPE, 16, seed=44, fwhm_z=(4.0, 24.0)))


def _views(seed, n, wr=(17, 260), hr=(9, 150)):
    cams, luts = synth.batch_views(SHAPE, seed, n_views=n, w_range=wr, h_range=hr)
    return cams, luts


def _one_by_one(R, cams, luts, mode="composite"):
    out = []
    for c, l in zip(cams, luts):
        R.set_lut(l)
        R.set_camera(c)
        out.append(R.render(mode=mode).cpu().numpy())
    return out


@pytest.mark.parametrize("path", [0, 1, 2])
@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("mode", ["composite", "mip"])
def test_batch_equals_single_views(R, cube, storage, mode, path):
    """Every batch kernel (the automatic choice, direct gathers, LDS boxes)
    reproduces the single-view renders bit for bit."""
    log(f"case: batch storage={storage} mode={mode} path={path}")
    R.load_volume(torch.from_numpy(cube), storage=storage)
    cams, luts = _views(7, 9)
    base = R.get_tuning()
    R.set_tuning(path=path)
    try:
        got = R.render_batch(cams, luts, mode=mode)
    finally:
        R.set_tuning(**base)
    torch.cuda.synchronize()
    ref = _one_by_one(R, cams, luts, mode)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert np.array_equal(g.cpu().numpy(), r), f"view {i} differs"
    # two of the views against the oracle
    vol = cube if storage == "f32" else torch.from_numpy(cube).half().float().numpy()
    for i in (0, 5):
        res = oracle.render(vol, luts[i], cams[i], mode=mode, eps_stop=2e-5)
        if mode == "composite":
            assert_accept(ref[i], res, TOL_COMPOSITE, what=f"batch view {i}")
        else:
            assert_accept(ref[i], res, 1e-6, rel=1e-6, what=f"batch view {i} MIP")


def test_graph_replays_match_eager(R, cube):
    """Capture once, replay with new cameras and outputs (same sizes), with
    eager work in between; every replay equals the eager images."""
    R.load_volume(torch.from_numpy(cube))
    cams, luts = _views(11, 6)
    packed = R.stack_luts(luts)           # one table tensor for every replay
    s = torch.cuda.Stream()
    n0 = R.graph_captures()
    for rep in range(4):
        # new camera positions with the same viewport sizes
        moved = [synth.orbit_camera(SHAPE, seed=100 * rep + i, w=c.full_w, h=c.full_h) for i, c in enumerate(cams)]
        with torch.cuda.stream(s):
            got = R.render_batch(moved, packed, use_graph=True, stream=s)
        s.synchronize()
        eager = _one_by_one(R, moved, luts)          # eager work between replays
        torch.cuda.synchronize()
        for i, (g, e) in enumerate(zip(got, eager)):
            assert np.array_equal(g.cpu().numpy(), e), f"replay {rep} view {i}"
    assert R.graph_captures() == n0 + 1
    # a different batch shape captures again
    cams2, luts2 = _views(12, 3)
    with torch.cuda.stream(s):
        R.render_batch(cams2, luts2, use_graph=True, stream=s)
    s.synchronize()
    assert R.graph_captures() == n0 + 2


def test_graph_recaptures_after_a_new_volume(R, cube):
    """A captured graph holds the volume description in its kernel argument.
    Loading another cube (other shape and storage type, possibly at the same
    address) must capture again, and the replay must equal the eager images
    of the new cube."""
    R.load_volume(torch.from_numpy(cube))
    cams, luts = _views(13, 4)
    packed = R.stack_luts(luts)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        R.render_batch(cams, packed, use_graph=True, stream=s)
    s.synchronize()
    n0 = R.graph_captures()
    small = np.ascontiguousarray(cube[:40, :44, :52])
    old_ptr = R.storage.data_ptr()
    R.load_volume(torch.from_numpy(small), storage="f16")
    log(f"storage reused at the same address: {R.storage.data_ptr() == old_ptr}")
    with torch.cuda.stream(s):
        got = R.render_batch(cams, packed, use_graph=True, stream=s)
    s.synchronize()
    assert R.graph_captures() == n0 + 1
    eager = _one_by_one(R, cams, luts)
    torch.cuda.synchronize()
    for i, (g, e) in enumerate(zip(got, eager)):
        assert np.array_equal(g.cpu().numpy(), e), f"view {i}"


def test_five_by_five_wall_in_one_batch(R, cube):
    """The 25 panels of a tiled frame rendered as one batch stitch into the
    full-frame render."""
    R.load_volume(torch.from_numpy(cube))
    lut = synth.lut_ramp()
    cam = synth.orbit_camera(SHAPE, seed=3, w=5 * 40, h=5 * 24)
    R.set_lut(lut)
    R.set_camera(cam)
    full = R.render().cpu().numpy()
    tiles = synth.tiles_5x5(cam, 40, 24)
    outs = R.render_batch(tiles, [lut])
    torch.cuda.synchronize()
    st = np.zeros_like(full)
    for t, o in zip(tiles, outs):
        x0, y0, w, h = t.tile
        st[y0:y0 + h, x0:x0 + w] = o.cpu().numpy()
    assert np.array_equal(st, full)


def test_autotune_and_cache(R, cube, tmp_path):
    R.load_volume(torch.from_numpy(cube))
    R.set_lut(synth.lut_ramp())
    R.set_camera(synth.orbit_camera(SHAPE, seed=1, w=300, h=200))
    path = str(tmp_path / "tune.json")
    t1 = R.autotune(cache_path=path)
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0][5] in (1, 2)
    R.set_tuning(path=1, packet_w=8, packet_h=8)
    t2 = R.autotune(cache_path=path)           # cache hit restores the tuned shape
    assert t2 == t1
    cams, luts = _views(5, 5)
    tb = R.autotune_batch(cams, luts, cache_path=path)
    assert len(json.load(open(path))) == 2 and tb["path"] in (1, 2)
    # the tuned shapes still render correctly
    got = R.render_batch(cams, luts)
    torch.cuda.synchronize()
    ref = _one_by_one(R, cams, luts)
    for g, r in zip(got, ref):
        assert np.array_equal(g.cpu().numpy(), r)


def test_batch_with_one_pixel_and_empty_views(R, cube):
    """1x1 viewports and a view that misses the cube, beside ordinary ones."""
    R.load_volume(torch.from_numpy(cube))
    lut = synth.lut_ramp()
    big = synth.orbit_camera(SHAPE, seed=31, w=64, h=48)
    one = big.with_tile(20, 30, 1, 1)
    miss = synth.Camera(synth.ORTHO, (500.0, 500.0, -10.0), (500.0, 500.0, 0.0), (0.0, -1.0, 0.0),
                        half_w=3.0, half_h=3.0, full_w=5, full_h=7)
    cams = [one, big, miss, big.with_tile(63, 47, 1, 1)]
    for mode in ("composite", "mip"):
        got = R.render_batch(cams, [lut], mode=mode)
        torch.cuda.synchronize()
        ref = _one_by_one(R, cams, [lut] * 4, mode)
        for i, (g, r) in enumerate(zip(got, ref)):
            assert np.array_equal(g.cpu().numpy(), r), f"{mode} view {i}"
        m = got[2].cpu().numpy()
        assert (m == 0).all() if mode == "composite" else np.isneginf(m).all()
