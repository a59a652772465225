"""GPU parity of the brick path: per-brick partial images (K3), their
visibility order and the sort-last "over" composite (K4), through the C ABI,
against the FP64 oracle's bricked render."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_1012_2909_amd import synth
from tests.gpu_util import TOL_COMPOSITE, TOL_MIP_REL, assert_accept, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1012_2909_amd import vr
    r = vr.Renderer(0)
    yield r
    r.close()


def _setup(R, vol, lut, cam, brick, storage="f32"):
    R.load_volume(torch.from_numpy(vol), storage=storage, brick=brick)
    R.set_lut(lut)
    R.set_camera(cam)


CAMS = {
    "persp": lambda shape: synth.orbit_camera(shape, seed=21, w=140, h=100),
    "persp2": lambda shape: synth.orbit_camera(shape, seed=5, w=120, h=90),
    "ortho": lambda shape: synth.Camera(synth.ORTHO, (-30.0, 40.0, -25.0), (23.0, 18.0, 30.0), (0.0, -1.0, 0.0),
                                        half_w=45.0, half_h=32.0, full_w=140, full_h=100),
}


@pytest.mark.parametrize("brick", [16, 13, 40])
@pytest.mark.parametrize("cam_name", ["persp", "ortho"])
def test_bricked_equals_single_pass_without_early_stop(R, brick, cam_name):
    log(f"case: bricked=single pass brick={brick} cam={cam_name}")
    shape = (60, 36, 46)
    vol = synth.make_cube(synth.CubeSpec(shape, 10, seed=3, fwhm_z=(4.0, 20.0)))
    lut = synth.lut_ramp(alpha_scale=1 / 8)
    cam = CAMS[cam_name](shape)
    _setup(R, vol, lut, cam, brick)
    br = R.render_bricked(ert=1.0).cpu().numpy()
    one = R.render(ert=1.0).cpu().numpy()
    assert np.abs(br - one).max() <= 1e-6
    res = oracle.render(vol, lut, cam, tau=1.0)
    assert_accept(br, res, TOL_COMPOSITE, what="bricked vs oracle single pass")
    # MIP: the maximum does not depend on the grouping: bit-identical
    brm = R.render_bricked(mode="mip", ert=1.0).cpu().numpy()
    onem = R.render(mode="mip").cpu().numpy()
    assert np.array_equal(brm, onem)
    brn = R.render_bricked(mode="mip", filt="nearest").cpu().numpy()
    onen = R.render(mode="mip", filt="nearest").cpu().numpy()
    assert np.array_equal(brn, onen)


@pytest.mark.parametrize("brick", [16, 23])
@pytest.mark.parametrize("cam_name", ["persp", "persp2", "ortho"])
def test_bricked_with_early_stop_matches_oracle(R, brick, cam_name):
    log(f"case: bricked ERT brick={brick} cam={cam_name}")
    shape = (64, 40, 48)
    vol = synth.make_cube(synth.CubeSpec(shape, 10, seed=4, fwhm_z=(4.0, 20.0)))
    lut = synth.lut_ramp(alpha_scale=0.5)
    cam = CAMS[cam_name](shape)
    _setup(R, vol, lut, cam, brick)
    img = R.render_bricked().cpu().numpy()
    res = oracle.render_bricked(vol, lut, cam, brick, eps_stop=2e-5)
    # flagged pixels are checked against the candidate interval (flipped
    # stop and count decisions); only brick-face ties are left out
    face = (res["flags"] & oracle.FLAG_BRICK) != 0
    assert face.sum() <= 2
    keep = ~face
    assert_accept(img[keep], {k: v[keep] for k, v in res.items()}, TOL_COMPOSITE,
                  what=f"bricked ERT brick={brick} cam={cam_name}")


@pytest.mark.parametrize("brick", [5, 7, 16])
@pytest.mark.parametrize("eye,target", [((21.3, 17.7, 29.1), (60.0, 5.0, 40.0)),
                                        ((35.6, 8.4, 12.2), (-8.0, 30.0, 50.0))])
def test_bricked_eye_inside_grid(R, brick, eye, target):
    """Perspective eye inside the cube, so inside the brick grid: the
    Manhattan order from the eye's cell must still be front to back.  Without
    the early stop the bricked render equals the single pass (1e-6) and the
    oracle's bricked render; MIP is bit-identical to the single pass."""
    log(f"case: bricked eye inside brick={brick} eye={eye}")
    shape = (60, 36, 46)
    vol = synth.make_cube(synth.CubeSpec(shape, 10, seed=3, fwhm_z=(4.0, 20.0)))
    lut = synth.lut_ramp(alpha_scale=1 / 8)
    cam = synth.Camera(synth.PERSPECTIVE, eye, target, (0.0, -1.0, 0.0), fovy_deg=100.0, full_w=96, full_h=72)
    _setup(R, vol, lut, cam, brick)
    br = R.render_bricked(ert=1.0).cpu().numpy()
    one = R.render(ert=1.0).cpu().numpy()
    assert np.abs(br - one).max() <= 1e-6
    assert_accept(br, oracle.render_bricked(vol, lut, cam, brick, tau=1.0), TOL_COMPOSITE,
                  what=f"bricked eye inside brick={brick}")
    brm = R.render_bricked(mode="mip", ert=1.0).cpu().numpy()
    assert np.array_equal(brm, R.render(mode="mip").cpu().numpy())


@pytest.mark.parametrize("mode,filt", [("composite", "trilinear"), ("mip", "trilinear"), ("mip", "nearest")])
def test_partials_match_oracle_and_footprints_are_conservative(R, mode, filt):
    shape = (50, 41, 37)
    B = 16
    vol = synth.make_cube(synth.CubeSpec(shape, 8, seed=6, fwhm_z=(4.0, 20.0)))
    lut = synth.lut_ramp(alpha_scale=0.5)
    cam = CAMS["persp"](shape)
    _setup(R, vol, lut, cam, B)
    parts, pool = R.render_bricks(mode=mode, filt=filt)
    torch.cuda.synchronize()
    nbx, nby, nbz = [(n + B - 1) // B for n in (shape[2], shape[1], shape[0])]
    ids = {p.brick_id for p in parts}
    assert len(ids) == len(parts)
    W, H = cam.tile[2], cam.tile[3]
    for p in parts:
        ch = 4 if mode == "composite" else 1
        n = p.w * p.h * ch
        buf = torch.empty(n, dtype=torch.float32, device="cuda")
        # copy the partial out of the pool (device pointer arithmetic)
        off = p.data - pool.data_ptr()
        got = pool[off:off + 4 * n].view(torch.float32).cpu().numpy().reshape(p.h, p.w, *((4,) if ch == 4 else ()))
        ref = oracle.render_bricked(vol, lut, cam, B, mode=mode, filt=filt, only_brick=p.brick_id, eps_stop=2e-5)
        sub = {k: v[p.y0:p.y0 + p.h, p.x0:p.x0 + p.w] for k, v in ref.items()}
        clean = sub["flags"] == 0
        if mode == "composite":
            assert np.abs(got - sub["out"])[clean].max(initial=0) <= TOL_COMPOSITE
        elif filt == "nearest":
            assert np.array_equal(got[clean], sub["out"][clean])
        else:
            d = np.abs(got - sub["out"])
            fin = np.isfinite(sub["out"])
            assert (got[~fin] == sub["out"][~fin]).all()
            assert (d[fin & clean] <= 1e-6 + TOL_MIP_REL * np.abs(sub["out"][fin & clean])).all()
        # nothing of this brick lies outside its footprint
        mask = np.ones((H, W), bool)
        mask[p.y0:p.y0 + p.h, p.x0:p.x0 + p.w] = False
        outside = ref["out"][mask]
        if mode == "composite":
            assert not outside.any()
        else:
            assert np.isneginf(outside).all()
    # every brick that some ray samples has a partial
    for b in range(nbx * nby * nbz):
        if b in ids:
            continue
        ref = oracle.render_bricked(vol, lut, cam, B, mode=mode, filt=filt, only_brick=b)["out"]
        assert (not ref.any()) if mode == "composite" else np.isneginf(ref).all()


def test_order_matches_oracle_keys(R):
    shape = (64, 48, 40)
    B = 16
    vol = synth.make_cube(synth.CubeSpec(shape, 2, seed=1))
    for cam_name in CAMS:
        cam = CAMS[cam_name](shape)
        _setup(R, vol, synth.lut_ramp(), cam, B)
        parts, _ = R.render_bricks()
        order = R.brick_order(parts)
        nbx, nby = (shape[2] + B - 1) // B, (shape[1] + B - 1) // B
        keys = []
        for i in order:
            bid = parts[i].brick_id
            keys.append((oracle.brick_key(cam, B, bid % nbx, (bid // nbx) % nby, bid // (nbx * nby)), bid))
        assert keys == sorted(keys)


def test_over_composite_of_given_partials(R):
    """K4 alone: composite oracle-made partials (inputs) and compare with the
    oracle's "over" of the same partials."""
    from paper_1012_2909_amd import vr
    rng = np.random.default_rng(3)
    W, H = 97, 61
    R.set_camera(synth.Camera(synth.ORTHO, (0.0, 0.0, -5.0), (0.0, 0.0, 0.0), (0.0, -1.0, 0.0),
                              half_w=1.0, half_h=1.0, full_w=W, full_h=H))
    tensors, parts, full = [], [], []
    for b in range(12):
        x0, y0 = int(rng.integers(0, W - 5)), int(rng.integers(0, H - 5))
        w, h = int(rng.integers(1, W - x0 + 1)), int(rng.integers(1, H - y0 + 1))
        a = rng.uniform(0, 1, (h, w, 1))
        rgba = np.concatenate([rng.uniform(0, 1, (h, w, 3)) * a, a], -1).astype(np.float32)   # premultiplied
        t = torch.from_numpy(rgba).cuda()
        tensors.append(t)
        parts.append(vr.Partial(t.data_ptr(), x0, y0, w, h, b, 0))
        f = np.zeros((H, W, 4))
        f[y0:y0 + h, x0:x0 + w] = rgba
        full.append(f)
    order = list(rng.permutation(12))
    got = R.composite_bricks(parts, order).cpu().numpy()
    ref = oracle.over(full, order)
    assert np.abs(got - ref).max() <= 1e-6
    # MIP: the maximum of the partial maxima (missing pixels are -inf)
    mt, mparts, mfull = [], [], []
    for i, p in enumerate(parts):
        v = rng.standard_normal((p.h, p.w)).astype(np.float32)
        t = torch.from_numpy(v).cuda()
        mt.append(t)
        mparts.append(vr.Partial(t.data_ptr(), p.x0, p.y0, p.w, p.h, i, 0))
        f = np.full((H, W), -np.inf)
        f[p.y0:p.y0 + p.h, p.x0:p.x0 + p.w] = v
        mfull.append(f)
    gotm = R.composite_bricks(mparts, order, mode="mip").cpu().numpy()
    assert np.array_equal(gotm, np.max(mfull, axis=0).astype(np.float32))
    torch.cuda.synchronize()


@pytest.mark.parametrize("brick", [16, 23, 64])
@pytest.mark.parametrize("cam_name", ["persp", "persp2", "ortho"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_lds_staged_bricks_equal_direct_gathers(R, brick, cam_name, storage):
    """K3 with LDS-staged boxes (the default) and K3 with direct gathers
    (tuning path 1) run the same arithmetic on the same samples: the
    bricked images are bit-identical, in both modes and both filters."""
    log(f"case: K3 staged = direct brick={brick} cam={cam_name} {storage}")
    shape = (64, 40, 48)
    vol = synth.make_cube(synth.CubeSpec(shape, 10, seed=4, fwhm_z=(4.0, 20.0)))
    lut = synth.lut_ramp(alpha_scale=0.5)
    _setup(R, vol, lut, CAMS[cam_name](shape), brick, storage)
    base = R.get_tuning()
    for mode, filt in [("composite", "trilinear"), ("composite", "nearest"), ("mip", "trilinear"),
                       ("mip", "nearest")]:
        staged = R.render_bricked(mode=mode, filt=filt).cpu().numpy()
        R.set_tuning(path=1)
        try:
            direct = R.render_bricked(mode=mode, filt=filt).cpu().numpy()
        finally:
            R.set_tuning(**base)
        assert np.array_equal(staged, direct), (mode, filt)


def test_bricked_full_frame_equals_stitched_panels(R):
    """The 5x5 wall rendered in one bricked call equals its 25 panels
    rendered one by one and stitched, bit for bit (each panel is a window of
    the same frame; each brick's partial covers its footprint in either)."""
    shape = (60, 36, 46)
    vol = synth.make_cube(synth.CubeSpec(shape, 10, seed=3, fwhm_z=(4.0, 20.0)))
    lut = synth.lut_ramp(alpha_scale=1 / 8)
    frame = synth.orbit_camera(shape, seed=21, w=160, h=90)
    _setup(R, vol, lut, frame, 16)
    for mode in ("composite", "mip"):
        full = R.render_bricked(mode=mode).cpu().numpy()
        for cam in synth.tiles_5x5(frame, 32, 18):
            R.set_camera(cam)
            x0, y0, w, h = cam.tile
            part = R.render_bricked(mode=mode).cpu().numpy()
            assert np.array_equal(part, full[y0:y0 + h, x0:x0 + w]), (mode, cam.tile)
        R.set_camera(frame)
