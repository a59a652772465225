"""GPU parity of the depth pass (K9) and the catalogue overlay (K10) through
the C ABI, against the FP64 oracle.

Depth: the GPU's t per pixel against the oracle's on the same cube and view;
where a decision (the opacity crossing, the early stop, the first maximum)
lies within its window the GPU value must be one of the oracle's candidate
depths [lo, hi].  t is written in FP32, so agreement is to 2^-23 relative.

Overlay: both sides draw the same catalogue over the same inputs, the
oracle's own render and depth cast to float32 (no input comes from the
GPU): unflagged pixels agree to FP32 rounding of the blend, flagged ones
(coverage, depth test or nearest box within 1e-9 of a tie) are counted."""
import numpy as np
import pytest
import torch

import oracle
from paper_1012_2909_amd import synth
from tests.gpu_util import log, mip_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1012_2909_amd import vr
    r = vr.Renderer(0)
    yield r
    r.close()


SPEC = synth.CubeSpec((72, 56, 64), 14, seed=61, fwhm_z=(4.0, 24.0))


@pytest.fixture(scope="module")
def cube():
    return synth.make_cube(SPEC)


def _check_depth(got, res, what):
    out, lo, hi, fl = res["out"], res["lo"], res["hi"], res["flags"]
    g = got.astype(np.float64)
    inf_ref = np.isinf(out)
    tol = 2.0 ** -23 * np.where(np.isfinite(out), np.abs(out), 0.0) + 1e-6
    clean = fl == 0
    ok_clean = np.where(inf_ref, g == out, np.abs(g - np.where(inf_ref, 0.0, out)) <= tol)
    bad = clean & ~ok_clean
    assert not bad.any(), f"{what}: {int(bad.sum())} unflagged px differ, first {np.argwhere(bad)[:5].tolist()}"
    amb = ~clean
    within = (np.isinf(g) & np.isinf(hi)) | ((g >= lo - 1e-3) & (g <= hi + 1e-3))
    assert within[amb].all(), f"{what}: flagged px outside their candidates"
    n_hit = int(np.isfinite(g).sum())
    log(f"{what}: {clean.sum()} exact px, {amb.sum()} flagged within candidates, {n_hit} with a depth")
    assert n_hit > 0


@pytest.mark.parametrize("mode,filt", [("composite", "trilinear"), ("composite", "nearest"),
                                       ("mip", "trilinear"), ("mip", "nearest")])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_depth_matches_oracle(R, cube, mode, filt, storage):
    log(f"case: depth {mode}/{filt} {storage}")
    R.load_volume(torch.from_numpy(cube), storage=storage)
    vol = cube if storage == "f32" else torch.from_numpy(cube).half().float().numpy()
    lut = synth.lut_ramp(alpha_scale=0.25)
    R.set_lut(lut)
    cam = synth.orbit_camera(SPEC.shape, seed=8, w=150, h=110)
    R.set_camera(cam)
    got = R.render_depth(mode=mode, filt=filt, level=0.5).cpu().numpy()
    eps_val = mip_tol(np.abs(vol).max()) if (mode == "mip" and filt == "trilinear") else 0.0
    res = oracle.depth(vol, lut, cam, mode=mode, filt=filt, level=0.5, eps_stop=2e-5, eps_val=eps_val)
    _check_depth(got, res, f"depth {mode}/{filt} {storage}")


def test_depth_tiles_stitch_bitexact(R, cube):
    R.load_volume(torch.from_numpy(cube))
    R.set_lut(synth.lut_ramp(alpha_scale=0.25))
    frame = synth.orbit_camera(SPEC.shape, seed=9, w=130, h=90)
    R.set_camera(frame)
    full = R.render_depth(level=0.3).cpu().numpy()
    for x0, y0, w, h in ((0, 0, 64, 40), (64, 40, 66, 50), (17, 61, 1, 1)):
        R.set_camera(frame.with_tile(x0, y0, w, h))
        part = R.render_depth(level=0.3).cpu().numpy()
        assert np.array_equal(part, full[y0:y0 + h, x0:x0 + w])


def test_depth_rejects_bricked_layout(R, cube):
    from paper_1012_2909_amd import vr
    R.load_volume(torch.from_numpy(cube), brick=24)
    R.set_lut(synth.lut_ramp())
    R.set_camera(synth.orbit_camera(SPEC.shape, seed=8, w=16, h=16))
    with pytest.raises(vr.VRError) as e:
        R.render_depth()
    assert e.value.code == vr.EUNSUPPORTED


@pytest.mark.parametrize("kind", ["persp", "ortho", "inside"])
def test_overlay_matches_oracle(R, cube, kind):
    log(f"case: overlay {kind}")
    lut = synth.lut_ramp(alpha_scale=0.25)
    if kind == "persp":
        cam = synth.orbit_camera(SPEC.shape, seed=8, w=160, h=120)
    elif kind == "ortho":
        cam = synth.Camera(synth.ORTHO, (-40.0, 70.0, -30.0), (32.0, 28.0, 36.0), (0.0, -1.0, 0.0),
                           half_w=60.0, half_h=45.0, full_w=160, full_h=120)
    else:   # eye inside the cube: boxes straddle the near plane
        cam = synth.Camera(synth.PERSPECTIVE, (30.0, 25.0, 20.0), (40.0, 30.0, 60.0), (0.0, -1.0, 0.0),
                           fovy_deg=80.0, full_w=160, full_h=120)
    boxes = synth.catalogue_boxes(SPEC, seed=3, n_false=300)
    # inputs from the oracle (FP64 render and depth, cast to float32)
    base = oracle.render(cube, lut, cam)["out"].astype(np.float32)
    dep = oracle.depth(cube, lut, cam, level=0.5)["out"].astype(np.float32)
    ref, fl = oracle.overlay(cam, boxes.astype(np.float64), base.astype(np.float64), half_width=0.75, depth=dep)
    R.load_volume(torch.from_numpy(cube))
    R.set_camera(cam)
    img = torch.from_numpy(base).cuda()
    R.overlay_boxes(torch.from_numpy(boxes), img, half_width=0.75, depth=torch.from_numpy(dep))
    got = img.cpu().numpy().astype(np.float64)
    clean = fl == 0
    err = np.abs(got - ref)[clean].max()
    drawn = int((np.abs(ref - base) > 0).any(axis=-1).sum())
    log(f"overlay {kind}: {drawn} px drawn, max err {err:.2e}, {int((~clean).sum())} flagged")
    # from inside the cube most edges lie behind the near emission
    assert drawn > (20 if kind == "inside" else 100)
    assert err <= 2e-7
    assert (~clean).sum() <= 4
    # without a depth image every covering edge is visible: more is drawn
    img2 = torch.from_numpy(base).cuda()
    R.overlay_boxes(torch.from_numpy(boxes), img2, half_width=0.75)
    ref2, fl2 = oracle.overlay(cam, boxes.astype(np.float64), base.astype(np.float64), half_width=0.75)
    clean2 = fl2 == 0
    assert np.abs(img2.cpu().numpy() - ref2)[clean2].max() <= 2e-7
    assert int((np.abs(ref2 - base) > 0).any(axis=-1).sum()) >= drawn
