"""vr_render_noalloc (the render for callers that cannot allocate device
memory) against vr_render with a caller workspace, through the C ABI: the
same kernels on the same inputs, so the images must be bit-identical.  Two
calls in a row on the library's fixed scratch, the second with a smaller
viewport, in object-order MIP (the path whose ray records live in the
scratch) and in the bundle kernel (whose tile order is sorted in the
scratch), plus the composite (no scratch) and the error paths."""
import numpy as np
import pytest
import torch

from paper_1012_2909_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1012_2909_amd import vr
    r = vr.Renderer(0)
    yield r
    r.close()


def test_noalloc_matches_workspace_render_on_two_calls(R):
    shape = (72, 60, 64)
    vol = synth.make_cube(synth.CubeSpec(shape, 12, seed=31, fwhm_z=(4.0, 24.0)))
    R.load_volume(torch.from_numpy(vol))
    R.set_lut(synth.lut_ramp())
    base = R.get_tuning()
    R.set_tuning(path=4)                       # MIP in object order: ray records in the scratch
    try:
        for i, (w, h) in enumerate(((300, 220), (97, 61))):     # the second call is smaller
            cam = synth.orbit_camera(shape, seed=40 + i, w=w, h=h)
            R.set_camera(cam)
            for filt in ("trilinear", "nearest"):
                need = R.workspace_bytes(mode="mip", filt=filt)
                assert need == w * h * 64, "object-order path not taken"
                log(f"case: noalloc call {i} {w}x{h} MIP {filt} ({need} B of scratch)")
                ref = R.render(mode="mip", filt=filt).cpu().numpy()
                # a prefilled output shows any pixel the call leaves unwritten
                out = torch.full((h, w), float("nan"), device="cuda")
                got = R.render_noalloc(mode="mip", filt=filt, out=out).cpu().numpy()
                assert np.array_equal(got, ref), f"call {i} {filt}"
                assert np.isfinite(ref).any()
            comp = R.render_noalloc().cpu().numpy()
            assert np.array_equal(comp, R.render().cpu().numpy())
    finally:
        R.set_tuning(**base)


def test_noalloc_bundle_order_on_two_calls(R):
    """The LDS-staged bundle kernel with its costliest-first tile order (the
    default order 3): the permutation lives in the scratch.  Two calls, the
    second smaller; each equals vr_render with a workspace and with none."""
    shape = (72, 60, 64)
    vol = synth.make_cube(synth.CubeSpec(shape, 12, seed=33, fwhm_z=(4.0, 24.0)))
    R.load_volume(torch.from_numpy(vol))
    R.set_lut(synth.lut_ramp())
    base = R.get_tuning()
    R.set_tuning(path=2, order=3)
    try:
        for i, (w, h) in enumerate(((300, 220), (97, 61))):
            cam = synth.orbit_camera(shape, seed=50 + i, w=w, h=h)
            R.set_camera(cam)
            for mode in ("mip", "composite"):
                need = R.workspace_bytes(mode=mode, ert=1.0)
                n = ((w + 15) // 16) * ((h + 15) // 16)
                assert need == (n * 4 + 255) // 256 * 256 + n, "bundle order not taken"
                log(f"case: noalloc call {i} {w}x{h} {mode} on the bundle kernel ({need} B of scratch)")
                ref = R.render(mode=mode, ert=1.0).cpu().numpy()
                shp = (h, w) if mode == "mip" else (h, w, 4)
                out = torch.full(shp, float("nan"), device="cuda")
                got = R.render_noalloc(mode=mode, ert=1.0, out=out).cpu().numpy()
                assert np.array_equal(got, ref), f"call {i} {mode}"
    finally:
        R.set_tuning(**base)


def test_noalloc_rejects_what_it_cannot_hold(R):
    from paper_1012_2909_amd import vr
    shape = (40, 36, 32)
    R.load_volume(torch.from_numpy(synth.make_cube(synth.CubeSpec(shape, 4, seed=32))))
    R.set_lut(synth.lut_ramp())
    assert vr.lib().vr_render_noalloc_max_bytes() == 128 << 20
    base = R.get_tuning()
    R.set_tuning(path=4)
    try:
        # 2048 x 1025 pixels of ray records exceed the 2^21 the scratch holds
        R.set_camera(synth.orbit_camera(shape, seed=1, w=2048, h=1025))
        with pytest.raises(vr.VRError) as e:
            R.render_noalloc(mode="mip")
        assert e.value.code == vr.ENOMEM
    finally:
        R.set_tuning(**base)
    R.set_camera(synth.orbit_camera(shape, seed=1, w=16, h=16))
    p = vr.params_struct("composite", "trilinear", 0.5, 0.99, "auto", True)
    out = torch.empty((16, 16, 4), device="cuda")
    rc = vr.lib().vr_render_noalloc(R.ctx, vr.C.byref(p), out.data_ptr(), None)
    assert rc == vr.EINVAL
