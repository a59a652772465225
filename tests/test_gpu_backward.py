"""GPU adjoint (vr_render_backward / VolumeRenderFn) against the FP64 oracle
adjoint, which the CPU tests pin to finite differences.

Tolerance: gradients are sums of many FP32 products accumulated with FP32
atomics in an arbitrary order; relative to the largest gradient entry we
allow 1e-4 (about 2^-13: a few hundred ulp of accumulated rounding)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1012_2909_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu
TOL_GRAD = 1e-4


@pytest.fixture(scope="module")
def R():
    from paper_1012_2909_amd import vr
    r = vr.Renderer(0)
    yield r
    r.close()


def _gpu_grads(R, vol, lut, cam, g, ert):
    R.load_volume(torch.from_numpy(vol), orientations=1)
    R.set_lut(lut)
    R.set_camera(cam)
    img, ws = R.render(ert=ert, save=True)
    gl = torch.zeros(lut.table.shape, dtype=torch.float32, device="cuda")
    gv = torch.zeros(vol.shape, dtype=torch.float32, device="cuda")
    R.render_backward(torch.from_numpy(g.astype(np.float32)), ws, gl, gv, ert=ert)
    torch.cuda.synchronize()
    return img.cpu().numpy(), gl.cpu().numpy(), gv.cpu().numpy()


def _compare(got, ref, what):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    log(f"{what}: max |err| / max |ref| = {err:.2e} (scale {scale:.3e})")
    assert scale > 0
    assert err <= TOL_GRAD, what


@pytest.mark.parametrize("tau", [1.0, 0.99])
def test_small_against_oracle(R, tau):
    vol = synth.make_cube(synth.CUBE_FD16)
    lut = synth.lut_random(55)
    lut = synth.Lut(lut.table * np.float32(0.5), lut.vmin, lut.vmax)
    cam = synth.orbit_camera(vol.shape, seed=5, w=32, h=32)
    g = np.random.default_rng(5).standard_normal((32, 32, 4))
    res = oracle.render(vol, lut, cam, tau=tau, eps_stop=1e-4)
    g[res["flags"] != 0] = 0.0             # pixels whose stop index is ambiguous
    img, gl, gv = _gpu_grads(R, vol, lut, cam, g, tau)
    ol, ov = oracle.backward(vol, lut, cam, g, tau=tau)
    _compare(gl, ol, f"table gradient tau={tau}")
    _compare(gv, ov, f"voxel gradient tau={tau}")


def test_full_size_l2_loss_through_autograd(R):
    """128x128x256 cube, 1024x1024 image, L2 loss to a target rendered with a
    hidden table; gradients through torch.autograd against the oracle."""
    from paper_1012_2909_amd.autograd import VolumeRenderFn
    vol = synth.make_cube(synth.CUBE_DIFF)
    hidden = synth.lut_random(55)
    start = synth.lut_ramp()
    cam = synth.orbit_camera(vol.shape, seed=5, w=1024, h=1024)
    tau = 0.99
    # target by the oracle (FP64) with the hidden table
    target = oracle.render(vol, hidden, cam, tau=tau, threads=0)["out"]
    v = torch.from_numpy(vol).cuda().requires_grad_(True)
    t = torch.from_numpy(start.table).cuda().requires_grad_(True)
    img = VolumeRenderFn.apply(v, t, R, cam, start.vmin, start.vmax, 0.5, tau)
    tgt = torch.from_numpy(target.astype(np.float32)).cuda()
    loss = ((img - tgt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    # the oracle adjoint with the same upstream gradient 2 (I - I*), using the
    # GPU image for I (the oracle's own image differs by <= 1e-5 per channel)
    g = 2.0 * (img.detach().cpu().numpy().astype(np.float64) - target)
    res = oracle.render(vol, start, cam, tau=tau, eps_stop=1e-4)
    amb = res["flags"] != 0
    log(f"ambiguous stop pixels: {int(amb.sum())}")
    g_masked = g.copy()
    g_masked[amb] = 0.0
    ol, ov = oracle.backward(vol, start, cam, g_masked, tau=tau)
    # GPU gradients with the same masking (through the C ABI directly)
    R.load_volume(torch.from_numpy(vol), orientations=1)
    R.set_lut(start)
    R.set_camera(cam)
    _, ws = R.render(ert=tau, save=True)
    gl = torch.zeros_like(t)
    gv = torch.zeros_like(v)
    R.render_backward(torch.from_numpy(g_masked.astype(np.float32)), ws, gl, gv, ert=tau)
    torch.cuda.synchronize()
    _compare(gl.cpu().numpy(), ol, "table gradient (1024^2)")
    _compare(gv.cpu().numpy(), ov, "voxel gradient (1024^2)")
    # and autograd's gradients equal the direct call's up to the masked pixels
    if not amb.any():
        assert torch.allclose(v.grad, gv, rtol=0, atol=TOL_GRAD * float(gv.abs().max()))


def test_backward_rejects_unsupported(R):
    from paper_1012_2909_amd import vr
    vol = synth.make_cube(synth.CUBE_FD16)
    R.load_volume(torch.from_numpy(vol), storage="f16", orientations=1)
    R.set_lut(synth.lut_ramp())
    R.set_camera(synth.orbit_camera(vol.shape, seed=5, w=8, h=8))
    _, ws = R.render(save=True)
    with pytest.raises(vr.VRError) as e:
        R.render_backward(torch.zeros((8, 8, 4)), ws, torch.zeros((256, 4), device="cuda"), None)
    assert e.value.code == vr.EUNSUPPORTED
