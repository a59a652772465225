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
    # autograd's gradients equal a direct call with the same, unmasked
    # upstream gradient: both replay the same GPU forward (the same stop
    # decisions), so no pixel needs masking and the table gradient (summed in
    # LDS, then one atomic per entry and workgroup) agrees to rounding order
    gl2 = torch.zeros_like(t)
    gv2 = torch.zeros_like(v)
    R.render_backward(torch.from_numpy(g.astype(np.float32)), ws, gl2, gv2, ert=tau)
    torch.cuda.synchronize()
    for name, a, b in (("voxel", v.grad, gv2), ("table", t.grad, gl2)):
        scale = float(b.abs().max())
        err = float((a - b).abs().max())
        log(f"autograd vs direct {name} gradient: max abs diff {err:.3e} (scale {scale:.3e})")
        assert scale > 0 and err <= 1e-5 * scale


def test_autograd_backward_uses_the_forward_scene(R):
    """The backward replays the rays of its own forward even when the
    renderer renders another camera and table in between."""
    from paper_1012_2909_amd.autograd import VolumeRenderFn
    vol = synth.make_cube(synth.CUBE_FD16)
    lut = synth.lut_ramp(alpha_scale=0.5)
    cam = synth.orbit_camera(vol.shape, seed=5, w=32, h=32)
    other = synth.orbit_camera(vol.shape, seed=9, w=32, h=32)
    grads = []
    for disturb in (False, True):
        v = torch.from_numpy(vol).cuda().requires_grad_(True)
        t = torch.from_numpy(lut.table).cuda().requires_grad_(True)
        img = VolumeRenderFn.apply(v, t, R, cam, lut.vmin, lut.vmax, 0.5, 1.0)
        if disturb:
            R.set_camera(other)
            R.set_lut(synth.lut_random(3))
            R.render(ert=1.0)
        (img ** 2).sum().backward()
        torch.cuda.synchronize()
        grads.append((v.grad.clone(), t.grad.clone()))
    for a, b in zip(grads[0], grads[1]):
        assert float((a - b).abs().max()) <= 1e-6 * float(a.abs().max())


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
