"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
closed forms, an exact-rational brute force, library routines and invariants.
CPU only.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1012_2909_amd import synth


def cube64():
    return synth.make_cube(synth.CUBE_64)


# ----------------------------------------------------------------------------
# camera
# ----------------------------------------------------------------------------
def test_axis_camera_maps_pixels_to_voxel_quarters():
    """View along z over the 64^3 face: pixel (row, col) -> x = (col+1/2)/4,
    y = (row+1/2)/4, z = -1, direction +z, exactly."""
    cam = synth.camera_axis_z()
    for col, row in [(0, 0), (255, 255), (17, 200), (128, 3)]:
        o, d = oracle.ray(cam, col, row)
        assert tuple(o) == ((col + 0.5) / 4, (row + 0.5) / 4, -1.0)
        assert tuple(d) == (0.0, 0.0, 1.0)


def test_perspective_basis_invariants():
    cam = synth.orbit_camera((128, 64, 96), seed=11, w=640, h=360)
    f, r, u = oracle.basis(cam)
    tgt = np.array(cam.target) - np.array(cam.eye)
    assert np.allclose(f, tgt / np.linalg.norm(tgt), atol=1e-15)
    assert abs(np.dot(f, r)) < 1e-15 and abs(np.dot(f, u)) < 1e-15 and abs(np.dot(r, u)) < 1e-15
    # right-handed: r x u = -f; up lies in the (f, u) plane on u's side
    assert np.allclose(np.cross(r, u), -f, atol=1e-15)
    assert np.dot(np.array(cam.up), u) > 0 and abs(np.dot(np.array(cam.up), r)) < 1e-12


def test_perspective_ray_angles():
    """A pixel's ray makes angle atan(|(sx, sy)|) with the view axis, where the
    frame's vertical half-extent is tan(fovy/2); rays are unit vectors."""
    W, H = 320, 200
    cam = synth.orbit_camera((64, 64, 64), seed=3, w=W, h=H, fovy_deg=40.0)
    f, r, u = oracle.basis(cam)
    th = math.tan(math.radians(20.0))
    for col, row in [(0, 0), (W - 1, H - 1), (160, 100), (7, 190)]:
        o, d = oracle.ray(cam, col, row)
        assert abs(np.linalg.norm(d) - 1) < 1e-15
        assert np.array_equal(o, np.array(cam.eye))
        # image-plane coordinates (distance 1 along f)
        x = np.dot(d, r) / np.dot(d, f)
        y = np.dot(d, u) / np.dot(d, f)
        assert abs(x - ((col + 0.5) / W * 2 - 1) * th * W / H) < 1e-13
        assert abs(y - (1 - (row + 0.5) / H * 2) * th) < 1e-13


# ----------------------------------------------------------------------------
# clip and sample count
# ----------------------------------------------------------------------------
def _inside(p, n):
    return all(0.0 <= p[a] <= n[a] for a in range(3))


def test_sample_count_matches_membership_bisection():
    """n = number of midpoint samples inside the chord, where the chord's
    entry/exit are found by bisection on box membership (no slab formulas)."""
    shape = (40, 24, 32)
    nz, ny, nx = shape
    cam = synth.orbit_camera(shape, seed=5, w=64, h=48)
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(60):
        col, row = int(rng.integers(0, 64)), int(rng.integers(0, 48))
        hit, t0, t1, n, o, d = oracle.ray_interval(shape, cam, col, row)
        # locate the chord by dense scan then bisection
        ts = np.linspace(0, 3 * np.linalg.norm(np.array(cam.eye)), 20001)
        ins = [_inside(o + t * d, (nx, ny, nz)) for t in ts]
        if not any(ins):
            assert not hit or n == 0
            continue
        i0 = ins.index(True)
        i1 = len(ins) - 1 - ins[::-1].index(True)

        def bis(a, b, want_inside_at_b):
            for _ in range(200):
                m = 0.5 * (a + b)
                if _inside(o + m * d, (nx, ny, nz)) == want_inside_at_b:
                    b = m
                else:
                    a = m
            return b

        te = bis(ts[i0 - 1], ts[i0], True)
        tx = bis(ts[i1 + 1], ts[i1], True)
        assert abs(te - t0) < 1e-9 and abs(tx - t1) < 1e-9
        L = tx - te
        n_ref = sum(1 for k in range(int(L / 0.5) + 3) if (k + 0.5) * 0.5 < L)
        assert n == n_ref
        checked += 1
    assert checked > 10


# ----------------------------------------------------------------------------
# P1: constant cube closed form
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("v0", [-1.0, 0.5, 2.25])
@pytest.mark.parametrize("tau", [1.0, 0.99])
def test_constant_cube_closed_form_axis(v0, tau):
    vol = np.full((64, 64, 64), v0, np.float32)
    lut = synth.lut_ramp()
    a = min(max((v0 + 3) / 13, 0), 1)
    cam = synth.camera_axis_z(w=32, h=32)
    res = oracle.render(vol, lut, cam, tau=tau)
    n = 128
    if tau < 1:
        n = min(n, math.ceil(math.log(1 - tau) / math.log(1 - a)))
    A = 1 - (1 - a) ** n
    img = res["out"]
    # table entries are float32(j/255); interpolation reproduces a to ~3e-8
    assert np.allclose(img[..., 3], A, atol=1e-7, rtol=0)
    assert np.allclose(img[..., 0], a * A, atol=1e-7, rtol=0)
    assert (res["taken"] == n).all()


def test_constant_cube_closed_form_oblique():
    """Per perspective ray: A = 1 - (1-a)^n with that ray's sample count."""
    shape = (48, 40, 56)
    vol = np.full(shape, 1.0, np.float32)
    lut = synth.lut_ramp(alpha_scale=1 / 16)
    cam = synth.orbit_camera(shape, seed=9, w=48, h=36)
    res = oracle.render(vol, lut, cam, tau=1.0)
    a = float(oracle.lut_eval(lut, 1.0)[0][3])
    c = float(oracle.lut_eval(lut, 1.0)[0][0])
    n = res["taken"]
    A_ref = 1 - (1 - a) ** n
    assert np.abs(res["out"][..., 3] - A_ref).max() < 1e-13
    assert np.abs(res["out"][..., 0] - c * A_ref).max() < 1e-13
    assert (n > 0).sum() > 200


# ----------------------------------------------------------------------------
# P2: nearest MIP = per-column max
# ----------------------------------------------------------------------------
def test_nearest_mip_is_column_max():
    vol = cube64()
    cam = synth.camera_axis_z()
    res = oracle.render(vol, synth.lut_ramp(), cam, mode="mip", filt="nearest")
    colmax = vol.max(axis=0)                         # (ny, nx)
    ref = np.repeat(np.repeat(colmax, 4, axis=0), 4, axis=1).astype(np.float64)
    assert np.array_equal(res["out"], ref)
    assert (res["flags"] == 0).all()


# ----------------------------------------------------------------------------
# P8: textbook recurrence along columns
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [1.0, 0.99])
def test_nearest_composite_is_column_recurrence(tau):
    vol = cube64()
    lut = synth.lut_ramp()
    cam = synth.camera_axis_z(w=64, h=64)   # one ray per voxel column (centres)
    res = oracle.render(vol, lut, cam, filt="nearest", tau=tau)
    # straight RGBA per voxel by numpy's piecewise-linear interpolation
    xk = np.linspace(lut.vmin, lut.vmax, lut.table.shape[0])
    rgba = np.stack([np.interp(vol.astype(np.float64), xk, lut.table[:, c].astype(np.float64))
                     for c in range(4)], axis=-1)        # (nz, ny, nx, 4)
    C = np.zeros((64, 64, 3))
    A = np.zeros((64, 64))
    done = np.zeros((64, 64), bool)
    for z in range(64):
        for _rep in range(2):       # step 1/2: each voxel is sampled twice
            a = rgba[z, :, :, 3]
            live = ~done
            C[live] += ((1 - A) * a)[live][:, None] * rgba[z, :, :, :3][live]
            A[live] += ((1 - A) * a)[live]
            if tau < 1:
                done |= A >= tau
    ref = np.concatenate([C, A[..., None]], axis=-1)
    assert np.abs(res["out"] - ref).max() < 1e-14


# ----------------------------------------------------------------------------
# P5 / P6: the table
# ----------------------------------------------------------------------------
def test_ramp_table_identity():
    lut = synth.lut_ramp()
    for s in np.linspace(-5, 12, 301):
        rgba = oracle.lut_eval(lut, s)[0]
        x = min(max((s + 3) / 13, 0), 1)
        assert np.abs(rgba - x).max() < 6e-8        # entries are float32(j/255)


def test_table_matches_numpy_interp():
    lut = synth.lut_random(4)
    xk = np.linspace(lut.vmin, lut.vmax, 256)
    for s in np.random.default_rng(1).uniform(-4, 11, 200):
        rgba = oracle.lut_eval(lut, s)[0]
        ref = [np.interp(s, xk, lut.table[:, c].astype(np.float64)) for c in range(4)]
        assert np.abs(rgba - ref).max() < 1e-14


def test_degenerate_tables():
    vol = cube64()
    cam = synth.orbit_camera(vol.shape, seed=2, w=40, h=30)
    t0 = synth.lut_ramp().table.copy()
    t0[:, 3] = 0
    z = oracle.render(vol, synth.Lut(t0, -3, 10), cam)
    assert np.array_equal(z["out"], np.zeros_like(z["out"]))
    t1 = synth.lut_random(7).table.copy()
    t1[:, 3] = 1
    lut1 = synth.Lut(t1, -3, 10)
    one = oracle.render(vol, lut1, cam)
    hitm = one["taken"] > 0
    assert (one["taken"][hitm] == 1).all()           # alpha 1 stops at the first sample
    # colour = table colour at the first sample's trilinear value
    rows, cols = np.nonzero(hitm)
    for (r_, c_) in list(zip(rows, cols))[:50]:
        hit, t0_, t1_, n, o, d = oracle.ray_interval(vol.shape, cam, c_, r_)
        p = o + (t0_ + 0.25) * d
        s, _, _ = oracle.trilinear(vol, p)
        rgba = oracle.lut_eval(lut1, s)[0]
        assert np.abs(one["out"][r_, c_] - np.r_[rgba[:3], 1.0]).max() < 1e-15


# ----------------------------------------------------------------------------
# trilinear: linear functions are reproduced
# ----------------------------------------------------------------------------
def test_trilinear_reproduces_linear_field():
    nz, ny, nx = 7, 5, 9
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c, d0 = 0.25, -0.5, 0.125, 2.0
    vol = (a * (i + 0.5) + b * (j + 0.5) + c * (k + 0.5) + d0).astype(np.float32)
    rng = np.random.default_rng(4)
    for _ in range(200):
        p = rng.uniform([0, 0, 0], [nx, ny, nz])
        q = np.clip(p, 0.5, np.array([nx, ny, nz]) - 0.5)      # clamp-to-edge extension
        ref = a * q[0] + b * q[1] + c * q[2] + d0
        v, idx, wt = oracle.trilinear(vol, p)
        assert abs(v - ref) < 1e-12
        assert abs(wt.sum() - 1) < 1e-15 and (wt >= 0).all()
        assert abs(np.dot(wt, vol.reshape(-1)[idx].astype(np.float64)) - v) < 1e-12


# ----------------------------------------------------------------------------
# P4: exact-rational brute force on 2^3 and 3^3 volumes
# ----------------------------------------------------------------------------
def _exact_case(n, seed):
    rng = np.random.default_rng(seed)
    vol = (rng.integers(-24, 80, size=(n, n, n)) / 8.0).astype(np.float32)   # dyadic
    table = (rng.integers(0, 17, size=(5, 4)) / 16.0).astype(np.float32)
    lut = synth.Lut(table, -4.0, 12.0)
    return vol, lut


BASES = {
    # f, r, u exact rational unit vectors with r = f x up (unit), u = r x f
    "oblique": ((F(1, 3), F(2, 3), F(2, 3)), (F(2, 3), F(1, 3), F(-2, 3)), (F(2, 3), F(-2, 3), F(1, 3))),
    "axis_x": ((F(1), F(0), F(0)), (F(0), F(0), F(1)), (F(0), F(1), F(0))),
}


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("basis", ["oblique", "axis_x"])
@pytest.mark.parametrize("mode", ["composite", "mip", "mip_nearest"])
def test_brute_force_tiny(n, basis, mode):
    vol, lut = _exact_case(n, seed=10 * n + len(basis))
    f, r, u = BASES[basis]
    c0 = [F(n, 2)] * 3
    eye = [c0[a] - 3 * n * f[a] for a in range(3)]
    W = H = 6
    half = F(3 * n, 4)
    # target and up are exact integer multiples of f and u
    cam = synth.Camera(synth.ORTHO, tuple(float(e) for e in eye),
                       tuple(float(e + 3 * fa) for e, fa in zip(eye, f)),
                       tuple(float(3 * x) for x in u), half_w=float(half), half_h=float(half),
                       full_w=W, full_h=H)
    # the oracle's basis is the exact one up to FP64 rounding
    fo, ro, uo = oracle.basis(cam)
    assert np.abs(fo - np.array([float(x) for x in f])).max() < 1e-15
    assert np.abs(ro - np.array([float(x) for x in r])).max() < 1e-15
    assert np.abs(uo - np.array([float(x) for x in u])).max() < 1e-15
    Vq = brute.to_frac_volume(vol)
    Lq = brute.to_frac_lut(lut.table)
    m = "mip" if mode.startswith("mip") else "composite"
    filt = "nearest" if mode == "mip_nearest" else "trilinear"
    res = oracle.render(vol, lut, cam, mode=m, filt=filt, tau=0.99)
    hits = exact = 0
    for row in range(H):
        for col in range(W):
            ref = brute.render_pixel(Vq, Lq, F(-4), F(12), eye, f, r, u, half, half, W, H, col, row,
                                     mode=m, filt=filt)
            got = res["out"][row, col]
            fl = res["flags"][row, col]
            # a dyadic exit can coincide with a sample (t_k = t1 exactly): FP64
            # may then keep or drop it, and the oracle lists both outcomes
            cands = [got] + ([res["lo"][row, col], res["hi"][row, col]] if fl else [])
            if m == "mip":
                if ref is None:
                    assert got == -np.inf
                    continue
                hits += 1
                if filt == "nearest" and fl == 0:
                    assert got == float(ref)
                else:
                    assert min(abs(c - float(ref)) for c in cands) <= 1e-12 * max(1.0, abs(float(ref)))
            else:
                ref = np.array([float(x) for x in ref])
                if ref[3] > 0:
                    hits += 1
                assert min(np.abs(c - ref).max() for c in cands) <= 1e-12
            exact += fl == 0
    assert hits >= 4 and exact >= 12


# ----------------------------------------------------------------------------
# P3: bricks composited separately equal the single pass (no early stop)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("B", [1, 5, 7, 16, 100])
@pytest.mark.parametrize("kind", ["persp", "ortho"])
def test_bricked_equals_single_pass(B, kind):
    shape = (20, 14, 17)
    spec = synth.CubeSpec(shape, 6, seed=21)
    vol = synth.make_cube(spec)
    lut = synth.lut_ramp(alpha_scale=1 / 8)
    if kind == "persp":
        cam = synth.orbit_camera(shape, seed=B, w=40, h=30)
    else:
        cam = synth.Camera(synth.ORTHO, (-30.0, 25.0, -20.0), (8.5, 7.0, 10.0), (0.0, -1.0, 0.0),
                           half_w=16.0, half_h=12.0, full_w=40, full_h=30)
    one = oracle.render(vol, lut, cam, tau=1.0)["out"]
    br = oracle.render_bricked(vol, lut, cam, B, tau=1.0)["out"]
    assert np.abs(one - br).max() <= 1e-12
    mip1 = oracle.render(vol, lut, cam, mode="mip", tau=1.0)["out"]
    mipb = oracle.render_bricked(vol, lut, cam, B, mode="mip")["out"]
    assert np.array_equal(mip1, mipb)


def test_brick_keys_increase_along_rays():
    """The key order is a visibility order: along every ray the bricks visited
    have strictly increasing keys (perspective and orthographic)."""
    shape = (40, 32, 48)
    B = 8
    for cam in [synth.orbit_camera(shape, seed=s, w=30, h=20) for s in range(4)] + [
            synth.Camera(synth.ORTHO, (-50.0, 60.0, 70.0), (24.0, 16.0, 20.0), (0.0, -1.0, 0.0),
                         half_w=40.0, half_h=30.0, full_w=30, full_h=20)]:
        for row in range(0, 20, 3):
            for col in range(0, 30, 3):
                hit, t0, t1, n, o, d = oracle.ray_interval(shape, cam, col, row)
                if not hit:
                    continue
                keys, last = [], None
                for k in range(n):
                    p = o + (t0 + (k + 0.5) * 0.5) * d
                    cell = tuple(min(int(p[a] // B), [48, 32, 40][a] // B - 1) for a in range(3))
                    if cell != last:
                        keys.append(oracle.brick_key(cam, B, *cell))
                        last = cell
                assert all(b > a for a, b in zip(keys, keys[1:]))


# ----------------------------------------------------------------------------
# candidate intervals
# ----------------------------------------------------------------------------
def test_candidate_interval_brackets_primary():
    vol = cube64()
    cam = synth.orbit_camera(vol.shape, seed=1, w=96, h=96)
    res = oracle.render(vol, synth.lut_ramp(), cam, eps_stop=1e-3)
    o, lo, hi = res["out"], res["lo"], res["hi"]
    assert (lo <= o + 1e-15).all() and (o <= hi + 1e-15).all()
    amb = (res["flags"] & oracle.FLAG_STOP) != 0
    assert amb.any()
    assert np.array_equal(lo[~amb], o[~amb]) and np.array_equal(hi[~amb], o[~amb])


# ----------------------------------------------------------------------------
# P9: gradients
# ----------------------------------------------------------------------------
def test_adjoint_constant_cube_closed_form():
    """dA/da = n (1-a)^(n-1) on a constant cube along z (a through alpha entries)."""
    vol = np.full((16, 16, 16), 2.0, np.float32)
    t = np.zeros((2, 4), np.float32)
    t[:, 3] = 0.125                      # constant alpha a = 1/8, colour 0
    lut = synth.Lut(t, -3, 10)
    cam = synth.camera_axis_z(16, 16, 16, w=4, h=4)
    g = np.zeros((4, 4, 4))
    g[..., 3] = 1.0                      # L = sum of A over pixels
    gl, gv = oracle.backward(vol, lut, cam, g, tau=1.0)
    n, a = 32, 0.125
    dA = n * (1 - a) ** (n - 1)
    # a = (1-w) L[0,3] + w L[1,3]; the two weights sum to one per sample
    assert abs(gl[:, 3].sum() - 16 * dA) < 1e-12
    assert np.abs(gv).max() == 0.0       # flat table: no value sensitivity


@pytest.mark.parametrize("tau", [1.0, 0.99])
def test_adjoint_matches_finite_differences(tau):
    vol = synth.make_cube(synth.CUBE_FD16)
    lut = synth.lut_random(55, n=256)
    lut = synth.Lut(lut.table * np.float32(0.5), lut.vmin, lut.vmax)
    cam = synth.orbit_camera(vol.shape, seed=5, w=32, h=32)
    rng = np.random.default_rng(5)
    g = rng.standard_normal((32, 32, 4))

    def loss(v, L):
        out = oracle.render(v, L, cam, tau=tau, threads=8)["out"]
        return float(np.sum(g * out))

    gl, gv = oracle.backward(vol, lut, cam, g, tau=tau)
    # table entries: the image is a polynomial in them, FD is exact to O(h^2)
    h = 1e-6
    base = lut.table.astype(np.float64)
    fd_l = np.zeros_like(base)
    for j in range(base.shape[0]):
        for c in range(4):
            tp, tm = base.copy(), base.copy()
            tp[j, c] += h
            tm[j, c] -= h
            # the table is float32 at the interface: perturb in float64 through a float32-exact step
            lp = synth.Lut(tp.astype(np.float32), lut.vmin, lut.vmax)
            lm = synth.Lut(tm.astype(np.float32), lut.vmin, lut.vmax)
            dh = float(lp.table[j, c]) - float(lm.table[j, c])
            fd_l[j, c] = (loss(vol, lp) - loss(vol, lm)) / dh
    scale_l = np.abs(gl).max()
    assert scale_l > 0
    assert np.abs(fd_l - gl).max() <= 1e-6 * scale_l
    # voxels: skip entries whose one-sided differences disagree (a table knot,
    # a clamp or a stop decision lies within h)
    hv = 2.0 ** -20
    flat = vol.reshape(-1)
    l0 = loss(vol, lut)
    errs, skipped = [], 0
    for idx in range(flat.size):
        vp, vm = flat.copy(), flat.copy()
        vp[idx] += np.float32(hv)
        vm[idx] -= np.float32(hv)
        hp = float(vp[idx]) - float(flat[idx])     # the float32-exact steps
        hm = float(flat[idx]) - float(vm[idx])
        lp = loss(vp.reshape(vol.shape), lut)
        lm = loss(vm.reshape(vol.shape), lut)
        fwd, bwd = (lp - l0) / hp, (l0 - lm) / hm
        if abs(fwd - bwd) > 1e-4 * max(1.0, abs(fwd)):
            skipped += 1
            continue
        errs.append(abs(0.5 * (fwd + bwd) - gv.reshape(-1)[idx]))
    scale_v = np.abs(gv).max()
    assert skipped < 0.01 * flat.size
    assert max(errs) <= 1e-6 * scale_v


# ----------------------------------------------------------------------------
# exact ties and an eye inside the cube
# ----------------------------------------------------------------------------
def test_sample_on_exit_face_is_excluded():
    """Step 2 along z through 5 planes: samples at z = 1, 3, 5; the one on the
    exit face (t_k = t1 exactly) is not taken."""
    vol = synth.make_cube(synth.CubeSpec((5, 4, 4), 1, seed=3))
    cam = synth.camera_axis_z(4, 4, 5, w=4, h=4)
    res = oracle.render(vol, synth.lut_ramp(), cam, mode="mip", filt="nearest", step=2.0, tau=1.0)
    assert (res["taken"] == 2).all()
    assert np.array_equal(res["out"], vol[[1, 3]].max(axis=0).astype(np.float64))


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_eye_inside_cube_starts_at_eye(kind):
    vol = np.full((64, 64, 64), 0.5, np.float32)
    if kind == "ortho":
        cam = synth.Camera(synth.ORTHO, (32.0, 32.0, 10.0), (32.0, 32.0, 11.0), (0.0, -1.0, 0.0),
                           half_w=8.0, half_h=8.0, full_w=8, full_h=8)
        res = oracle.render(vol, synth.lut_ramp(), cam, tau=1.0)
        assert (res["taken"] == 108).all()        # (k + 1/2)/2 < 54
    else:
        cam = synth.Camera(synth.PERSPECTIVE, (32.0, 32.0, 32.0), (32.0, 32.0, 40.0), (0.0, -1.0, 0.0),
                           fovy_deg=60.0, full_w=8, full_h=8)
        res = oracle.render(vol, synth.lut_ramp(), cam, tau=1.0)
        for row in range(8):
            for col in range(8):
                hit, t0, t1, n, o, d = oracle.ray_interval(vol.shape, cam, col, row)
                assert t0 == 0.0 and hit
                # exit distance to the z = 64 face (the nearest exit for this frustum)
                assert abs(t1 - 32.0 / d[2]) < 1e-12
                assert res["taken"][row, col] == math.ceil(t1 / 0.5 - 0.5)


# ----------------------------------------------------------------------------
# brick partition: per-brick partials are the column recurrence over the
# brick's z-range, with the brick's own early stop
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [1.0, 0.99])
def test_brick_partials_are_column_segments(tau):
    vol = cube64()
    lut = synth.lut_ramp(alpha_scale=0.25)
    B = 16
    cam = synth.camera_axis_z(w=64, h=64)
    xk = np.linspace(lut.vmin, lut.vmax, lut.table.shape[0])
    rgba = np.stack([np.interp(vol.astype(np.float64), xk, lut.table[:, c].astype(np.float64))
                     for c in range(4)], axis=-1)
    parts = []
    for bz in range(4):
        C = np.zeros((64, 64, 3))
        A = np.zeros((64, 64))
        done = np.zeros((64, 64), bool)
        for z in range(bz * B, bz * B + B):
            for _rep in range(2):
                a = rgba[z, :, :, 3]
                live = ~done
                C[live] += ((1 - A) * a)[live][:, None] * rgba[z, :, :, :3][live]
                A[live] += ((1 - A) * a)[live]
                if tau < 1:
                    done |= A >= tau
        parts.append(np.concatenate([C, A[..., None]], axis=-1))
    for bz in range(4):
        for (bx, by) in [(0, 0), (3, 1)]:
            bid = (bz * 4 + by) * 4 + bx
            got = oracle.render_bricked(vol, lut, cam, B, filt="nearest", tau=tau, only_brick=bid)["out"]
            sl = np.s_[by * 16:(by + 1) * 16, bx * 16:(bx + 1) * 16]
            assert np.abs(got[sl] - parts[bz][sl]).max() < 1e-14
            mask = np.ones((64, 64), bool)
            mask[sl] = False
            assert not got[mask].any()
    full = oracle.render_bricked(vol, lut, cam, B, filt="nearest", tau=tau)["out"]
    ref = np.zeros((64, 64, 4))
    for bz in range(4):                       # +z view: keys increase with bz
        ref = ref + (1 - ref[..., 3:4]) * parts[bz]
    assert np.abs(full - ref).max() < 1e-14


# ----------------------------------------------------------------------------
# candidate outcomes, pinned one decision at a time: each case builds an exact
# tie of one discontinuous decision (the exit test, the stop test, the nearest
# cell) on a single axis-aligned ray, and the oracle's lo / hi must equal the
# exact-rational render with that one decision flipped by hand
# ----------------------------------------------------------------------------
def _axis_ray_camera(x, y):
    """Orthographic 1x1 frame whose single ray starts at (x, y, -1) and runs
    along +z (sx = sy = 0, so the origin is the eye exactly)."""
    return synth.Camera(synth.ORTHO, (x, y, -1.0), (x, y, 0.0), (0.0, -1.0, 0.0),
                        half_w=0.5, half_h=0.5, full_w=1, full_h=1)


_AXIS_BASIS = ((F(0), F(0), F(1)), (F(1), F(0), F(0)), (F(0), F(-1), F(0)))


def _brute_axis(vol, lut, x, y, **kw):
    f, r, u = _AXIS_BASIS
    return brute.render_pixel(brute.to_frac_volume(vol), brute.to_frac_lut(lut.table), F(lut.vmin), F(lut.vmax),
                              [F(x), F(y), F(-1)], f, r, u, F(1, 2), F(1, 2), 1, 1, 0, 0, **kw)


def _frac_close(got, ref, tol=1e-15):
    ref = np.atleast_1d(np.array([float(v) for v in np.atleast_1d(ref)]))
    return np.abs(np.atleast_1d(got) - ref).max() <= tol


def test_count_candidates_flip_the_exit_test():
    """Samples at z = 0.5, 1.5, 2.5, 3.5 of a 4-deep column (t0 = 1, t1 = 5,
    step 1).  A window of 0.55 around t1 reaches the last sample inside
    (t = 4.5) and the first one outside (t = 5.5): lo is the render that drops
    the last sample (3 samples), hi the render that takes one more (5), out
    the render of the 4 of the definition."""
    vol = np.array([-2.0, 5.0, 1.5, 7.25], np.float32).reshape(4, 1, 1)
    lut = synth.lut_dyadic([[0, 0, 0, 0], [1.0, 0.5, 0.25, 0.5]], -4.0, 12.0)
    cam = _axis_ray_camera(0.5, 0.5)
    eps_t = 0.11   # window = eps_t * |t1| = 0.55 > 0.5
    res = oracle.render(vol, lut, cam, step=1.0, tau=1.0, eps_t=eps_t)
    assert res["flags"][0, 0] == oracle.FLAG_COUNT and res["taken"][0, 0] == 4
    for key, count in (("out", None), ("lo", 3), ("hi", 5)):
        ref = _brute_axis(vol, lut, 0.5, 0.5, step=F(1), tau=F(1), count=count)
        assert _frac_close(res[key][0, 0], ref), key
    # the candidates differ from each other (so an off-by-one is visible)
    assert len({tuple(res[k][0, 0]) for k in ("out", "lo", "hi")}) == 3
    mip = oracle.render(vol, lut, cam, mode="mip", step=1.0, eps_t=eps_t)
    for key, count in (("out", None), ("lo", 3), ("hi", 5)):
        assert mip[key][0, 0] == float(_brute_axis(vol, lut, 0.5, 0.5, step=F(1), mode="mip", count=count)), key
    assert mip["lo"][0, 0] == 5.0 and mip["out"][0, 0] == 7.25
    # outside the window nothing is flagged and all three agree
    tight = oracle.render(vol, lut, cam, step=1.0, tau=1.0, eps_t=0.09)
    assert tight["flags"][0, 0] == 0
    assert np.array_equal(tight["lo"], tight["out"]) and np.array_equal(tight["hi"], tight["out"])


@pytest.mark.parametrize("side", [-1, 1])
def test_stop_candidates_flip_the_stop_test(side):
    """Constant alpha 1/2 (table rgba = s on [0, 1], cube of 0.5): A runs 1/2,
    3/4, 7/8 exactly.  With tau = 3/4 -/+ eps/2 the threshold lies inside the
    window around A = 3/4: lo is the render that stops at tau - eps, hi the
    one that stops at tau + eps (the exact render with the stop test moved),
    and the closed form C = A/2, A = 1 - 2^-n holds for each."""
    vol = np.full((8, 1, 1), 0.5, np.float32)
    lut = synth.lut_dyadic([[0, 0, 0, 0], [1, 1, 1, 1]], 0.0, 1.0)
    cam = _axis_ray_camera(0.5, 0.5)
    eps = 1e-3
    tau = 0.75 + side * eps / 2
    res = oracle.render(vol, lut, cam, step=1.0, tau=tau, eps_stop=eps)
    assert res["flags"][0, 0] & oracle.FLAG_STOP
    n_main = 2 if side < 0 else 3
    for key, t, n in (("out", F(tau), n_main), ("lo", F(tau) - F(eps), 2), ("hi", F(tau) + F(eps), 3)):
        ref = _brute_axis(vol, lut, 0.5, 0.5, step=F(1), tau=t)
        assert _frac_close(res[key][0, 0], ref), key
        A = 1.0 - 0.5 ** n
        assert np.array_equal(res[key][0, 0], [A / 2, A / 2, A / 2, A]), key
    assert res["taken"][0, 0] == n_main


def test_cell_candidates_flip_the_nearest_cell():
    """Nearest MIP along z through x = 3 exactly (the face between voxels 2
    and 3) and through x = 3 - 2^-30 (just inside voxel 2): the candidates
    are the two voxels on either side of that face and no other.  Voxels one
    further away hold the extremes (10 and -5), so a window that reached them
    would show."""
    vals = np.array([0.0, 10.0, 1.0, 2.0, -5.0, 7.0], np.float32)
    vol = vals.reshape(1, 1, 6)
    lut = synth.lut_ramp()
    for x, main, other, off in ((3.0, 2.0, 1.0, -1), (3.0 - 2.0 ** -30, 1.0, 2.0, 1)):
        cam = _axis_ray_camera(x, 0.5)
        res = oracle.render(vol, lut, cam, mode="mip", filt="nearest")
        assert res["flags"][0, 0] == oracle.FLAG_CELL
        ref_main = _brute_axis(vol, lut, x, 0.5, mode="mip", filt="nearest")
        ref_flip = _brute_axis(vol, lut, x, 0.5, mode="mip", filt="nearest", cell_offset=(F(off), F(0), F(0)))
        assert (float(ref_main), float(ref_flip)) == (main, other)
        assert res["out"][0, 0] == main
        assert res["lo"][0, 0] == min(main, other) and res["hi"][0, 0] == max(main, other)


# ----------------------------------------------------------------------------
# bricks with the eye inside the brick grid
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("B", [5, 7, 16])
@pytest.mark.parametrize("eye,target", [((7.3, 6.7, 11.1), (30.0, 2.0, 18.0)),
                                        ((12.6, 3.4, 4.2), (-8.0, 12.0, 16.0))])
def test_bricked_equals_single_pass_eye_inside_grid(B, eye, target):
    """Perspective eye inside the cube (so inside the brick grid, off every
    brick face): rays leave the eye's brick in all directions, and the
    Manhattan key from the eye's cell must still order the partials front to
    back.  Without early stop the bricked render equals the single pass."""
    shape = (20, 14, 17)
    vol = synth.make_cube(synth.CubeSpec(shape, 6, seed=22))
    lut = synth.lut_ramp(alpha_scale=1 / 4)
    cam = synth.Camera(synth.PERSPECTIVE, eye, target, (0.0, -1.0, 0.0), fovy_deg=100.0, full_w=40, full_h=30)
    one = oracle.render(vol, lut, cam, tau=1.0)["out"]
    br = oracle.render_bricked(vol, lut, cam, B, tau=1.0)["out"]
    assert one[..., 3].min() > 0.05          # every ray composites several bricks
    assert np.abs(one - br).max() <= 1e-12


def test_bricked_stop_candidates_cover_every_combination():
    """Two bricks of 4 samples each along one axis ray, constant alpha 1/2,
    tau = 3/4 + eps/2: each brick stops after 3 samples (A = 7/8), or after 2
    with the stop decision flipped (A = 3/4).  The "over" of the two partials
    is then 1 - 2^-(n0+n1) with n0, n1 in {2, 3}: the candidate interval
    spans both bricks flipped (1 - 2^-4) to neither (1 - 2^-6), with C = A/2
    throughout."""
    vol = np.full((8, 1, 1), 0.5, np.float32)
    lut = synth.lut_dyadic([[0, 0, 0, 0], [1, 1, 1, 1]], 0.0, 1.0)
    cam = _axis_ray_camera(0.5, 0.5)
    eps = 1e-3
    res = oracle.render_bricked(vol, lut, cam, 4, step=1.0, tau=0.75 + eps / 2, eps_stop=eps)
    assert res["flags"][0, 0] & oracle.FLAG_STOP
    for key, n in (("out", 6), ("lo", 4), ("hi", 6)):
        A = 1.0 - 0.5 ** n
        assert np.array_equal(res[key][0, 0], [A / 2, A / 2, A / 2, A]), key
    # without a tie in the window the interval collapses onto the result
    res = oracle.render_bricked(vol, lut, cam, 4, step=1.0, tau=0.8, eps_stop=eps)
    assert res["flags"][0, 0] == 0
    assert np.array_equal(res["lo"], res["out"]) and np.array_equal(res["hi"], res["out"])


def test_bricked_candidates_bracket_the_result():
    """On a noisy cube with early stop, every bricked result lies inside its
    candidate interval, unflagged pixels have a collapsed interval, and the
    flagged ones include stop ties."""
    shape = (24, 20, 22)
    vol = synth.make_cube(synth.CubeSpec(shape, 8, seed=23))
    lut = synth.lut_ramp(alpha_scale=0.5)
    cam = synth.orbit_camera(shape, seed=7, w=48, h=40)
    res = oracle.render_bricked(vol, lut, cam, 7, eps_stop=1e-3)
    o, lo, hi, fl = res["out"], res["lo"], res["hi"], res["flags"]
    assert (lo <= o + 1e-15).all() and (o <= hi + 1e-15).all()
    clean = fl == 0
    assert np.array_equal(lo[clean], o[clean]) and np.array_equal(hi[clean], o[clean])
    assert ((fl & oracle.FLAG_STOP) != 0).any()


# ----------------------------------------------------------------------------
# depth and catalogue overlay
# ----------------------------------------------------------------------------
def test_depth_composite_closed_form():
    """Constant alpha 1/2 along one axis ray (t0 = 1, step 1): A after k + 1
    samples is 1 - 2^-(k+1), so the first crossing of level 0.8 is sample 2
    (t = 3.5); level 0.5 is reached exactly at sample 0, a tie whose flipped
    outcomes are samples 0 and 1 (t = 1.5, 2.5); a level above the early
    stop's A is never reached."""
    vol = np.full((8, 1, 1), 0.5, np.float32)
    lut = synth.lut_dyadic([[0, 0, 0, 0], [1, 1, 1, 1]], 0.0, 1.0)
    cam = _axis_ray_camera(0.5, 0.5)
    d = oracle.depth(vol, lut, cam, step=1.0, tau=1.0, level=0.8)
    assert d["out"][0, 0] == 3.5 and d["flags"][0, 0] == 0 and d["lo"][0, 0] == d["hi"][0, 0] == 3.5
    d = oracle.depth(vol, lut, cam, step=1.0, tau=1.0, level=0.5, eps_stop=1e-3)
    assert d["out"][0, 0] == 1.5 and d["lo"][0, 0] == 1.5 and d["hi"][0, 0] == 2.5
    assert d["flags"][0, 0] & oracle.FLAG_STOP
    # early stop at tau 0.7 (after sample 1, A = 3/4) comes before level 0.9
    d = oracle.depth(vol, lut, cam, step=1.0, tau=0.7, level=0.9)
    assert d["out"][0, 0] == np.inf


def test_depth_mip_first_maximum():
    """Nearest MIP along z through column x = 2 (t = z + 1): the maximum 9
    sits in voxels z = 3 and z = 5; the depth is the first sample inside
    z = 3 (z = 3.25 at step 0.5, t = 4.25).  A miss has infinite depth."""
    vol = np.zeros((8, 1, 4), np.float32)
    vol[3, 0, 2] = 9.0
    vol[5, 0, 2] = 9.0
    vol[6, 0, 1] = 11.0
    lut = synth.lut_ramp()
    d = oracle.depth(vol, lut, _axis_ray_camera(2.5, 0.5), mode="mip", filt="nearest")
    assert d["out"][0, 0] == 4.25 and d["flags"][0, 0] == 0
    d = oracle.depth(vol, lut, _axis_ray_camera(1.5, 0.5), mode="mip", filt="nearest")
    assert d["out"][0, 0] == 7.25
    d = oracle.depth(vol, lut, _axis_ray_camera(7.5, 0.5), mode="mip", filt="nearest")
    assert d["out"][0, 0] == np.inf
    # trilinear: samples at z = 3.25 and 3.75 both read 3/4 of the 9 (6.75),
    # and so do z = 5.25 and 5.75; the first of them is the depth, and with a
    # value window any of the four could be first
    d = oracle.depth(vol, lut, _axis_ray_camera(2.5, 0.5), mode="mip")
    assert d["out"][0, 0] == 4.25 and d["flags"][0, 0] == 0
    d = oracle.depth(vol, lut, _axis_ray_camera(2.5, 0.5), mode="mip", eps_val=1e-6)
    assert d["out"][0, 0] == 4.25
    assert d["lo"][0, 0] == 4.25 and d["hi"][0, 0] == 6.75 and d["flags"][0, 0] & oracle.FLAG_CELL


def test_overlay_orthographic_by_hand():
    """View along +z over the 64^3 face at 256^2 (pixel centre (c+1/2,
    row+1/2) <-> world (x, y) = ((c+1/2)/4, (row+1/2)/4)).  A box over
    x in [8, 16], y in [8, 12], z in [10, 20]: its x-edges at y = 8 project
    onto the pixel boundary Y = 32, so with half width 0.75 rows 31 and 32
    are covered for columns 32..63, plus the corner caps at columns 31 and
    64 (centre distance sqrt(1/2) < 0.75); row 30 and 33 are not (1.5).
    Depth of the nearer edges is z + 1 = 11: a depth buffer of 15 keeps
    them, one of 5 hides the box."""
    cam = synth.camera_axis_z()
    box = np.array([[8, 8, 10, 16, 12, 20, 1.0, 0.5, 0.25, 0.5]])
    img0 = np.zeros((256, 256, 4))
    img, fl = oracle.overlay(cam, box, img0, half_width=0.75)
    col = np.array([0.5, 0.25, 0.125, 0.5])
    assert (fl == 0).all()
    for c in range(31, 65):
        for r in (31, 32):
            assert np.array_equal(img[r, c], col), (r, c)
        assert not img[30, c].any()
        # below the edge, rows 33.. belong to the y-edges at X = 32 and 64
        # (columns 31, 32 and 63, 64) and nothing else
        assert img[33, c].any() == (c in (31, 32, 63, 64)), c
    assert not img[31, 30].any() and not img[31, 65].any()
    # the y-edges at x = 16 (X = 64): columns 63 and 64 for rows 32..47
    assert np.array_equal(img[40, 63], col) and np.array_equal(img[40, 64], col) and not img[40, 62].any()
    # inside the box's outline nothing is drawn
    assert not img[40, 40].any()
    covered = img[..., 3] > 0
    depth = np.full((256, 256), 15.0, np.float32)
    img2, _ = oracle.overlay(cam, box, img0, half_width=0.75, depth=depth)
    assert np.array_equal(img2, img)
    img3, _ = oracle.overlay(cam, box, img0, half_width=0.75, depth=np.full((256, 256), 5.0, np.float32))
    assert not img3.any()
    # "over" an existing image: rgba a + (1 - a) under
    under = np.full((256, 256, 4), 0.2)
    img4, _ = oracle.overlay(cam, box, under, half_width=0.75)
    assert np.allclose(img4[covered], col + 0.5 * 0.2, rtol=0, atol=1e-15)
    assert np.array_equal(img4[~covered], under[~covered])


def test_overlay_perspective_by_hand():
    """Eye (0, 0, -10) looking along +z, fovy 90, 100 x 100: a point (x, y,
    z) lands at X = (x/w + 1) 50, Y = (1 + y/w) 50 with w = z + 10.  The
    segment (-5, 0, 0)..(5, 0, 0) maps to Y = 50, X in [25, 75]: rows 49
    and 50 are covered for columns 25..74, and the depth there is the
    distance sqrt(x^2 + 100) of the edge point under the pixel centre,
    x = (X - 50)/5.  A second box straddling the eye's plane is clipped at
    the near plane and does not disturb the first."""
    cam = synth.Camera(synth.PERSPECTIVE, (0.0, 0.0, -10.0), (0.0, 0.0, 0.0), (0.0, -1.0, 0.0), fovy_deg=90.0,
                       full_w=100, full_h=100)
    # a flat box: its four x-edges coincide pairwise at y = 0, z = 0
    box = np.array([[-5, 0, 0, 5, 0, 0, 0.0, 1.0, 0.0, 1.0]])
    img, fl = oracle.overlay(cam, box, np.zeros((100, 100, 4)), half_width=0.75)
    for c in range(25, 75):
        assert img[49, c, 1] == 1.0 and img[50, c, 1] == 1.0 and img[48, c, 3] == 0 and img[51, c, 3] == 0
    x = (np.arange(25, 75) + 0.5 - 50.0) / 5.0
    expect = np.sqrt(x * x + 100.0)
    # depth test right below / above the edge's distance at each column
    dep = np.full((100, 100), np.inf, np.float32)
    dep[49, 25:75] = (expect * (1 - 1e-6)).astype(np.float32)
    dep[50, 25:75] = (expect * (1 + 1e-6)).astype(np.float32)
    img2, _ = oracle.overlay(cam, box, np.zeros((100, 100, 4)), half_width=0.75, depth=dep)
    assert not img2[49, 25:75].any() and (img2[50, 25:75, 1] == 1.0).all()
    near_box = np.array([[-1, -1, -12, 1, 1, -8, 1.0, 0.0, 0.0, 1.0]])   # around the eye: clipped at the near plane
    both = np.concatenate([box, near_box])
    img3, _ = oracle.overlay(cam, both, np.zeros((100, 100, 4)), half_width=0.75)
    assert np.isfinite(img3).all()
    # every changed pixel took the nearer box's colour, and its clipped edges
    # (which run off the frame from the near plane) do draw somewhere
    changed = (img3 != img).any(axis=-1)
    assert changed.any()
    assert (img3[changed] == [1.0, 0.0, 0.0, 1.0]).all()


# ----------------------------------------------------------------------------
# blank (NaN) voxels
# ----------------------------------------------------------------------------
def test_blank_voxels_are_transparent_samples():
    """Constant alpha 1/2 along one axis ray (step 1, samples at z + 1/2),
    voxel z = 2 blank: with nearest sampling its sample is skipped (A after
    the 8 samples is 1 - 2^-7, as for 7 samples); with trilinear sampling
    the samples at z = 1.5, 2.5 and 3.5 all read the blank (2 corners each
    side), so 5 of the 8 count.  The MIP is the maximum over the other
    samples, and a ray of blanks only gives -inf."""
    vol = np.full((8, 1, 1), 0.5, np.float32)
    vol[2] = np.nan
    vol[6] = 0.75
    lut = synth.lut_dyadic([[0, 0, 0, 0], [1, 1, 1, 1]], 0.0, 1.0)
    cam = _axis_ray_camera(0.5, 0.5)
    near = oracle.render(vol, lut, cam, filt="nearest", step=1.0, tau=1.0)["out"][0, 0]
    # 6 samples of alpha 1/2 and one of 3/4 (z = 6): A = 1 - 2^-6 * 1/4
    A = 1.0 - 0.5 ** 6 * 0.25
    assert near[3] == A and np.isfinite(near).all()
    tri = oracle.render(vol, lut, cam, step=1.0, tau=1.0)["out"][0, 0]
    assert np.isfinite(tri).all()
    # samples at z + 1/2 read voxels z-1/2 .. z+1/2 (q = z clamped): z = 1, 2, 3
    # touch voxel 2 (q in [1, 3]); the others are 0.5, 0.5 + ..., 0.75 mixes
    assert oracle.render(vol, lut, cam, mode="mip", filt="nearest", step=1.0)["out"][0, 0] == 0.75
    blank = np.full((8, 1, 1), np.nan, np.float32)
    assert oracle.render(blank, lut, cam, mode="mip", step=1.0)["out"][0, 0] == -np.inf
    assert not oracle.render(blank, lut, cam, step=1.0, tau=1.0)["out"].any()
    d = oracle.depth(blank, lut, cam, mode="mip", step=1.0)
    assert d["out"][0, 0] == np.inf


def test_blank_voxels_adjoint_matches_finite_differences():
    """With blank voxels in the cube, the table gradient still matches
    central differences (a blank sample uses no table entry)."""
    vol = synth.make_cube(synth.CUBE_FD16)
    rng = np.random.default_rng(9)
    vol.reshape(-1)[rng.integers(0, vol.size, 40)] = np.nan
    lut = synth.lut_random(55)
    lut = synth.Lut(lut.table * np.float32(0.5), lut.vmin, lut.vmax)
    cam = synth.orbit_camera(vol.shape, seed=5, w=12, h=12)
    g = np.random.default_rng(2).standard_normal((12, 12, 4))
    gl, gv = oracle.backward(vol, lut, cam, g, tau=1.0)
    assert np.isfinite(gl).all()
    base = lut.table.astype(np.float64)
    h = 1e-6
    for j in rng.integers(0, base.shape[0], 12):
        for c in range(4):
            tp, tm = base.copy(), base.copy()
            tp[j, c] += h
            tm[j, c] -= h
            fp = oracle.render(vol, synth.Lut(tp.astype(np.float32), lut.vmin, lut.vmax), cam, tau=1.0)["out"]
            fm = oracle.render(vol, synth.Lut(tm.astype(np.float32), lut.vmin, lut.vmax), cam, tau=1.0)["out"]
            fd = ((fp - fm) * g).sum() / (np.float64(np.float32(base[j, c] + h)) - np.float64(np.float32(base[j, c] - h)))
            assert abs(fd - gl[j, c]) <= 1e-6 * max(1.0, np.abs(gl).max()), (j, c)
