"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np

# Tolerances (per element, absolute):
#  - composite RGBA, FP32 storage: 1e-5 (the stated bar);
#  - composite RGBA, FP16/BF16 storage against the oracle on the original
#    FP32 cube: 2e-3; against the oracle on the storage-rounded cube: 1e-5;
#  - trilinear MIP: two parts.  (1) The FP32 interpolation of 8 corners in
#    7 lerps, each a subtraction and an FMA, with weights converted from
#    32-bit fractions: one lerp level adds at most 5u M (u = 2^-24, M the
#    largest corner magnitude: u|b-a| + u|r| + u f|b-a|), three levels 15u M,
#    and the oracle's FP64 result is rounded once more (u |s|): 16u M.
#    (2) The sample positions: the GPU starts each ray at the fixed-point
#    position rounded to 2^-32 and adds a per-sample increment rounded to
#    2^-32 per axis, so sample k sits within (k + 1) 2^-33 voxel of the
#    exact point on every axis; the trilinear field's slope along an axis is
#    at most G, the largest difference of neighbouring voxels, so the value
#    moves by at most 3 G (n + 1) 2^-33 over a ray of n samples.
#    mip_tol(M) is part (1) alone, which small test cubes and short rays stay
#    within; mip_tol(M, G, n) adds part (2) per pixel (n the ray's sample
#    count) for the full-size cubes whose rays run to thousands of samples;
#  - nearest MIP: bit-exact.
TOL_COMPOSITE = 1e-5
TOL_LOWP = 2e-3
TOL_MIP_REL = 1e-6


def mip_tol(vmax, grad=None, n=None):
    """Absolute bound of |GPU - oracle| for a trilinear MIP value of a cube
    whose largest magnitude is vmax; with grad (largest neighbour
    difference) and n (samples of the pixel's ray, scalar or array) the
    position term is added (see above)."""
    t = 16.0 * 2.0 ** -24 * float(vmax)
    if grad is not None and n is not None:
        t = t + 3.0 * float(grad) * (np.asarray(n, dtype=np.float64) + 1.0) * 2.0 ** -33
    return t


def max_neighbour_diff(vol, planes=64):
    """Largest |V[i+1] - V[i]| along any axis, in slabs of z-planes."""
    g = 0.0
    nz = vol.shape[0]
    for z0 in range(0, nz, planes):
        z1 = min(nz, z0 + planes + 1)
        blk = np.asarray(vol[z0:z1], dtype=np.float32)
        g = max(g, float(np.abs(np.diff(blk, axis=0)).max()) if blk.shape[0] > 1 else 0.0,
                float(np.abs(np.diff(blk, axis=1)).max()), float(np.abs(np.diff(blk, axis=2)).max()))
    return g


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def accept(gpu, res, tol, rel=0.0):
    """Per element: |gpu - oracle| <= tol (+ rel |oracle|), or, on pixels the
    oracle flagged as having several correct results, gpu inside [lo, hi]
    widened by the same tolerance.  Returns (ok_mask, max_err_unflagged)."""
    out, lo, hi, fl = res["out"], res["lo"], res["hi"], res["flags"]
    g = np.asarray(gpu, dtype=np.float64)
    if g.ndim == out.ndim and g.ndim == fl.ndim + 1:
        flm = fl[..., None] != 0
    else:
        flm = fl != 0
    fin = np.isfinite(out)
    err = np.where(fin, np.abs(g - np.where(fin, out, 0.0)), np.where(g == out, 0.0, np.inf))
    t = tol + rel * np.where(fin, np.abs(out), 0.0)
    ok = err <= t
    ok |= flm & (g >= lo - t) & (g <= hi + t)
    ok |= (~fin) & (g == out)
    unfl = ~np.broadcast_to(flm, err.shape)
    mx = float(err[unfl].max()) if unfl.any() else 0.0
    return ok, mx


def assert_accept(gpu, res, tol, rel=0.0, what=""):
    ok, mx = accept(gpu, res, tol, rel)
    bad = np.argwhere(~ok)
    log(f"{what}: max err (unflagged) {mx:.3e}, flagged px {(res['flags'] != 0).sum()}, bad {len(bad)}")
    assert ok.all(), f"{what}: {len(bad)} elements out of tolerance, first {bad[:5].tolist()}"
    return mx


def assert_bitexact_mip(gpu, res, what=""):
    g = np.asarray(gpu, dtype=np.float64)
    out, lo, hi, fl = res["out"], res["lo"], res["hi"], res["flags"]
    clean = fl == 0
    assert np.array_equal(g[clean], out[clean]), f"{what}: nearest MIP not bit-exact"
    amb = ~clean
    assert ((g[amb] >= lo[amb]) & (g[amb] <= hi[amb])).all(), f"{what}: ambiguous pixels outside candidates"
    log(f"{what}: bit-exact on {clean.sum()} px, {amb.sum()} ambiguous px within candidates")
