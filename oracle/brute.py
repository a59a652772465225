"""Exact-rational brute-force renderer for tiny volumes.

TEST INFRASTRUCTURE.  An independent second implementation of the same
definition as vr_oracle.c, in exact rational arithmetic (fractions.Fraction),
enumerating every sample by hand: used to pin the FP64 oracle on 2^3 and 3^3
volumes.  It supports orthographic cameras whose basis (f, r, u) is given as
exact rational unit vectors, so that every ray origin, direction, clip
parameter, sample position, trilinear weight, table weight and composite step
is a rational number.

Rules (the same readings as the oracle): voxel centres at i + 1/2; origin
eye + sx r + sy u with sx = (2(c+1/2)/W - 1) half_w, sy = (1 - 2(row+1/2)/H) half_h;
direction f; slab clip to [0, N]^3 with t0 = max(tn, 0); samples at
t0 + (k + 1/2) step while < t1; trilinear with clamp-to-edge (q = p - 1/2
clamped to [0, N-1], i = min(floor q, N-2)); table with linear interpolation;
front-to-back composite with the stop after the sample once A >= tau.
"""
from __future__ import annotations

from fractions import Fraction as F
import math


def _floor(q: F) -> int:
    return math.floor(q)


def _slab(o, d, n):
    t_near, t_far = None, None
    for a in range(3):
        if d[a] == 0:
            if o[a] < 0 or o[a] > n[a]:
                return None
            continue
        ta = (F(0) - o[a]) / d[a]
        tb = (F(n[a]) - o[a]) / d[a]
        if ta > tb:
            ta, tb = tb, ta
        t_near = ta if t_near is None or ta > t_near else t_near
        t_far = tb if t_far is None or tb < t_far else t_far
    if t_near is None:
        return None
    if t_near > t_far:
        return None
    t0 = t_near if t_near > 0 else F(0)
    if t_far <= t0:
        return None
    return t0, t_far


def _tri(V, n, p):
    # V[k][j][i]; n = (nx, ny, nz)
    idx, fr = [], []
    for a in range(3):
        if n[a] == 1:
            idx.append(0)
            fr.append(F(0))
            continue
        q = p[a] - F(1, 2)
        q = min(max(q, F(0)), F(n[a] - 1))
        i = min(_floor(q), n[a] - 2)
        idx.append(i)
        fr.append(q - i)
    val = F(0)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (fr[0] if dx else 1 - fr[0]) * (fr[1] if dy else 1 - fr[1]) * (fr[2] if dz else 1 - fr[2])
                if w == 0:
                    continue
                i = min(idx[0] + dx, n[0] - 1)
                j = min(idx[1] + dy, n[1] - 1)
                k = min(idx[2] + dz, n[2] - 1)
                val += w * V[k][j][i]
    return val


def _near(V, n, p):
    c = [min(max(_floor(p[a]), 0), n[a] - 1) for a in range(3)]
    return V[c[2]][c[1]][c[0]]


def _lut(L, vmin, vmax, s):
    nl = len(L)
    u = (s - vmin) / (vmax - vmin)
    u = min(max(u, F(0)), F(1))
    x = u * (nl - 1)
    j = min(_floor(x), nl - 2)
    w = x - j
    return [(1 - w) * L[j][c] + w * L[j + 1][c] for c in range(4)]


def render_pixel(V, L, vmin, vmax, eye, f, r, u, half_w, half_h, W, H, col, row,
                 step=F(1, 2), tau=F(99, 100), mode="composite", filt="trilinear",
                 count=None, cell_offset=None):
    """Exact render of one full-frame pixel (all arguments Fractions / ints).

    The two keyword arguments flip one discontinuous decision by hand, to
    spell out a candidate outcome: `count` takes exactly that many samples
    t0 + (k + 1/2) step, k < count, in place of the exit test t_k < t1;
    `cell_offset` (three exact offsets) moves the position at which the
    nearest voxel is looked up, e.g. (-1, 0, 0) to take the cell on the
    other side of a face the sample lies on."""
    nz, ny, nx = len(V), len(V[0]), len(V[0][0])
    n = (nx, ny, nz)
    sx = (F(2) * (col + F(1, 2)) / W - 1) * half_w
    sy = (1 - F(2) * (row + F(1, 2)) / H) * half_h
    o = [eye[a] + sx * r[a] + sy * u[a] for a in range(3)]
    d = list(f)
    cl = _slab(o, d, n)
    if mode == "mip":
        if cl is None:
            return None
    elif cl is None:
        return [F(0)] * 4
    t0, t1 = cl
    k = 0
    C = [F(0)] * 3
    A = F(0)
    m = None
    while (t0 + (k + F(1, 2)) * step < t1) if count is None else k < count:
        t = t0 + (k + F(1, 2)) * step
        p = [o[a] + t * d[a] for a in range(3)]
        if filt == "nearest":
            s = _near(V, n, p if cell_offset is None else [p[a] + cell_offset[a] for a in range(3)])
        else:
            s = _tri(V, n, p)
        if mode == "mip":
            m = s if m is None or s > m else m
        else:
            rgba = _lut(L, vmin, vmax, s)
            a = rgba[3]
            for c in range(3):
                C[c] += (1 - A) * a * rgba[c]
            A += (1 - A) * a
            if tau < 1 and A >= tau:
                break
        k += 1
    if mode == "mip":
        return m
    return C + [A]


def to_frac_volume(vol):
    nz, ny, nx = vol.shape
    return [[[F(float(vol[k, j, i])) for i in range(nx)] for j in range(ny)] for k in range(nz)]


def to_frac_lut(table):
    return [[F(float(table[j, c])) for c in range(4)] for j in range(table.shape[0])]
