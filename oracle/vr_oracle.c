/*
 * vr_oracle.c -- plain, slow FP64 reference ray caster.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU renderer, and the GPU renderer never
 * calls it.
 *
 * What it computes: the ray-casting volume rendering the paper's framework
 * performs on spectral cubes (abstract and section 1: interactive rendering
 * of the cube by GPU ray casting; section 3: a static render of the current
 * view at an output size the user picks, and a 5x5 wall of 1920x1080
 * panels).  The paper gives no formulas, so every rule
 * below is a stated reading, chosen so that a test can pin it:
 *
 *  World      voxel units; the cube occupies [0,nx]x[0,ny]x[0,nz]; voxel
 *             (i,j,k) has its centre at (i+1/2, j+1/2, k+1/2) and is stored
 *             at V[(k*ny + j)*nx + i].
 *  Camera     f = unit(target - eye), r = unit(f x up), u = r x f.  Full-frame
 *             pixel (c, row) has sx = (2(c+1/2)/W - 1) a, sy = (1 - 2(row+1/2)/H) b.
 *             Perspective: a = tan(fovy/2) W/H, b = tan(fovy/2), origin eye,
 *             direction unit(f + sx r + sy u).  Orthographic: a = half_w,
 *             b = half_h, origin eye + sx r + sy u, direction f.
 *  Clip       slab test against the box gives [tn, tf]; t0 = max(tn, 0),
 *             t1 = tf; a ray misses when t1 <= t0.  A zero direction
 *             component keeps the ray iff the origin lies in that slab.
 *  Samples    t_k = t0 + (k + 1/2) step for k = 0, 1, ... while t_k < t1.
 *  Trilinear  q = p - 1/2 per axis; corners floor(q) and floor(q) + 1, each
 *             clamped to [0, N-1] (the cube extended by repeating its
 *             faces), weight f = q - floor(q) on the second; interpolate
 *             along x, then y, then z.  Inside the cube this is plain
 *             trilinear interpolation, and beyond its outer voxel centres
 *             the value is the edge voxel's (clamp-to-edge).
 *  Nearest    i = clamp(floor p, 0, N-1).
 *  Table      u = clamp((s - vmin)/(vmax - vmin), 0, 1); x = u (n-1);
 *             j = min(floor x, n-2); w = x - j; rgba = (1-w) L[j] + w L[j+1];
 *             entries are straight (not premultiplied) RGBA.
 *  Composite  C = 0, A = 0; per sample: C += (1-A) a c; A += (1-A) a; stop
 *             after the sample once A >= tau (tau >= 1: never).  Output is
 *             premultiplied (C, A) with no background.
 *  MIP        m = max_k s_k; -inf when the ray takes no sample.
 *  Blanks     a NaN voxel (a blank, as FITS cubes mark them) makes every
 *             sample whose interpolation footprint holds it NaN; such a
 *             sample is transparent (rgba 0) in the composite and takes no
 *             part in the MIP maximum, but it is still a sample of the ray.
 *  Bricks     edge-B bricks partition space into half-open boxes; a sample
 *             belongs to the brick holding its position (the last brick on
 *             the cube's far faces).  Each brick composites its own samples
 *             with its own early stop; partials are combined front to back
 *             with the "over" operator in increasing key order: the
 *             Manhattan distance of the brick cell from the eye's cell for
 *             a perspective camera, sum_a sign(d_a) i_a for an orthographic
 *             one (ties by brick id).
 *
 * Candidate outcomes (where several results are correct).  The stop decision
 * A >= tau, the last-sample test t_k < t1 and the nearest cell floor(p) are
 * discontinuous.  When the FP64 quantity lies within a window of its
 * threshold the oracle widens its answer to the interval [lo, hi] of all
 * outcomes reachable by flipping those decisions, and flags the pixel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t kind; /* 0 orthographic, 1 perspective */
    double eye[3], target[3], up[3];
    double fovy_deg, half_w, half_h;
    int32_t full_w, full_h;
    int32_t tile_x0, tile_y0, tile_w, tile_h;
} orc_camera;

typedef struct {
    int32_t mode;    /* 0 composite, 1 MIP */
    int32_t filter;  /* 0 trilinear, 1 nearest */
    double step;
    double tau;      /* early-stop opacity; >= 1 disables */
    double eps_stop; /* window around tau */
    double eps_t;    /* window around t1 for the last sample (relative to max(1,|t1|)) */
    double eps_pos;  /* window around integer coordinates for nearest cells */
} orc_params;

typedef struct {
    const float *vol;
    int64_t nx, ny, nz;
    const float *lut;
    int32_t nlut;
    double vmin, vmax;
} orc_scene;

enum { FLAG_STOP = 1, FLAG_COUNT = 2, FLAG_CELL = 4, FLAG_BRICK = 8 };

/* ------------------------------------------------------------------ */
/* small vector helpers                                               */
/* ------------------------------------------------------------------ */
static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static void unit3(double v[3]) {
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

/* Camera basis f, r, u. */
void orc_basis(const orc_camera *c, double f[3], double r[3], double u[3]) {
    for (int a = 0; a < 3; ++a) f[a] = c->target[a] - c->eye[a];
    unit3(f);
    cross3(f, c->up, r);
    unit3(r);
    cross3(r, f, u);
}

/* Ray through full-frame pixel (col, row): origin o, unit direction d. */
void orc_ray(const orc_camera *c, int64_t col, int64_t row, double o[3], double d[3]) {
    double f[3], r[3], u[3];
    orc_basis(c, f, r, u);
    double W = c->full_w, H = c->full_h, a, b;
    if (c->kind == 1) {
        double th = tan(c->fovy_deg * M_PI / 360.0);
        a = th * W / H;
        b = th;
    } else {
        a = c->half_w;
        b = c->half_h;
    }
    double sx = (2.0 * (col + 0.5) / W - 1.0) * a;
    double sy = (1.0 - 2.0 * (row + 0.5) / H) * b;
    if (c->kind == 1) {
        for (int k = 0; k < 3; ++k) { o[k] = c->eye[k]; d[k] = f[k] + sx * r[k] + sy * u[k]; }
        unit3(d);
    } else {
        for (int k = 0; k < 3; ++k) { o[k] = c->eye[k] + sx * r[k] + sy * u[k]; d[k] = f[k]; }
    }
}

/* Slab test against [lo, hi]; returns 1 and [tn, tf] when the line meets the box. */
int orc_slab(const double o[3], const double d[3], const double lo[3], const double hi[3],
             double *tn, double *tf) {
    double a0 = -INFINITY, a1 = INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < lo[k] || o[k] > hi[k]) return 0;
            continue;
        }
        double ta = (lo[k] - o[k]) / d[k];
        double tb = (hi[k] - o[k]) / d[k];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > a0) a0 = ta;
        if (tb < a1) a1 = tb;
    }
    *tn = a0;
    *tf = a1;
    return a0 <= a1;
}

/* Ray interval [t0, t1) inside the cube; 0 when the ray misses. */
static int clip_cube(const orc_scene *s, const double o[3], const double d[3], double *t0, double *t1) {
    double lo[3] = {0, 0, 0}, hi[3] = {(double)s->nx, (double)s->ny, (double)s->nz};
    double tn, tf;
    if (!orc_slab(o, d, lo, hi, &tn, &tf)) return 0;
    *t0 = tn > 0.0 ? tn : 0.0;
    *t1 = tf;
    return *t1 > *t0;
}

/* ------------------------------------------------------------------ */
/* sampling                                                           */
/* ------------------------------------------------------------------ */
static double voxel(const orc_scene *s, int64_t i, int64_t j, int64_t k) {
    return (double)s->vol[(k * s->ny + j) * s->nx + i];
}

/* Clamp-to-edge, read as the cube extended by repeating its faces: the two
 * corners of axis position p are the voxels floor(q) and floor(q) + 1 of
 * q = p - 1/2, each index clamped to [0, n-1], with weight f = q - floor(q)
 * on the second.  Inside [0, n-1] this is plain linear interpolation; beyond
 * it both corners are the edge voxel, so the value is the edge voxel's.  The
 * two corners are the sample's footprint along the axis (what makes it blank
 * when one holds a NaN). */
static void tri_axis(double p, int64_t n, int64_t *i0, int64_t *i1, double *f) {
    double q = p - 0.5;
    double fl = floor(q);
    int64_t a = (int64_t)fl, b = a + 1;
    *i0 = a < 0 ? 0 : (a > n - 1 ? n - 1 : a);
    *i1 = b < 0 ? 0 : (b > n - 1 ? n - 1 : b);
    *f = q - fl;
}

/* Trilinear value; corners/weights returned for the adjoint when wanted. */
double orc_trilinear(const orc_scene *s, const double p[3], int64_t idx[8], double wt[8]) {
    int64_t i, j, k, i1, j1, k1;
    double fx, fy, fz;
    tri_axis(p[0], s->nx, &i, &i1, &fx);
    tri_axis(p[1], s->ny, &j, &j1, &fy);
    tri_axis(p[2], s->nz, &k, &k1, &fz);
    double c000 = voxel(s, i, j, k), c100 = voxel(s, i1, j, k);
    double c010 = voxel(s, i, j1, k), c110 = voxel(s, i1, j1, k);
    double c001 = voxel(s, i, j, k1), c101 = voxel(s, i1, j, k1);
    double c011 = voxel(s, i, j1, k1), c111 = voxel(s, i1, j1, k1);
    double x00 = c000 + fx * (c100 - c000), x10 = c010 + fx * (c110 - c010);
    double x01 = c001 + fx * (c101 - c001), x11 = c011 + fx * (c111 - c011);
    double y0 = x00 + fy * (x10 - x00), y1 = x01 + fy * (x11 - x01);
    double v = y0 + fz * (y1 - y0);
    if (idx) {
        int64_t I[2] = {i, i1}, J[2] = {j, j1}, K[2] = {k, k1};
        double WX[2] = {1 - fx, fx}, WY[2] = {1 - fy, fy}, WZ[2] = {1 - fz, fz};
        int c = 0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx, ++c) {
                    idx[c] = (K[dz] * s->ny + J[dy]) * s->nx + I[dx];
                    wt[c] = WX[dx] * WY[dy] * WZ[dz];
                }
    }
    return v;
}

static int64_t near_axis(double p, int64_t n) {
    int64_t i = (int64_t)floor(p);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    return i;
}

/* Nearest value, plus the min/max over neighbouring cells whenever a
 * coordinate lies within eps of a cell face (the candidates). */
static double nearest(const orc_scene *s, const double p[3], double eps, double *lo, double *hi, int *amb) {
    int64_t c[3], alt[3];
    int64_t n[3] = {s->nx, s->ny, s->nz};
    int any = 0;
    for (int a = 0; a < 3; ++a) {
        c[a] = near_axis(p[a], n[a]);
        alt[a] = c[a];
        double fr = p[a] - floor(p[a]);
        if (fr < eps) alt[a] = near_axis(p[a] - 1.0, n[a]);
        else if (fr > 1.0 - eps) alt[a] = near_axis(p[a] + 1.0, n[a]);
        if (alt[a] != c[a]) any = 1;
    }
    double v = voxel(s, c[0], c[1], c[2]);
    double mn = v, mx = v;
    if (any) {
        /* over the candidate cells; a blank (NaN) candidate may drop the
         * sample altogether, so the low end is then -inf */
        int blank = 0;
        mn = INFINITY;
        mx = -INFINITY;
        for (int m = 0; m < 8; ++m) {
            int64_t q0 = (m & 1) ? alt[0] : c[0], q1 = (m & 2) ? alt[1] : c[1], q2 = (m & 4) ? alt[2] : c[2];
            double w = voxel(s, q0, q1, q2);
            if (isnan(w)) { blank = 1; continue; }
            if (w < mn) mn = w;
            if (w > mx) mx = w;
        }
        if (blank) mn = -INFINITY;
        if (mx == -INFINITY) mx = v;        /* every candidate blank */
    }
    *lo = mn; *hi = mx; *amb = any;
    return v;
}

/* Transfer function; returns the table slope d rgba / d s in dv (0 when clamped).
 * A NaN value (a blank voxel in the sample's footprint) maps to transparent
 * black: rgba = 0, slope 0, and *jj = -1 marks that no entry was used. */
void orc_lut(const float *L, int32_t n, double vmin, double vmax, double s, double rgba[4],
             int32_t *jj, double *ww, double dv[4]) {
    if (isnan(s)) {
        for (int c = 0; c < 4; ++c) {
            rgba[c] = 0.0;
            if (dv) dv[c] = 0.0;
        }
        if (jj) *jj = -1;
        if (ww) *ww = 0.0;
        return;
    }
    double u = (s - vmin) / (vmax - vmin);
    int clamped = 0;
    if (u <= 0.0) { u = 0.0; clamped = 1; }
    if (u >= 1.0) { u = 1.0; clamped = 1; }
    double x = u * (double)(n - 1);
    int32_t j = (int32_t)floor(x);
    if (j > n - 2) j = n - 2;
    double w = x - (double)j;
    for (int c = 0; c < 4; ++c) {
        double a = L[4 * j + c], b = L[4 * (j + 1) + c];
        rgba[c] = (1.0 - w) * a + w * b;
        if (dv) dv[c] = clamped ? 0.0 : (b - a) * (double)(n - 1) / (vmax - vmin);
    }
    if (jj) *jj = j;
    if (ww) *ww = w;
}

/* ------------------------------------------------------------------ */
/* one ray                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    double o[3], d[3];
    double t0, t1;
    int64_t n;      /* samples by definition */
    int64_t n_lo, n_hi; /* candidate counts for the last-sample test */
    int hit;
} ray_t;

static void ray_prepare(const orc_scene *s, const orc_camera *cam, const orc_params *p,
                        int64_t col, int64_t row, ray_t *r) {
    orc_ray(cam, col, row, r->o, r->d);
    r->hit = clip_cube(s, r->o, r->d, &r->t0, &r->t1);
    r->n = r->n_lo = r->n_hi = 0;
    if (!r->hit) return;
    int64_t k = 0;
    while (r->t0 + (k + 0.5) * p->step < r->t1) ++k;
    r->n = r->n_lo = r->n_hi = k;
    double win = p->eps_t * (fabs(r->t1) > 1.0 ? fabs(r->t1) : 1.0);
    if (k > 0 && r->t1 - (r->t0 + (k - 0.5) * p->step) < win) r->n_lo = k - 1;
    if ((r->t0 + (k + 0.5) * p->step) - r->t1 < win) r->n_hi = k + 1;
}

static void sample_pos(const ray_t *r, double step, int64_t k, double pos[3]) {
    double t = r->t0 + (k + 0.5) * step;
    for (int a = 0; a < 3; ++a) pos[a] = r->o[a] + t * r->d[a];
}

/* Composite or MIP of one ray.  out/lo/hi have 4 (composite) or 1 (MIP)
 * entries; returns flags; *taken = samples processed up to the stop. */
static int render_ray(const orc_scene *s, const orc_params *p, const ray_t *r,
                      double *out, double *lo, double *hi, int64_t *taken) {
    int flags = 0;
    if (r->n_lo != r->n || r->n_hi != r->n) flags |= FLAG_COUNT;
    if (p->mode == 1) {
        double m = -INFINITY, mlo = -INFINITY, mhi = -INFINITY;
        for (int64_t k = 0; k < r->n_hi; ++k) {
            double pos[3], v, vl, vh;
            sample_pos(r, p->step, k, pos);
            if (p->filter == 1) {
                int amb;
                v = nearest(s, pos, p->eps_pos, &vl, &vh, &amb);
                if (amb) flags |= FLAG_CELL;
            } else {
                v = orc_trilinear(s, pos, NULL, NULL);
                vl = vh = v;
            }
            if (k < r->n && v > m) m = v;
            if (k < r->n_lo && vl > mlo) mlo = vl;
            if (vh > mhi) mhi = vh;
        }
        out[0] = m; lo[0] = mlo; hi[0] = mhi;
        *taken = r->n;
        return flags;
    }
    double C[3] = {0, 0, 0}, A = 0.0;
    int have_main = 0, have_lo = 0, have_hi = 0;
    double tau = p->tau;
    for (int c = 0; c < 4; ++c) out[c] = lo[c] = hi[c] = 0.0;
    *taken = 0;
    int ert = tau < 1.0;
    for (int64_t k = 0; k < r->n_hi; ++k) {
        double pos[3], v, rgba[4];
        sample_pos(r, p->step, k, pos);
        if (p->filter == 1) {
            double vl, vh;
            int amb;
            v = nearest(s, pos, p->eps_pos, &vl, &vh, &amb);
            if (amb) flags |= FLAG_CELL;
        } else {
            v = orc_trilinear(s, pos, NULL, NULL);
        }
        orc_lut(s->lut, s->nlut, s->vmin, s->vmax, v, rgba, NULL, NULL, NULL);
        double a = rgba[3];
        for (int c = 0; c < 3; ++c) C[c] += (1.0 - A) * a * rgba[c];
        A += (1.0 - A) * a;
        int last_main = (k == r->n - 1), last_lo = (k == r->n_lo - 1), last_hi = (k == r->n_hi - 1);
        if (!have_main && k < r->n && ((ert && A >= tau) || last_main)) {
            have_main = 1;
            out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = A;
            *taken = k + 1;
        }
        if (!have_lo && k < r->n_lo && ((ert && A >= tau - p->eps_stop) || last_lo)) {
            have_lo = 1;
            lo[0] = C[0]; lo[1] = C[1]; lo[2] = C[2]; lo[3] = A;
        }
        if (!have_hi && ((ert && A >= tau + p->eps_stop) || last_hi)) {
            have_hi = 1;
            hi[0] = C[0]; hi[1] = C[1]; hi[2] = C[2]; hi[3] = A;
        }
        if (ert && fabs(A - tau) < p->eps_stop) flags |= FLAG_STOP;
        if (have_hi) break;
    }
    return flags;
}

static int nthreads_of(int nt) {
#ifdef _OPENMP
    return nt > 0 ? nt : omp_get_max_threads();
#else
    (void)nt;
    return 1;
#endif
}

/* Render a list of tile-local pixels (pix = NULL: the whole tile, row-major).
 * chans = 4 (composite) or 1 (MIP).  lo, hi, flags, taken may be NULL. */
int orc_render(const float *vol, int64_t nx, int64_t ny, int64_t nz,
               const float *lut, int32_t nlut, double vmin, double vmax,
               const orc_camera *cam, const orc_params *p,
               const int32_t *pix, int64_t npix,
               double *out, double *lo, double *hi, int32_t *flags, int64_t *taken, int nthreads) {
    orc_scene s = {vol, nx, ny, nz, lut, nlut, vmin, vmax};
    int chans = p->mode == 1 ? 1 : 4;
    if (!pix) npix = (int64_t)cam->tile_w * cam->tile_h;
    int nt = nthreads_of(nthreads);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t x, y;
        if (pix) { x = pix[2 * q]; y = pix[2 * q + 1]; }
        else { x = q % cam->tile_w; y = q / cam->tile_w; }
        ray_t r;
        ray_prepare(&s, cam, p, cam->tile_x0 + x, cam->tile_y0 + y, &r);
        double o4[4], l4[4], h4[4];
        int64_t tk = 0;
        int fl = 0;
        if (!r.hit) {
            for (int c = 0; c < 4; ++c) o4[c] = l4[c] = h4[c] = (p->mode == 1 ? -INFINITY : 0.0);
        } else {
            fl = render_ray(&s, p, &r, o4, l4, h4, &tk);
        }
        for (int c = 0; c < chans; ++c) {
            out[q * chans + c] = o4[c];
            if (lo) lo[q * chans + c] = l4[c];
            if (hi) hi[q * chans + c] = h4[c];
        }
        if (flags) flags[q] = fl;
        if (taken) taken[q] = tk;
    }
    return 0;
}

/* Per-pixel ray interval (for tests of the clip): t0, t1, n, hit. */
int orc_ray_interval(const float *vol, int64_t nx, int64_t ny, int64_t nz,
                     const orc_camera *cam, const orc_params *p, int64_t col, int64_t row,
                     double *o, double *d, double *t0, double *t1, int64_t *n) {
    orc_scene s = {vol, nx, ny, nz, NULL, 0, 0, 1};
    ray_t r;
    ray_prepare(&s, cam, p, col, row, &r);
    for (int a = 0; a < 3; ++a) { o[a] = r.o[a]; d[a] = r.d[a]; }
    *t0 = r.t0; *t1 = r.t1; *n = r.n;
    return r.hit;
}

/* ------------------------------------------------------------------ */
/* depth (section 2: what a catalogue overlay is tested against)      */
/* ------------------------------------------------------------------ */
/* Depth of one ray, as the ray parameter t = t0 + (k + 1/2) step of a
 * sample k, or +inf:
 *  composite: the first sample (among those taken, up to the stop) after
 *             which the accumulated opacity A reaches `level`;
 *  MIP:       the first sample whose value equals the ray's maximum.
 * `count` samples are taken (the ray's n, or a flipped candidate), the stop
 * test uses `tau`, the crossing test `level`. */
static double depth_ray(const orc_scene *s, const orc_params *p, const ray_t *r, int64_t count, double tau,
                        double level) {
    int ert = tau < 1.0;
    if (p->mode == 1) {
        double m = -INFINITY, best = INFINITY;
        for (int64_t k = 0; k < count; ++k) {
            double pos[3], v;
            sample_pos(r, p->step, k, pos);
            if (p->filter == 1) {
                double vl, vh;
                int amb;
                v = nearest(s, pos, p->eps_pos, &vl, &vh, &amb);
            } else {
                v = orc_trilinear(s, pos, NULL, NULL);
            }
            if (v > m) { m = v; best = r->t0 + (k + 0.5) * p->step; }
        }
        return best;
    }
    double A = 0.0;
    for (int64_t k = 0; k < count; ++k) {
        double pos[3], v, rgba[4];
        sample_pos(r, p->step, k, pos);
        if (p->filter == 1) {
            double vl, vh;
            int amb;
            v = nearest(s, pos, p->eps_pos, &vl, &vh, &amb);
        } else {
            v = orc_trilinear(s, pos, NULL, NULL);
        }
        orc_lut(s->lut, s->nlut, s->vmin, s->vmax, v, rgba, NULL, NULL, NULL);
        A += (1.0 - A) * rgba[3];
        if (A >= level) return r->t0 + (k + 0.5) * p->step;
        if (ert && A >= tau) break;
    }
    return INFINITY;
}

/* Per-pixel depth (see depth_ray).  lo / hi receive the smallest and largest
 * depth over the flipped decisions: the sample count (n_lo, n, n_hi), the
 * stop and crossing tests moved by -/+ eps_stop (composite), and, for MIP,
 * every sample whose value could be the maximum once the values move by
 * eps_val (trilinear: the FP32 interpolation's rounding) or the nearest
 * cell flips.  flags gets FLAG_STOP when lo < hi for a composite, FLAG_CELL
 * for a MIP tie, FLAG_COUNT as in orc_render. */
int orc_depth(const float *vol, int64_t nx, int64_t ny, int64_t nz,
              const float *lut, int32_t nlut, double vmin, double vmax,
              const orc_camera *cam, const orc_params *p, double level, double eps_val,
              const int32_t *pix, int64_t npix, double *out, double *lo, double *hi, int32_t *flags,
              int nthreads) {
    orc_scene s = {vol, nx, ny, nz, lut, nlut, vmin, vmax};
    if (!pix) npix = (int64_t)cam->tile_w * cam->tile_h;
    int nt = nthreads_of(nthreads);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t x, y;
        if (pix) { x = pix[2 * q]; y = pix[2 * q + 1]; }
        else { x = q % cam->tile_w; y = q / cam->tile_w; }
        ray_t r;
        ray_prepare(&s, cam, p, cam->tile_x0 + x, cam->tile_y0 + y, &r);
        double d = INFINITY, dl = INFINITY, dh = INFINITY;
        int fl = 0;
        if (r.hit) {
            if (r.n_lo != r.n || r.n_hi != r.n) fl |= FLAG_COUNT;
            d = depth_ray(&s, p, &r, r.n, p->tau, level);
            dl = dh = d;
            int64_t counts[3] = {r.n_lo, r.n, r.n_hi};
            if (p->mode != 1) {
                double taus[3] = {p->tau, p->tau - p->eps_stop, p->tau + p->eps_stop};
                double levels[3] = {level, level - p->eps_stop, level + p->eps_stop};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        for (int c = 0; c < 3; ++c) {
                            double e = depth_ray(&s, p, &r, counts[a], taus[b], levels[c]);
                            if (e < dl) dl = e;
                            if (e > dh) dh = e;
                        }
                if (dl < dh) fl |= FLAG_STOP;
            } else {
                /* sample k can be the first maximum under some choice of
                 * the values within their windows [vl, vh] iff its highest
                 * value beats the lowest of every earlier sample strictly
                 * and ties or beats the lowest of every later one (samples
                 * past n_lo may be absent, so only those before n_lo must
                 * be beaten) */
                int64_t m = r.n_hi;
                double *vl = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
                double *vh = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
                for (int64_t k = 0; k < m; ++k) {
                    double pos[3], v;
                    int amb = 0;
                    sample_pos(&r, p->step, k, pos);
                    if (p->filter == 1) v = nearest(&s, pos, p->eps_pos, &vl[k], &vh[k], &amb);
                    else { v = orc_trilinear(&s, pos, NULL, NULL); vl[k] = v - eps_val; vh[k] = v + eps_val; }
                    (void)v;
                }
                double pre = -INFINITY;
                for (int64_t k = 0; k < m; ++k) {
                    double suf = -INFINITY;
                    for (int64_t j = k + 1; j < r.n_lo; ++j)
                        if (vl[j] > suf) suf = vl[j];
                    if (vh[k] > pre && vh[k] >= suf) {
                        double t = r.t0 + (k + 0.5) * p->step;
                        if (t < dl) dl = t;
                        if (t > dh || dh == INFINITY) dh = t;
                    }
                    if (k < r.n_lo && vl[k] > pre) pre = vl[k];
                }
                free(vl);
                free(vh);
                if (d < dl) dl = d;
                if (d != INFINITY && d > dh) dh = d;
                if (dl < dh) fl |= FLAG_CELL;
            }
        }
        out[q] = d;
        if (lo) lo[q] = dl;
        if (hi) hi[q] = dh;
        if (flags) flags[q] = fl;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* catalogue overlay (section 2: source bounding cubes drawn as       */
/* wireframe boxes over the render)                                   */
/* ------------------------------------------------------------------ */
/* Position of world point P in full-frame pixel coordinates (pixel (c, row)
 * has its centre at (c + 1/2, row + 1/2)) and its view depth w (distance
 * along f); perspective points need w > 0. */
static void project_px(const orc_camera *c, const double f[3], const double r[3], const double u[3],
                       const double P[3], double *X, double *Y, double *w) {
    double d[3] = {P[0] - c->eye[0], P[1] - c->eye[1], P[2] - c->eye[2]};
    double wf = d[0] * f[0] + d[1] * f[1] + d[2] * f[2];
    double xr = d[0] * r[0] + d[1] * r[1] + d[2] * r[2];
    double yu = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    double a, b, sx, sy;
    if (c->kind == 1) {
        double th = tan(c->fovy_deg * M_PI / 360.0);
        a = th * c->full_w / c->full_h;
        b = th;
        sx = xr / wf;
        sy = yu / wf;
    } else {
        a = c->half_w;
        b = c->half_h;
        sx = xr;
        sy = yu;
    }
    *X = (sx / a + 1.0) * 0.5 * c->full_w;
    *Y = (1.0 - sy / b) * 0.5 * c->full_h;
    *w = wf;
}

/* Overlay n wireframe boxes (box i: lo[3], hi[3] in voxel coordinates, then
 * straight RGBA; 10 doubles) on a premultiplied RGBA tile (image, modified
 * in place).  For every pixel and every edge of every box: the edge (the
 * part in front of the near plane w >= near for a perspective camera) is
 * projected to full-frame pixel coordinates; the pixel is covered when the
 * distance from its centre to the projected segment is at most half_width;
 * the edge's depth there is the ray distance of the 3D point that projects
 * to the segment's point nearest the centre (|P - eye| for a perspective
 * camera, (P - eye).f for an orthographic one).  The edge is visible when
 * that depth is at most depth[pixel] (depth NULL: always).  The pixel takes
 * the nearest visible covering edge (ties: lower box, then lower edge
 * index) and becomes rgba_premultiplied + (1 - a) image.  flags: 1 when a
 * coverage, depth-test or nearest-edge decision lies within eps (relative
 * to max(1, |quantity|)) of its threshold. */
int orc_overlay(const orc_camera *cam, const double *boxes, int64_t n, double half_width, double near,
                const float *depth, double eps, double *image, int32_t *flags, int nthreads) {
    double f[3], r[3], u[3];
    orc_basis(cam, f, r, u);
    int64_t npix = (int64_t)cam->tile_w * cam->tile_h;
    int nt = nthreads_of(nthreads);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
    for (int64_t q = 0; q < npix; ++q) {
        double qx = cam->tile_x0 + (double)(q % cam->tile_w) + 0.5;
        double qy = cam->tile_y0 + (double)(q / cam->tile_w) + 0.5;
        double zb = depth ? (double)depth[q] : INFINITY;
        int64_t best_box = -1;
        double best_t = INFINITY, second_t = INFINITY;   /* nearest two boxes */
        int fl = 0;
        for (int64_t i = 0; i < n; ++i) {
            const double *B = boxes + 10 * i;
            double box_t = INFINITY;                      /* nearest visible edge of box i */
            for (int e = 0; e < 12; ++e) {
                /* edge e runs along axis e / 4; the other two axes take
                 * lo or hi by the two bits of e % 4 */
                int ax = e / 4, o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
                double P0[3], P1[3];
                P0[ax] = B[ax]; P1[ax] = B[3 + ax];
                P0[o1] = P1[o1] = (e & 1) ? B[3 + o1] : B[o1];
                P0[o2] = P1[o2] = (e & 2) ? B[3 + o2] : B[o2];
                double X0, Y0, w0, X1, Y1, w1;
                if (cam->kind == 1) {
                    double wa = (P0[0] - cam->eye[0]) * f[0] + (P0[1] - cam->eye[1]) * f[1] +
                                (P0[2] - cam->eye[2]) * f[2];
                    double wb = (P1[0] - cam->eye[0]) * f[0] + (P1[1] - cam->eye[1]) * f[1] +
                                (P1[2] - cam->eye[2]) * f[2];
                    if (wa < near && wb < near) continue;
                    if (wa < near || wb < near) {
                        /* clip the part behind the near plane */
                        double t = (near - wa) / (wb - wa);
                        double C[3];
                        for (int k = 0; k < 3; ++k) C[k] = P0[k] + t * (P1[k] - P0[k]);
                        if (wa < near) memcpy(P0, C, sizeof C); else memcpy(P1, C, sizeof C);
                    }
                }
                project_px(cam, f, r, u, P0, &X0, &Y0, &w0);
                project_px(cam, f, r, u, P1, &X1, &Y1, &w1);
                double dx = X1 - X0, dy = Y1 - Y0, L2 = dx * dx + dy * dy;
                double sp = L2 > 0.0 ? ((qx - X0) * dx + (qy - Y0) * dy) / L2 : 0.0;
                if (sp < 0.0) sp = 0.0;
                if (sp > 1.0) sp = 1.0;
                double ex = X0 + sp * dx - qx, ey = Y0 + sp * dy - qy;
                double dist = sqrt(ex * ex + ey * ey);
                if (fabs(dist - half_width) < eps * (half_width > 1.0 ? half_width : 1.0)) fl |= 1;
                if (dist > half_width) continue;
                double uu = cam->kind == 1 ? sp * w0 / (sp * w0 + (1.0 - sp) * w1) : sp;
                double P[3], t;
                for (int k = 0; k < 3; ++k) P[k] = P0[k] + uu * (P1[k] - P0[k]);
                if (cam->kind == 1) {
                    double d0 = P[0] - cam->eye[0], d1 = P[1] - cam->eye[1], d2 = P[2] - cam->eye[2];
                    t = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                } else {
                    t = (P[0] - cam->eye[0]) * f[0] + (P[1] - cam->eye[1]) * f[1] + (P[2] - cam->eye[2]) * f[2];
                }
                double sc = fabs(t) > 1.0 ? fabs(t) : 1.0;
                if (isfinite(zb) && fabs(t - zb) < eps * sc) fl |= 1;
                if (!(t <= zb)) continue;
                if (t < box_t) box_t = t;
            }
            if (box_t < best_t) {
                second_t = best_t;
                best_t = box_t;
                best_box = i;
            } else if (box_t < second_t) {
                second_t = box_t;
            }
        }
        if (best_box >= 0 && second_t - best_t < eps * (fabs(best_t) > 1.0 ? fabs(best_t) : 1.0)) fl |= 1;
        if (best_box >= 0) {
            const double *c = boxes + 10 * best_box + 6;
            double *px = image + 4 * q;
            for (int k = 0; k < 3; ++k) px[k] = c[k] * c[3] + (1.0 - c[3]) * px[k];
            px[3] = c[3] + (1.0 - c[3]) * px[3];
        }
        if (flags) flags[q] = fl;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* bricks                                                             */
/* ------------------------------------------------------------------ */
static int64_t brick_cell(double p, int64_t B, int64_t nb) {
    int64_t c = (int64_t)floor(p / (double)B);
    if (c < 0) c = 0;
    if (c > nb - 1) c = nb - 1;
    return c;
}

/* Visibility key of brick (bx, by, bz). */
int64_t orc_brick_key(const orc_camera *cam, int64_t B, int64_t bx, int64_t by, int64_t bz) {
    int64_t b[3] = {bx, by, bz};
    if (cam->kind == 1) {
        int64_t key = 0;
        for (int a = 0; a < 3; ++a) {
            int64_t c = (int64_t)floor(cam->eye[a] / (double)B);
            key += llabs(b[a] - c);
        }
        return key;
    }
    double f[3], r[3], u[3];
    orc_basis(cam, f, r, u);
    int64_t key = 0;
    for (int a = 0; a < 3; ++a) key += (f[a] > 0 ? 1 : (f[a] < 0 ? -1 : 0)) * b[a];
    return key;
}

/* One brick's share of a ray: its key and id, and its partial in three
 * variants: [0] with the stop test A >= tau, [1] with tau - eps_stop, [2]
 * with tau + eps_stop (the stop decision flipped either way). */
typedef struct { int64_t key, id; double c[3][4]; int stopped[3]; } part_t;
static int part_cmp(const void *x, const void *y) {
    const part_t *a = x, *b = y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* Per-brick partials of the first `count` samples of ray r, in ray order
 * (bricks are convex, so each brick's samples are contiguous).  Returns the
 * number of partials in *parts (grown as needed); ORs flags into *fl. */
static int64_t brick_pass(const orc_scene *s, const orc_camera *cam, const orc_params *p, const ray_t *r,
                          int64_t B, const int64_t nb[3], int64_t count, part_t **parts, int64_t *cap, int *fl) {
    int ert = p->tau < 1.0;
    double thr[3] = {p->tau, p->tau - p->eps_stop, p->tau + p->eps_stop};
    int64_t np = 0, cur = -1;
    part_t *pc = NULL;
    for (int64_t k = 0; r->hit && k < count; ++k) {
        double pos[3];
        sample_pos(r, p->step, k, pos);
        int64_t cell[3];
        for (int a = 0; a < 3; ++a) {
            cell[a] = brick_cell(pos[a], B, nb[a]);
            double rel = pos[a] / (double)B - floor(pos[a] / (double)B);
            if ((rel * B < p->eps_pos || (1.0 - rel) * B < p->eps_pos) && pos[a] > 0 &&
                pos[a] < (double)(a == 0 ? s->nx : a == 1 ? s->ny : s->nz))
                *fl |= FLAG_BRICK;
        }
        int64_t id = (cell[2] * nb[1] + cell[1]) * nb[0] + cell[0];
        if (id != cur) {
            if (np == *cap) { *cap *= 2; *parts = realloc(*parts, sizeof(part_t) * (size_t)*cap); }
            pc = &(*parts)[np++];
            pc->id = id;
            pc->key = orc_brick_key(cam, B, cell[0], cell[1], cell[2]);
            for (int v = 0; v < 3; ++v) {
                pc->c[v][0] = pc->c[v][1] = pc->c[v][2] = pc->c[v][3] = 0.0;
                if (p->mode == 1) pc->c[v][0] = -INFINITY;
                pc->stopped[v] = 0;
            }
            cur = id;
        }
        double v, rgba[4];
        if (p->filter == 1) {
            double vl, vh;
            int amb;
            v = nearest(s, pos, p->eps_pos, &vl, &vh, &amb);
            if (amb) *fl |= FLAG_CELL;
        } else {
            v = orc_trilinear(s, pos, NULL, NULL);
        }
        if (p->mode == 1) {
            for (int w = 0; w < 3; ++w)
                if (v > pc->c[w][0]) pc->c[w][0] = v;
            continue;
        }
        orc_lut(s->lut, s->nlut, s->vmin, s->vmax, v, rgba, NULL, NULL, NULL);
        for (int w = 0; w < 3; ++w) {
            if (pc->stopped[w]) continue;
            double A = pc->c[w][3], a = rgba[3];
            for (int c = 0; c < 3; ++c) pc->c[w][c] += (1.0 - A) * a * rgba[c];
            pc->c[w][3] = A + (1.0 - A) * a;
            if (w == 0 && ert && fabs(pc->c[0][3] - p->tau) < p->eps_stop) *fl |= FLAG_STOP;
            if (ert && pc->c[w][3] >= thr[w]) pc->stopped[w] = 1;
        }
    }
    return np;
}

/* "Over" (composite) or maximum (MIP) of partials already in key order,
 * taking variant sel[i] of partial i. */
static void compose(const orc_params *p, const part_t *parts, int64_t np, const int *sel, double res[4]) {
    res[0] = res[1] = res[2] = res[3] = 0.0;
    if (p->mode == 1) res[0] = -INFINITY;
    for (int64_t i = 0; i < np; ++i) {
        const double *c = parts[i].c[sel ? sel[i] : 0];
        if (p->mode == 1) {
            if (c[0] > res[0]) res[0] = c[0];
        } else {
            double T = 1.0 - res[3];
            for (int ch = 0; ch < 4; ++ch) res[ch] += T * c[ch];
        }
    }
}

/* Bricked render: per-brick partials (own early stop), then "over" in key
 * order.  Composite: 4 channels; MIP: max over partial maxima.
 * If only_brick >= 0, writes that brick's partial instead of the composite.
 * flags gets FLAG_BRICK when a sample lies within eps_pos of a brick face,
 * FLAG_STOP when a brick's stop decision is within eps_stop of tau and
 * FLAG_COUNT when the ray's last-sample test is within its window.
 * lo / hi (may be NULL) receive, per channel, the smallest and largest
 * result over every combination of flipped decisions: the ray's sample
 * count n_lo, n or n_hi, and per brick whose stop decision lies in the
 * window, the stop at tau - eps_stop, tau or tau + eps_stop (a flipped
 * decision of one brick changes what "over" does with every brick behind
 * it, so the combinations are enumerated).  A brick-face tie (FLAG_BRICK)
 * is flagged only: lo / hi do not cover it. */
int orc_render_bricked(const float *vol, int64_t nx, int64_t ny, int64_t nz,
                       const float *lut, int32_t nlut, double vmin, double vmax,
                       const orc_camera *cam, const orc_params *p, int64_t B, int64_t only_brick,
                       const int32_t *pix, int64_t npix, double *out, double *lo, double *hi,
                       int32_t *flags, int nthreads) {
    orc_scene s = {vol, nx, ny, nz, lut, nlut, vmin, vmax};
    int chans = p->mode == 1 ? 1 : 4;
    int64_t nb[3] = {(nx + B - 1) / B, (ny + B - 1) / B, (nz + B - 1) / B};
    if (!pix) npix = (int64_t)cam->tile_w * cam->tile_h;
    int nt = nthreads_of(nthreads);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t x, y;
        if (pix) { x = pix[2 * q]; y = pix[2 * q + 1]; }
        else { x = q % cam->tile_w; y = q / cam->tile_w; }
        ray_t r;
        ray_prepare(&s, cam, p, cam->tile_x0 + x, cam->tile_y0 + y, &r);
        int fl = 0;
        if (r.hit && (r.n_lo != r.n || r.n_hi != r.n)) fl |= FLAG_COUNT;
        int64_t cap = 16;
        part_t *parts = malloc(sizeof(part_t) * (size_t)cap);
        double res[4], rlo[4], rhi[4];
        int64_t np = brick_pass(&s, cam, p, &r, B, nb, r.hit ? r.n : 0, &parts, &cap, &fl);
        if (only_brick >= 0) {
            res[0] = res[1] = res[2] = res[3] = 0.0;
            if (p->mode == 1) res[0] = -INFINITY;
            for (int64_t i = 0; i < np; ++i)
                if (parts[i].id == only_brick) memcpy(res, parts[i].c[0], sizeof res);
            memcpy(rlo, res, sizeof res);
            memcpy(rhi, res, sizeof res);
        } else {
            qsort(parts, (size_t)np, sizeof(part_t), part_cmp);
            compose(p, parts, np, NULL, res);
            memcpy(rlo, res, sizeof res);
            memcpy(rhi, res, sizeof res);
            /* candidate outcomes: every count variant, and per variant every
             * choice of stop for the bricks whose stop lies in the window */
            int64_t counts[3] = {r.n_lo, r.n, r.n_hi};
            for (int cv = 0; cv < 3 && r.hit; ++cv) {
                if (cv != 1 && counts[cv] == r.n) continue;
                int64_t m = cv == 1 ? np : brick_pass(&s, cam, p, &r, B, nb, counts[cv], &parts, &cap, &fl);
                if (cv != 1) qsort(parts, (size_t)m, sizeof(part_t), part_cmp);
                int *sel = calloc((size_t)(m > 0 ? m : 1), sizeof(int));
                int64_t amb[12], na = 0;
                for (int64_t i = 0; i < m && p->mode != 1; ++i) {
                    int differs = memcmp(parts[i].c[0], parts[i].c[1], sizeof parts[i].c[0]) != 0 ||
                                  memcmp(parts[i].c[0], parts[i].c[2], sizeof parts[i].c[0]) != 0;
                    if (differs && na < 12) amb[na++] = i;
                }
                int64_t combos = 1;
                for (int64_t i = 0; i < na; ++i) combos *= 3;
                for (int64_t cb = 0; cb < combos; ++cb) {
                    int64_t t = cb;
                    for (int64_t i = 0; i < na; ++i) { sel[amb[i]] = (int)(t % 3); t /= 3; }
                    double alt[4];
                    compose(p, parts, m, sel, alt);
                    for (int c = 0; c < 4; ++c) {
                        if (alt[c] < rlo[c]) rlo[c] = alt[c];
                        if (alt[c] > rhi[c]) rhi[c] = alt[c];
                    }
                }
                free(sel);
            }
            if (p->mode == 1 && p->filter == 1) {
                /* nearest MIP: the cell candidates, as in the single pass */
                double vlo = -INFINITY, vhi = -INFINITY;
                for (int64_t k = 0; r.hit && k < r.n_hi; ++k) {
                    double pos[3], vl, vh;
                    int a;
                    sample_pos(&r, p->step, k, pos);
                    nearest(&s, pos, p->eps_pos, &vl, &vh, &a);
                    if (k < r.n_lo && vl > vlo) vlo = vl;
                    if (vh > vhi) vhi = vh;
                }
                if (vlo < rlo[0]) rlo[0] = vlo;
                if (vhi > rhi[0]) rhi[0] = vhi;
            }
        }
        for (int c = 0; c < chans; ++c) {
            out[q * chans + c] = res[c];
            if (lo) lo[q * chans + c] = rlo[c];
            if (hi) hi[q * chans + c] = rhi[c];
        }
        if (flags) flags[q] = fl;
        free(parts);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* adjoint                                                            */
/* ------------------------------------------------------------------ */
/* Gradients of L with respect to the table and the voxels for the
 * composite render, given dL/d(out) per pixel (4 channels, premultiplied).
 * The stop index is held fixed.  With T_k = prod_{j<k}(1-a_j),
 * S_k = sum_{j>k} a_j c_j prod_{k<i<j}(1-a_i) and P_k = prod_{j>k}(1-a_j):
 *   dL/dc_k = gC T_k a_k,   dL/da_k = T_k [gC.(c_k - S_k) + gA P_k],
 * then through the table's linear interpolation and the trilinear weights
 * (clamped corners receive the weight of the coordinate they clamp to).
 * grad_lut (n x 4) and grad_vol (nz*ny*nx) are accumulated (+=). */
int orc_backward(const float *vol, int64_t nx, int64_t ny, int64_t nz,
                 const float *lut, int32_t nlut, double vmin, double vmax,
                 const orc_camera *cam, const orc_params *p, const double *gout,
                 double *grad_lut, double *grad_vol, int nthreads) {
    orc_scene s = {vol, nx, ny, nz, lut, nlut, vmin, vmax};
    int64_t npix = (int64_t)cam->tile_w * cam->tile_h, nvox = nx * ny * nz;
    int nt = nthreads_of(nthreads);
    double *gl_all = calloc((size_t)nt * nlut * 4, sizeof(double));
    double *gv_all = calloc((size_t)nt * nvox, sizeof(double));
    int ert = p->tau < 1.0;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gl = gl_all + (size_t)tid * nlut * 4;
        double *gv = gv_all + (size_t)tid * nvox;
        int64_t cap = 0;
        double *al = NULL, *cc = NULL, *dv = NULL, *wl = NULL, *wt = NULL;
        int32_t *jl = NULL;
        int64_t *ix = NULL;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npix; ++q) {
            int64_t x = q % cam->tile_w, y = q / cam->tile_w;
            ray_t r;
            ray_prepare(&s, cam, p, cam->tile_x0 + x, cam->tile_y0 + y, &r);
            if (!r.hit || r.n == 0) continue;
            if (r.n > cap) {
                cap = r.n;
                al = realloc(al, sizeof(double) * cap);
                cc = realloc(cc, sizeof(double) * cap * 3);
                dv = realloc(dv, sizeof(double) * cap * 4);
                wl = realloc(wl, sizeof(double) * cap);
                jl = realloc(jl, sizeof(int32_t) * cap);
                wt = realloc(wt, sizeof(double) * cap * 8);
                ix = realloc(ix, sizeof(int64_t) * cap * 8);
            }
            /* forward: record the samples actually taken */
            double A = 0.0;
            int64_t m = 0;
            for (int64_t k = 0; k < r.n; ++k) {
                double pos[3], rgba[4];
                sample_pos(&r, p->step, k, pos);
                double v = orc_trilinear(&s, pos, ix + 8 * k, wt + 8 * k);
                orc_lut(lut, nlut, vmin, vmax, v, rgba, jl + k, wl + k, dv + 4 * k);
                al[k] = rgba[3];
                cc[3 * k] = rgba[0]; cc[3 * k + 1] = rgba[1]; cc[3 * k + 2] = rgba[2];
                A += (1.0 - A) * rgba[3];
                m = k + 1;
                if (ert && A >= p->tau) break;
            }
            /* transmittance in front of each sample */
            const double *g = gout + 4 * q;
            double T = 1.0;
            double *Tk = malloc(sizeof(double) * m);
            for (int64_t k = 0; k < m; ++k) { Tk[k] = T; T *= (1.0 - al[k]); }
            /* reverse sweep with suffix quantities S (3 channels) and P */
            double S[3] = {0, 0, 0}, P = 1.0;
            for (int64_t k = m - 1; k >= 0; --k) {
                double a = al[k], t = Tk[k];
                double d_rgba[4];
                for (int c = 0; c < 3; ++c) d_rgba[c] = g[c] * t * a;
                double da = g[3] * P;
                for (int c = 0; c < 3; ++c) da += g[c] * (cc[3 * k + c] - S[c]);
                d_rgba[3] = t * da;
                double gs = 0.0;
                int32_t j = jl[k];
                double w = wl[k];
                for (int c = 0; c < 4 && j >= 0; ++c) {   /* j < 0: a blank sample uses no entry */
                    gl[4 * j + c] += (1.0 - w) * d_rgba[c];
                    gl[4 * (j + 1) + c] += w * d_rgba[c];
                    gs += d_rgba[c] * dv[4 * k + c];
                }
                for (int c8 = 0; c8 < 8; ++c8) gv[ix[8 * k + c8]] += wt[8 * k + c8] * gs;
                for (int c = 0; c < 3; ++c) S[c] = a * cc[3 * k + c] + (1.0 - a) * S[c];
                P *= (1.0 - a);
            }
            free(Tk);
        }
        free(al); free(cc); free(dv); free(wl); free(jl); free(wt); free(ix);
    }
    for (int t = 0; t < nt; ++t) {
        for (int64_t i = 0; i < (int64_t)nlut * 4; ++i) grad_lut[i] += gl_all[(size_t)t * nlut * 4 + i];
        for (int64_t i = 0; i < nvox; ++i) grad_vol[i] += gv_all[(size_t)t * nvox + i];
    }
    free(gl_all);
    free(gv_all);
    return 0;
}
