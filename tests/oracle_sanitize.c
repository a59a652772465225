/* Drives every entry point of the FP64 oracle on a small cube with blank
 * (NaN) voxels, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitize.py): an out-of-bounds read, a cast
 * of NaN to an integer index or an overflow aborts the run.  Test
 * infrastructure only. */
#include "../oracle/vr_oracle.c"

#include <stdio.h>

static uint32_t lcg = 12345u;
static double urand(void) { lcg = lcg * 1664525u + 1013904223u; return (lcg >> 8) / 16777216.0; }

int main(void) {
    enum { NX = 12, NY = 10, NZ = 9, NL = 256, W = 24, H = 18 };
    static float vol[NX * NY * NZ], lut[NL * 4];
    for (int i = 0; i < NX * NY * NZ; ++i) vol[i] = (float)(6.0 * urand() - 2.0);
    for (int i = 0; i < NX * NY * NZ; i += 7) vol[i] = NAN;          /* blanks */
    for (int j = 0; j < NL; ++j)
        for (int c = 0; c < 4; ++c) lut[4 * j + c] = (float)j / (NL - 1) * (c == 3 ? 0.3f : 1.0f);
    orc_camera cams[3] = {
        {1, {-8.0, -6.0, -14.0}, {6.0, 5.0, 4.5}, {0.0, -1.0, 0.0}, 40.0, 0.0, 0.0, W, H, 0, 0, W, H},
        {1, {5.3, 4.1, 3.7}, {20.0, 2.0, 9.0}, {0.0, -1.0, 0.0}, 100.0, 0.0, 0.0, W, H, 0, 0, W, H},
        {0, {-10.0, 12.0, -9.0}, {6.0, 5.0, 4.5}, {0.0, -1.0, 0.0}, 0.0, 9.0, 7.0, W, H, 0, 0, W, H}};
    static double out[W * H * 4], lo[W * H * 4], hi[W * H * 4], gl[NL * 4], gv[NX * NY * NZ], img[W * H * 4];
    static double gout[W * H * 4];
    static int32_t flags[W * H];
    static int64_t taken[W * H];
    double boxes[2 * 10] = {1, 1, 1, 5, 4, 6, 1, 0, 0, 1, -3, 2, -2, 4, 8, 20, 0, 1, 0, 0.5};
    for (int i = 0; i < W * H * 4; ++i) gout[i] = urand() - 0.5;
    for (int c = 0; c < 3; ++c)
        for (int mode = 0; mode < 2; ++mode)
            for (int filt = 0; filt < 2; ++filt) {
                orc_params p = {mode, filt, 0.5, 0.9, 1e-3, 1e-9, 1e-7};
                orc_render(vol, NX, NY, NZ, lut, NL, -2.0, 4.0, &cams[c], &p, NULL, 0, out, lo, hi, flags, taken, 2);
                orc_render_bricked(vol, NX, NY, NZ, lut, NL, -2.0, 4.0, &cams[c], &p, 4, -1, NULL, 0, out, lo, hi,
                                   flags, 2);
                orc_depth(vol, NX, NY, NZ, lut, NL, -2.0, 4.0, &cams[c], &p, 0.5, 1e-6, NULL, 0, out, lo, hi, flags,
                          2);
                if (mode == 0 && filt == 0) {
                    for (int i = 0; i < NL * 4; ++i) gl[i] = 0.0;
                    for (int i = 0; i < NX * NY * NZ; ++i) gv[i] = 0.0;
                    orc_backward(vol, NX, NY, NZ, lut, NL, -2.0, 4.0, &cams[c], &p, gout, gl, gv, 2);
                }
                for (int i = 0; i < W * H * 4; ++i) img[i] = 0.1;
                orc_overlay(&cams[c], boxes, 2, 0.75, 1e-3, NULL, 1e-9, img, flags, 2);
            }
    printf("oracle sanitizer run done\n");
    return 0;
}
