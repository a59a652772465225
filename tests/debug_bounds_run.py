"""Exercise every kernel family through the debug library (all sources
compiled with VR_DEBUG_BOUNDS) and print, as one JSON line, the number of
index-range violations its checks counted.  Run as its own process by
tests/test_gpu_debug_bounds.py with VRCUBE_LIB naming the debug library."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

from paper_1012_2909_amd import synth, vr  # noqa: E402


def main():
    counts = {}
    R = vr.Renderer(0)
    try:
        shape = (70, 45, 52)
        vol = synth.make_cube(synth.CubeSpec(shape, 10, seed=23, fwhm_z=(4.0, 20.0)))
        R.load_volume(torch.from_numpy(vol), orientations=3)
        R.set_lut(synth.lut_ramp(alpha_scale=0.25))
        base = R.get_tuning()
        cams = [synth.orbit_camera(shape, seed=s, w=96, h=72) for s in (3, 9, 14)]
        cams.append(synth.Camera(synth.PERSPECTIVE, (35.0, 22.0, 26.0), (10.0, 5.0, 60.0), (0.0, -1.0, 0.0),
                                 fovy_deg=70.0, full_w=64, full_h=48))   # eye inside the cube
        for ci, cam in enumerate(cams):
            R.set_camera(cam)
            for path in (1, 2, 3, 4):
                R.set_tuning(**{**base, "path": path})
                for kw in (dict(mode="composite"), dict(mode="composite", ert=1.0), dict(mode="mip"),
                           dict(mode="mip", filt="nearest")):
                    if path == 4 and kw["mode"] != "mip":
                        continue
                    R.render(**kw)
            R.set_tuning(**base)
            img, ws = R.render(save=True)
            gl = torch.zeros((256, 4), device="cuda")
            gv = torch.zeros(shape, device="cuda")
            R.render_backward(torch.ones_like(img), ws, gl, gv)
            R.render_depth()
            counts[f"single pass, camera {ci}"] = int(R.debug_bounds_violations())
        views = [c for c in cams[:3]]
        R.render_batch(views, mode="composite")
        R.render_batch(views, mode="mip")
        counts["batch"] = int(R.debug_bounds_violations())
        for brick in (16, 13):
            R.load_volume(torch.from_numpy(vol), brick=brick)
            R.set_lut(synth.lut_ramp(alpha_scale=0.25))
            for cam in cams:
                R.set_camera(cam)
                for path in (0, 1):
                    R.set_tuning(**{**base, "path": path})
                    R.render_bricked(mode="composite")
                    R.render_bricked(mode="mip")
                    R.render_bricked(mode="mip", filt="nearest")
                R.set_tuning(**base)
            counts[f"bricks {brick}"] = int(R.debug_bounds_violations())
    finally:
        R.close()
    print(json.dumps({"lib": os.path.basename(vr.LIB_PATH), "violations": counts}), flush=True)


if __name__ == "__main__":
    main()
