"""Throughput of the ray caster on the 8 GiB spectral cube at 1920x1080.

Workload: the 1024x1024x2048 float32 cube (noise + 500 sources, seed 2),
1920x1080 perspective orbit cameras (fovy 30, bounding-sphere fit) at 16
seeded orbit angles, step 0.5 voxel.  One step renders one frame (the next
angle) in both modes: composite (256-entry grey ramp over [-3, 10], early
stop at alpha 0.99) and trilinear maximum-intensity projection.  Inputs are
resident in HBM before the timed region; the volume layout (transcode) is
timed separately.  Launch shapes are the library's defaults: the path (LDS-staged
voxel boxes for MIP, direct gathers for the early-stopping composite) and
the LDS budget are chosen per view.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 16] [--warmup 2] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue ceiling: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one lane-instruction
# slot per lane and clock (a wave64 instruction takes 4 clocks of a SIMD;
# the 157.3 TFLOP/s FP32 figure counts packed FMAs, two flops each, twice this)
VALU_PEAK = 256 * 4 * 16 * 2.4e9


def stored_valu(key):
    """VALU lane-instruction slots per sample measured by the counters in
    profiles/traffic.json for this kernel revision, or None."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        v = json.load(open(tf)).get("valu")
        if v and v.get("kernel_rev") == kernel_revision():
            return float(v[key])
    except (OSError, ValueError, KeyError, TypeError):
        pass
    return None


def valu_ceiling(key, samples, ms):
    """The ALU side of a kernel's roofline: counted VALU work over its time
    against VALU_PEAK (None without counters for this revision)."""
    per = stored_valu(key)
    if per is None:
        return None
    achieved = per * samples / (ms * 1e-3)
    return {"bound": "alu", "achieved": round(achieved / 1e12, 2), "peak": round(VALU_PEAK / 1e12, 2),
            "unit": "T VALU lane-instructions/s", "frac": round(achieved / VALU_PEAK, 4),
            "valu_per_sample": per}
N_ANGLES = 16


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def angle_seeds():
    return [int(s) for s in np.random.default_rng(2).integers(0, 2**31 - 1, N_ANGLES)]


def kernel_revision():
    """Hash of the kernels' sources: stored traffic counters are only valid
    for the revision they were measured on."""
    h = hashlib.sha1()
    for f in ("k_slab.hip", "k_march.hip", "k_mipblk.hip", "vr_common.h", "vr_api.hip"):
        h.update(open(os.path.join(ROOT, "paper_1012_2909_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work of the oracle sample")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "all"],
                    help="storage type of the cube ('all': each in turn, bricked64 only)")
    ap.add_argument("--streamed-slots", type=int, default=0,
                    help="bricked64: also render one frame streamed from pinned host memory through a cache of this "
                         "many bricks (FP16)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune one launch shape per mode on the first angle (default: the library's automatic "
                         "per-view choice of path and LDS budget)")
    ap.add_argument("--tune-cache", default="/tmp/vrcube_tune.json", help="autotuner cache file ('' for none)")
    ap.add_argument("--measure-cache", default="/tmp/vrcube_bench_measure.json",
                    help="cache of the per-angle sample counts and touched blocks ('' for none)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP16/BF16-storage, batched, backward and bricked variants reported beside the main "
                         "figure")
    ap.add_argument("--no-bricked", action="store_true", help="skip the bricked 64 GiB variant")
    ap.add_argument("--workload", default="spectral8", choices=["spectral8", "bricked64", "deep8", "backward",
                                                                "choices"],
                    help="spectral8: the headline 8 GiB cube at 1920x1080 (default); bricked64: the 64 GiB cube as "
                         "256^3 bricks, the 9600x5400 frame of the 5x5 wall; deep8: the 8 GiB cube's composite with the alpha/64 "
                         "ramp alone; backward: forward + adjoint on the 128x128x256 cube at 1024x1024 alone; "
                         "choices: the 8 GiB frames under each design choice and its alternative, one render per case "
                         "and angle (the last three for counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy 4 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.workload == "spectral8" and args.storage == "all":
        ap.error("--storage all applies to --workload bricked64")

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the multi-GPU sort-last exchange is "
              f"described in the design notes, not built", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_1012_2909_amd import synth, vr

    dev = torch.device("cuda", 0)
    if args.copy_probe:
        a = torch.ones(1 << 29, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 4 copies of 2 GiB (2 GiB read + 2 GiB written each)")
        return
    if args.workload == "bricked64":
        run_bricked64(args)
        return
    if args.workload in ("deep8", "backward"):
        run_single(args)
        return
    if args.workload == "choices":
        run_choices(args)
        return
    spec = synth.CUBE_8GIB
    W, H = 1920, 1080
    step = 0.5
    t = time.time()
    vol = synth.make_cube(spec)
    log(f"cube {spec.shape} generated in {time.time() - t:.1f}s")
    cams = [synth.orbit_camera(spec.shape, seed=s, w=W, h=H) for s in angle_seeds()]
    lut = synth.lut_ramp()

    R = vr.Renderer(0)
    src = torch.from_numpy(vol).to(dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    R.load_volume(src, storage=args.storage, brick=0, orientations=3)
    e1.record()
    torch.cuda.synchronize()
    load_ms = e0.elapsed_time(e1)
    esz = {"f32": 4, "f16": 2, "bf16": 2}[args.storage]
    store_bytes = R.storage.numel()
    load_gbs = (vol.nbytes + store_bytes) / (load_ms * 1e-3) / 1e9
    log(f"layout transcode (3 orientation copies, {store_bytes / 1e9:.1f} GB) {load_ms:.2f} ms, {load_gbs:.0f} GB/s moved")
    del src
    torch.cuda.empty_cache()
    R.set_lut(lut)

    modes = {"composite": dict(mode="composite", filt="trilinear", step=step, ert=0.99),
             "mip": dict(mode="mip", filt="trilinear", step=step, ert=0.99)}
    outs = {"composite": torch.empty((H, W, 4), dtype=torch.float32, device=dev),
            "mip": torch.empty((H, W), dtype=torch.float32, device=dev)}

    # launch shapes per mode (autotuned on the first angle)
    tunes = {}
    R.set_camera(cams[0])
    for name, kw in modes.items():
        if not args.tune:
            tunes[name] = R.get_tuning()
        else:
            tunes[name] = R.autotune(mode=kw["mode"], filt=kw["filt"], step=step, ert=kw["ert"],
                                     cache_path=args.tune_cache or None)
        log(f"{name}: launch shape {tunes[name]}")

    # measurement passes (not timed): samples per frame and touched blocks per
    # angle.  Cached per source revision so that a profiled rerun holds only
    # the timed launches.
    mkey = f"{kernel_revision()}|{args.storage}|{spec.shape}|{W}x{H}|{step}"
    mpath = args.measure_cache
    samples = touched = None
    if mpath and os.path.exists(mpath):
        try:
            m = json.load(open(mpath))
            if m.get("key") == mkey:
                samples, touched = m["samples"], m["touched"]
                log(f"sample counts and touched blocks from {mpath}")
        except (OSError, ValueError, KeyError):
            samples = touched = None
    if samples is None:
        samples = {n: [] for n in modes}
        touched = {n: [] for n in modes}
        for c in cams:
            R.set_camera(c)
            for name, kw in modes.items():
                R.set_tuning(**tunes[name])
                samples[name].append(int(R.count_samples(**kw).to(torch.int64).sum().item()))
                touched[name].append(R.touched_blocks(mode=kw["mode"], filt=kw["filt"], step=step, ert=kw["ert"]))
        if mpath:
            with open(mpath, "w") as f:
                json.dump({"key": mkey, "samples": samples, "touched": touched}, f)
    for name in modes:
        log(f"{name}: {np.mean(samples[name]) / 1e9:.3f} G samples/frame (mean of {N_ANGLES} angles), "
            f"{np.mean(touched[name]):.0f} touched 8^3 blocks")
    out_bytes = {"composite": W * H * 16, "mip": W * H * 4}
    alg_bytes = {n: [b * 512 * esz + out_bytes[n] + (lut.table.nbytes if n == "composite" else 0)
                     for b in touched[n]] for n in modes}

    # one workspace for every timed render (the object-order MIP's ray records,
    # the bundle order), allocated before the timed region
    ws_need = 1
    for c in cams:
        R.set_camera(c)
        for name, kw in modes.items():
            R.set_tuning(**tunes[name])
            ws_need = max(ws_need, R.workspace_bytes(mode=kw["mode"], filt=kw["filt"], step=step, ert=kw["ert"]))
    ws = torch.empty(ws_need, dtype=torch.uint8, device=dev)
    # one untimed render of every angle in every mode: the kernels of the timed
    # steps are then loaded (a code object is loaded at its first launch, some
    # milliseconds) whatever the warm-up count
    for c in cams:
        R.set_camera(c)
        for name, kw in modes.items():
            R.set_tuning(**tunes[name])
            R.render(out=outs[name], workspace=ws, **kw)
    torch.cuda.synchronize()

    def run_step(k, evs=None):
        R.set_camera(cams[k % N_ANGLES])
        for name, kw in modes.items():
            R.set_tuning(**tunes[name])
            if evs is not None:
                evs[name][0].record()
            R.render(out=outs[name], workspace=ws, **kw)
            if evs is not None:
                evs[name][1].record()

    for k in range(args.warmup):
        run_step(k)
    torch.cuda.synchronize()
    ev = [{n: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for n in modes}
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        run_step(k, ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch = {n: [ev[k][n][0].elapsed_time(ev[k][n][1]) for k in range(args.steps)] for n in modes}
    ms_step = wall * 1e3 / args.steps
    total_samples = sum(samples[n][k % N_ANGLES] for n in modes for k in range(args.steps))
    value = total_samples / wall / 1e9
    mean_ms = {n: float(np.mean(v)) for n, v in per_launch.items()}
    fps = {n: 1e3 / mean_ms[n] for n in mean_ms}
    gsps = {n: sum(samples[n][k % N_ANGLES] for k in range(args.steps)) / (sum(per_launch[n]) * 1e-3) / 1e9
            for n in modes}
    frac = {n: float(np.mean([alg_bytes[n][k % N_ANGLES] / (per_launch[n][k] * 1e-3) / 1e9 / HBM_PEAK_GBS
                              for k in range(args.steps)])) for n in modes}
    log(f"step {ms_step:.3f} ms; per launch {mean_ms}; fps {fps}")

    # roofline of the dominant kernel: the MIP march over the whole cube
    dom = max(mean_ms, key=mean_ms.get)
    alg_per_launch = float(np.mean([alg_bytes[dom][k % N_ANGLES] for k in range(args.steps)]))
    achieved = alg_per_launch / (mean_ms[dom] * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            tr = json.load(open(tf))
            e = tr.get(f"{dom}_{args.storage}")
            if e and e.get("kernel_rev") == kernel_revision():
                traffic = e["bytes_per_launch"]
        except (OSError, ValueError, KeyError):
            traffic = None
    mip_kernels = {0: "MIP frame: k_slab (ray bundles), or k_raytable + k_mip_blocks + k_mip_decode (object order) "
                      "on views oblique to the axes",
                   1: "k_march<MIP>", 2: "k_slab<MIP>", 3: "k_march_c<MIP>",
                   4: "k_raytable + k_mip_blocks + k_mip_decode"}
    kname = {"mip": mip_kernels.get(tunes["mip"]["path"], "MIP"),
             "composite": "k_march<COMPOSITE>" if tunes["composite"]["path"] != 2 else "k_slab<COMPOSITE>"}
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname[dom],
            "algorithmic_bytes_per_launch": int(alg_per_launch)}
    valu_roof = None
    if dom == "mip" and args.storage == "f32" and tunes["mip"]["path"] == 0:
        valu_roof = valu_ceiling("mip_f32", float(np.mean([samples["mip"][k % N_ANGLES] for k in range(args.steps)])),
                                 mean_ms["mip"])

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(vol, lut, cams[0], step, args.cpu_seconds)
    variants = None
    if not args.no_variants and args.storage == "f32":
        variants = run_variants(R, vol, cams, lut, modes, samples, mean_ms, step)
    if not args.no_variants and not args.no_bricked and args.storage == "f32":
        # the bricked 64 GiB cube (FP32, FP16, BF16 storage) and a frame of it
        # streamed from pinned host memory through a quarter-size brick cache
        R.storage = None
        del vol
        torch.cuda.empty_cache()
        t = time.time()
        vol64 = synth.make_cube(synth.CUBE_64GIB)
        log(f"cube {synth.CUBE_64GIB.shape} generated in {time.time() - t:.1f}s")
        b64 = bricked64_measure(vol64, ["f32", "f16", "bf16"], 5, streamed_slots=256, log_fn=log)
        del vol64
        nvox = 4096 * 2048 * 2048
        for st, r in b64["storage"].items():
            esz = 4 if st == "f32" else 2
            for mode in ("composite", "mip"):
                alg = nvox * esz + 9600 * 5400 * (16 if mode == "composite" else 4)
                r[mode]["hbm_roofline_frac"] = round(alg / (r[mode]["ms_per_frame"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                if st == "f32":
                    r[mode]["valu_ceiling_k3"] = valu_ceiling(f"bricked64_f32_{mode}", r[mode]["samples_per_frame"],
                                                              r[mode]["ms_per_frame"])
        variants = variants or {}
        variants["bricked_64gib_9600x5400"] = b64

    rec = {
        "metric": "G ray-samples/s + fps at 1920x1080 on 8 GiB cube; % HBM roofline",
        "value": round(value, 3),
        "unit": "G ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"{args.storage}-storage/f32",
        "data": "synthetic",
        "config": {"workload": "1024x1024x2048 float32 cube (8 GiB, noise + 500 sources), 1920x1080 perspective "
                               f"orbit cameras at {N_ANGLES} seeded angles, step 0.5 voxel; per step one frame in "
                               "composite (ramp table, stop at alpha 0.99) and trilinear MIP",
                   "storage": args.storage, "frames_per_step": 2, "orientation_copies": 3},
        "fps": {k: round(v, 2) for k, v in fps.items()},
        "gsamples_per_s": {k: round(v, 2) for k, v in gsps.items()},
        "samples_per_frame_mean": {n: int(np.mean(samples[n])) for n in modes},
        "samples_per_angle": {n: [int(x) for x in samples[n]] for n in modes},
        "hbm_roofline_frac": {n: round(v, 4) for n, v in frac.items()},
        "ms_per_angle": {n: [round(float(np.mean([per_launch[n][k] for k in range(args.steps) if k % N_ANGLES == a])), 3)
                             for a in range(min(N_ANGLES, args.steps))] for n in modes},
        "launch_shapes": tunes,
        "load_volume": {"ms": round(load_ms, 3), "GBps_moved": round(load_gbs, 1)},
        "roofline": roof,
        "valu_ceiling": valu_roof,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(rec), flush=True)
    R.close()


def _time_ms(fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_variants(R, vol, cams, lut, modes, samples, fp32_ms, step):
    """The storage, batching and differentiation forms of the renderer, each
    beside the plain FP32 render on this GPU, with its accuracy against the
    FP64 oracle on seeded pixels."""
    import torch
    import oracle
    from paper_1012_2909_amd import synth, vr
    from paper_1012_2909_amd.autograd import VolumeRenderFn   # noqa: F401  (the differentiable entry point)
    out = {}
    dev = torch.device("cuda", 0)
    W, H = 1920, 1080
    pix = synth.sample_pixels(W, H, 3000, 7)
    grid = np.stack(np.meshgrid(np.arange(3, W, 8), np.arange(3, H, 8)), -1).reshape(-1, 2).astype(np.int32)
    gm = oracle.render(vol, lut, cams[0], mode="mip", pixels=grid, step=step)["out"]
    bright = grid[np.isfinite(gm) & (gm >= 8.0)][:1500]
    # (1) FP16 / BF16 storage of the 8 GiB cube: 16 angles, both modes
    for st in ("f16", "bf16"):
        src = torch.from_numpy(vol).to(dev)
        R.load_volume(src, storage=st, brick=0, orientations=3)
        del src
        torch.cuda.empty_cache()
        R.set_lut(lut)
        ms = {}
        for name, kw in modes.items():
            t = []
            for c in cams:
                R.set_camera(c)
                o = torch.empty((H, W, 4) if name == "composite" else (H, W), device=dev)
                t.append(_time_ms(lambda: R.render(out=o, **kw), 2))
            ms[name] = float(np.mean(t))
        R.set_camera(cams[0])
        img = R.render(**modes["composite"]).cpu().numpy()
        ref = oracle.render(vol, lut, cams[0], pixels=pix, step=step)
        g = img[pix[:, 1], pix[:, 0]].astype(np.float64)
        clean = ref["flags"] == 0
        err = float(np.abs(g[clean] - ref["out"][clean]).max())
        # the worst case: pixels whose rays cross bright voxels (the oracle's
        # MIP >= 8 on a strided grid of the frame), where the rounding of the
        # stored values moves alpha most
        g_b = img[bright[:, 1], bright[:, 0]].astype(np.float64)
        ref_b = oracle.render(vol, lut, cams[0], pixels=bright, step=step)
        cl_b = ref_b["flags"] == 0
        err_b = float(np.abs(g_b[cl_b] - ref_b["out"][cl_b]).max()) if cl_b.any() else None
        out[f"{st}_storage"] = {
            "workload": "8 GiB cube, 1920x1080, 16 orbit angles", "storage_bytes": int(R.storage.numel()),
            "ms_per_frame": {k: round(v, 3) for k, v in ms.items()},
            "speedup_vs_f32": {k: round(fp32_ms[k] / ms[k], 3) for k in ms},
            "gsamples_per_s": {k: round(float(np.mean(samples[k])) / (ms[k] * 1e-3) / 1e9, 2) for k in ms},
            "composite_max_abs_err_vs_fp64_oracle_on_f32_cube": err,
            "composite_max_abs_err_on_bright_pixels": err_b, "bar": 2e-3,
            "meets_bar": bool(max(err, err_b or 0.0) <= 2e-3),
            "accuracy_sample": f"{int(clean.sum())} seeded pixels of the first angle; {int(cl_b.sum())} pixels "
                               f"whose ray's maximum is >= 8 (bright sources)"}
        log(f"variant {st} storage: {out[f'{st}_storage']}")
    # (1b) the deep composite: ramp table with alpha / 64 (rays run ~1300
    # samples before the early stop), FP32 storage, 16 angles; the library
    # picks the LDS-staged kernel because no ray can stop within 64 voxels
    src = torch.from_numpy(vol).to(dev)
    R.load_volume(src, storage="f32", brick=0, orientations=3)
    del src
    torch.cuda.empty_cache()
    lutb = synth.lut_ramp(alpha_scale=1.0 / 64.0)
    R.set_lut(lutb)
    kw = dict(mode="composite", filt="trilinear", step=step, ert=0.99)
    o = torch.empty((H, W, 4), device=dev)
    t_b, s_b, a_b = [], [], []
    for c in cams:
        R.set_camera(c)
        s_b.append(int(R.count_samples(**kw).to(torch.int64).sum().item()))
        a_b.append(R.touched_blocks(mode="composite", filt="trilinear", step=step, ert=0.99) * 512 * 4 + W * H * 16)
        t_b.append(_time_ms(lambda: R.render(out=o, **kw), 3))
    R.set_camera(cams[0])
    img = R.render(**kw).cpu().numpy()
    pb = synth.sample_pixels(W, H, 400, 8)
    rb = oracle.render(vol, lutb, cams[0], pixels=pb, step=step, eps_stop=2e-5)
    gb = img[pb[:, 1], pb[:, 0]].astype(np.float64)
    clb = rb["flags"] == 0
    mip_ms = fp32_ms["mip"]
    out["deep_composite_alpha_over_64"] = {
        "workload": "8 GiB cube, 1920x1080, 16 orbit angles, ramp table with alpha / 64, stop at 0.99",
        "ms_per_frame": round(float(np.mean(t_b)), 3), "ms_per_angle": [round(x, 3) for x in t_b],
        "over_mip_frame": round(float(np.mean(t_b)) / mip_ms, 3),
        "gsamples_per_s": round(float(np.sum(s_b)) / (float(np.sum(t_b)) * 1e-3) / 1e9, 2),
        "samples_per_frame_mean": int(np.mean(s_b)),
        "roofline": {"bound": "hbm", "algorithmic_bytes_per_frame": int(np.mean(a_b)),
                     "achieved_GBps": round(float(np.mean([a / (t * 1e-3) / 1e9 for a, t in zip(a_b, t_b)])), 1),
                     "frac": round(float(np.mean([a / (t * 1e-3) / 1e9 / HBM_PEAK_GBS for a, t in zip(a_b, t_b)])), 4)},
        "composite_max_abs_err_vs_fp64_oracle": float(np.abs(gb[clb] - rb["out"][clb]).max()), "bar": 1e-5,
        "accuracy_sample": f"{int(clb.sum())} seeded pixels of the first angle"}
    log(f"variant deep composite: {out['deep_composite_alpha_over_64']}")
    R.set_lut(lut)
    R.storage = None
    torch.cuda.empty_cache()
    # (2) batched: 64 uneven views of the 512 MiB cube, FP16 storage, one
    # persistent launch replayed from a HIP graph, against the same views one
    # by one and against FP32 storage
    spec = synth.CUBE_512MIB
    v4 = synth.make_cube(spec)
    bcams, bluts = synth.batch_views(spec.shape, 4, n_views=64)
    res = {}
    for st in ("f16", "f32"):
        R.load_volume(torch.from_numpy(v4).to(dev), storage=st)
        packed = R.stack_luts(bluts)
        nsamp = 0
        for c, l in zip(bcams, bluts):
            R.set_lut(l)
            R.set_camera(c)
            nsamp += int(R.count_samples().to(torch.int64).sum().item())
        s = torch.cuda.Stream()
        outs = [torch.empty((c.tile[3], c.tile[2], 4), device=dev) for c in bcams]

        def batch():
            with torch.cuda.stream(s):
                R.render_batch(bcams, packed, outs=outs, use_graph=True, stream=s)
            s.synchronize()
        t_graph = _time_ms(batch, 5)

        def one_by_one():
            for c, l in zip(bcams, bluts):
                R.set_lut(l)
                R.set_camera(c)
                R.render()
        t_single = _time_ms(one_by_one, 2)
        t_tuned = None
        if st == "f16":
            # the autotuner's choice of bundle, LDS budget, slab and persistent groups
            base = R.get_tuning()
            R.autotune_batch(bcams, bluts)
            tuned = R.get_tuning()
            t_tuned = _time_ms(batch, 5)
            R.set_tuning(**base)
        res[st] = (t_graph, t_single, nsamp, t_tuned, tuned if st == "f16" else None)
        if st == "f16":
            worst = 0.0
            for i in range(0, 64, 8):
                p = synth.sample_pixels(bcams[i].tile[2], bcams[i].tile[3], 200, 40 + i)
                r_ = oracle.render(v4, bluts[i], bcams[i], pixels=p, step=step)
                g = outs[i].cpu().numpy()[p[:, 1], p[:, 0]].astype(np.float64)
                cl = r_["flags"] == 0
                worst = max(worst, float(np.abs(g[cl] - r_["out"][cl]).max()))
    out["batch_64_views_f16"] = {
        "workload": "512x512x1024 cube, 64 orbit views of 256..1920 x 256..1080 px, random tables",
        "graph_ms": round(res["f16"][0], 3), "one_by_one_ms": round(res["f16"][1], 3),
        "graph_speedup_vs_one_by_one": round(res["f16"][1] / res["f16"][0], 2),
        "f32_storage_graph_ms": round(res["f32"][0], 3),
        "autotuned_graph_ms": round(res["f16"][3], 3), "autotuned_launch_shape": res["f16"][4],
        "autotuned_speedup_vs_default": round(res["f16"][0] / res["f16"][3], 3),
        "gsamples_per_s": round(res["f16"][2] / (res["f16"][0] * 1e-3) / 1e9, 2),
        "composite_max_abs_err_vs_fp64_oracle_on_f32_cube": worst, "bar": 2e-3,
        "accuracy_sample": "200 seeded pixels of every 8th view"}
    log(f"variant batch: {out['batch_64_views_f16']}")
    del v4
    # (3) differentiation: forward with checkpoints + adjoint on the
    # 128x128x256 cube at 1024x1024, against the plain forward
    spec = synth.CUBE_DIFF
    v5 = synth.make_cube(spec)
    cam = synth.orbit_camera(spec.shape, seed=5, w=1024, h=1024)
    R.load_volume(torch.from_numpy(v5).to(dev), orientations=1)
    R.set_lut(lut)
    R.set_camera(cam)
    t_plain = _time_ms(lambda: R.render(), 5)
    img, ws = R.render(save=True)
    gimg = torch.ones_like(img)
    gl = torch.zeros((lut.table.shape[0], 4), device=dev)
    gv = torch.zeros(spec.shape, device=dev)
    t_fwd = _time_ms(lambda: R.render(save=True, workspace=ws), 5)

    def bwd():
        gl.zero_()
        gv.zero_()
        R.render_backward(gimg, ws, gl, gv)
    t_bwd = _time_ms(bwd, 5)
    out["backward_128x128x256_1024x1024"] = {
        "forward_ms": round(t_plain, 3), "forward_with_checkpoints_ms": round(t_fwd, 3),
        "backward_ms": round(t_bwd, 3), "backward_over_forward": round(t_bwd / t_plain, 2),
        "accuracy": "gradients vs the FP64 oracle adjoint within 1e-4 of the largest entry (GPU test suite)"}
    log(f"variant backward: {out['backward_128x128x256_1024x1024']}")
    return out


def bricked64_measure(vol, storages, steps, streamed_slots=0, log_fn=None):
    """The 64 GiB cube as 256^3 bricks (one-voxel apron), the 9600x5400 frame
    of the 5x5 wall of 1920x1080 panels: per-brick partial images then the
    sort-last "over"; composite (ramp table with alpha / 64, early stop at
    0.99) and trilinear MIP, for each storage type; optionally one frame
    streamed from pinned host memory through a cache of `streamed_slots`
    bricks (FP16).  Returns a dict of results."""
    import torch
    from paper_1012_2909_amd import synth, vr
    dev = torch.device("cuda", 0)
    spec = synth.CUBE_64GIB
    R = vr.Renderer(0)
    lut = synth.lut_ramp(alpha_scale=1.0 / 64.0)
    frame = synth.orbit_camera(spec.shape, seed=3, w=9600, h=5400)
    # the wall's frame is rendered in one call: every brick renders its
    # partial over its whole footprint once (the 25 panels are windows of the
    # same frame and stitch to it bit for bit), instead of once per panel it
    # covers
    R.set_camera(frame)
    out = {"workload": "2048x2048x4096 float32 cube (64 GiB) as 256^3 bricks, 9600x5400 frame (the 5x5 wall of "
                       "1920x1080 panels) rendered in one call", "storage": {}}
    samples = {}
    for st in storages:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        R.describe_volume(spec.shape, storage=st, brick=256)
        torch.cuda.synchronize()
        e0.record()
        for z0 in range(0, spec.shape[0], 256):
            R.load_slab(torch.from_numpy(vol[z0:z0 + 256]).to(dev), z0)
        e1.record()
        torch.cuda.synchronize()
        R.set_lut(lut)
        res = {"storage_bytes": int(R.storage.numel()), "load_ms_including_upload": round(e0.elapsed_time(e1), 1)}
        for mode in ("composite", "mip"):
            if mode not in samples:
                samples[mode] = int(R.count_samples(mode=mode).to(torch.int64).sum().item())
            ms = _time_ms(lambda: R.render_bricked(mode=mode), steps)
            res[mode] = {"ms_per_frame": round(ms, 2), "frames_timed": steps,
                         "gsamples_per_s": round(samples[mode] / (ms * 1e-3) / 1e9, 2),
                         "samples_per_frame": samples[mode]}
            if log_fn:
                log_fn(f"bricked {st} {mode}: {res[mode]}")
        out["storage"][st] = res
    if streamed_slots:
        t = time.time()
        host = vr.pack_bricks_host(vol, storage="f16", brick=256)
        pack_s = time.time() - t
        R.storage = None
        torch.cuda.empty_cache()
        R.describe_streamed_volume(spec.shape, host, storage="f16", brick=256, cache_slots=streamed_slots)
        R.set_lut(lut)
        res = {"slots": streamed_slots, "bricks": 1024, "host_bytes": int(host.numel()),
               "pack_seconds": round(pack_s, 1)}
        for mode in ("composite", "mip"):
            c0, h0, _ = R.stream_stats()
            torch.cuda.synchronize()
            t = time.perf_counter()
            R.render_bricked(mode=mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            c1, h1, _ = R.stream_stats()
            bb = host.numel() / 1024
            res[mode] = {"ms_per_frame": round(dt * 1e3, 1), "bricks_copied": c1 - c0, "cache_hits": h1 - h0,
                         "host_to_device_GBps": round((c1 - c0) * bb / dt / 1e9, 1)}
            if log_fn:
                log_fn(f"streamed f16 {mode}: {res[mode]}")
        out["streamed_f16"] = res
        R.storage = None
        del host
    R.close()
    return out


def run_bricked64(args):
    """Bricked 64 GiB frame alone (prints one JSON line of its own)."""
    from paper_1012_2909_amd import synth
    t = time.time()
    vol = synth.make_cube(synth.CUBE_64GIB)
    log(f"cube {synth.CUBE_64GIB.shape} generated in {time.time() - t:.1f}s")
    storages = ["f32", "f16", "bf16"] if args.storage == "all" else [args.storage]
    res = bricked64_measure(vol, storages, max(5, args.steps // 4), args.streamed_slots, log)
    print(json.dumps(res), flush=True)


# Design choices and their alternatives on the 8 GiB cube (mode, what, tuning):
# LDS-staged voxel boxes against direct gathers, the orientation copy chosen per
# view against copy 0 alone, and for early-stopping composites fixed 16x4 ray
# packets against one-row packets and against ballot compaction of finished
# rays.  Every case is one kernel per frame.
CHOICES = [
    ("mip", "LDS-staged voxel boxes, automatic copy (k_slab)", dict(path=2)),
    ("mip", "direct gathers, automatic copy (k_march_u)", dict(path=1)),
    ("mip", "LDS-staged voxel boxes, x-fastest copy forced (k_slab)", dict(path=2, copy=0)),
    ("composite", "16x4 ray packets (k_march_u)", dict(path=1)),
    ("composite", "64x1 ray packets (k_march_u)", dict(path=1, packet_w=64, packet_h=1)),
    ("composite", "16x4 packets with ballot compaction of finished rays (k_march_c)", dict(path=3)),
]
CHOICE_ANGLES = 4


def run_choices(args):
    """One render per (case, angle) in CHOICES order on the first
    CHOICE_ANGLES angles -- the order the counter passes see the kernels in --
    then timed repeats and the sample counts.  Prints one JSON line."""
    import torch
    from paper_1012_2909_amd import synth, vr
    dev = torch.device("cuda", 0)
    spec = synth.CUBE_8GIB
    vol = synth.make_cube(spec)
    R = vr.Renderer(0)
    R.load_volume(torch.from_numpy(vol).to(dev), orientations=3)
    del vol
    R.set_lut(synth.lut_ramp())
    cams = [synth.orbit_camera(spec.shape, seed=s, w=1920, h=1080) for s in angle_seeds()[:CHOICE_ANGLES]]
    base = R.get_tuning()
    outs = {m: torch.empty((1080, 1920) if m == "mip" else (1080, 1920, 4), device=dev) for m in ("mip", "composite")}
    for mode, _, tune in CHOICES:              # the counted renders, in order
        R.set_tuning(**{**base, **tune})
        for cam in cams:
            R.set_camera(cam)
            R.render(mode=mode, out=outs[mode])
    torch.cuda.synchronize()
    res = []
    for mode, what, tune in CHOICES:
        R.set_tuning(**{**base, **tune})
        ms, n = [], 0
        for cam in cams:
            R.set_camera(cam)
            ms.append(_time_ms(lambda: R.render(mode=mode, out=outs[mode]), max(1, args.steps // 4)))
            n += int(R.count_samples(mode=mode).to(torch.int64).sum().item())
        res.append({"mode": mode, "case": what, "tuning": tune, "ms_per_frame": [round(x, 3) for x in ms],
                    "samples": n})
    R.set_tuning(**base)
    R.close()
    print(json.dumps({"workload": f"8 GiB cube, 1920x1080, first {CHOICE_ANGLES} orbit angles", "cases": res}),
          flush=True)


def run_single(args):
    """One workload alone, for counter runs: the deep composite of the 8 GiB
    cube over the 16 angles, or forward + adjoint on the differentiable
    cube.  Prints one JSON line of its own."""
    import torch
    from paper_1012_2909_amd import synth, vr
    dev = torch.device("cuda", 0)
    R = vr.Renderer(0)
    steps = max(1, args.steps)
    if args.workload == "deep8":
        spec = synth.CUBE_8GIB
        vol = synth.make_cube(spec)
        R.load_volume(torch.from_numpy(vol).to(dev), orientations=3)
        R.set_lut(synth.lut_ramp(alpha_scale=1.0 / 64.0))
        cams = [synth.orbit_camera(spec.shape, seed=s, w=1920, h=1080) for s in angle_seeds()]
        o = torch.empty((1080, 1920, 4), device=dev)
        ms = []
        for k in range(steps):
            R.set_camera(cams[k % N_ANGLES])
            ms.append(_time_ms(lambda: R.render(out=o), 1))
        res = {"workload": "8 GiB cube, 1920x1080, ramp alpha/64 composite", "ms_per_frame": ms}
    else:
        spec = synth.CUBE_DIFF
        vol = synth.make_cube(spec)
        R.load_volume(torch.from_numpy(vol).to(dev), orientations=1)
        lut = synth.lut_ramp()
        R.set_lut(lut)
        R.set_camera(synth.orbit_camera(spec.shape, seed=5, w=1024, h=1024))
        img, ws = R.render(save=True)
        gimg = torch.ones_like(img)
        gl = torch.zeros((lut.table.shape[0], 4), device=dev)
        gv = torch.zeros(spec.shape, device=dev)
        ms = []
        for _ in range(steps):
            R.render(save=True, workspace=ws, out=img)
            gl.zero_()
            gv.zero_()
            ms.append(_time_ms(lambda: R.render_backward(gimg, ws, gl, gv), 1))
        res = {"workload": "128x128x256 cube, 1024x1024, forward with checkpoints + adjoint", "backward_ms": ms}
    R.close()
    print(json.dumps(res), flush=True)


def cpu_baseline(vol, lut, cam, step, seconds):
    """The FP64 oracle on a bounded, seeded sample of the first angle's pixels
    (both modes), timed on the host cores."""
    import oracle
    threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "0")) or 64))
    W, H = cam.tile[2], cam.tile[3]
    rng = np.random.default_rng(12345)
    # size the sample from a probe of pixels that hit the cube (misses cost nothing)
    probe = np.stack([rng.integers(0, W, 2000), rng.integers(0, H, 2000)], 1).astype(np.int32)
    t = time.perf_counter()
    oracle.render(vol, lut, cam, mode="mip", pixels=probe, step=step, threads=threads)
    oracle.render(vol, lut, cam, pixels=probe, step=step, threads=threads)
    per_px = max((time.perf_counter() - t) / len(probe), 1e-8)
    n = int(min(W * H, max(2000, seconds / per_px)))
    pix = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], 1).astype(np.int32)
    log(f"cpu baseline: FP64 oracle on {n} seeded pixels x 2 modes, {threads} threads")
    t = time.perf_counter()
    a = oracle.render(vol, lut, cam, mode="mip", pixels=pix, step=step, threads=threads)
    b = oracle.render(vol, lut, cam, pixels=pix, step=step, threads=threads)
    dt = time.perf_counter() - t
    s = int(a["taken"].sum() + b["taken"].sum())
    return {"value": round(s / dt / 1e9, 5), "unit": "G ray-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} seeded pixels of the first 1920x1080 angle, MIP + composite: {s} samples in {dt:.1f}s"}


if __name__ == "__main__":
    main()
