"""Throughput of the ray caster on the 8 GiB spectral cube at 1920x1080.

One step renders one 1920x1080 frame of the 1024x1024x2048 float32 cube
(noise + 500 sources) from a perspective orbit camera (seed 2, fovy 30,
step 0.5 voxel) in both modes: composite (256-entry grey ramp over
[-3, 10], early stop at alpha 0.99) and maximum-intensity projection
(trilinear).  Inputs are resident in HBM before the timed region; the
volume layout (transcode) is timed separately.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work of the oracle sample")
    ap.add_argument("--brick", type=int, default=0, help="brick edge of the layout (0 = one brick)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sort-last exchange "
              f"is a design, not a build", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_1012_2909_amd import synth, vr

    dev = torch.device("cuda", 0)
    spec = synth.CUBE_8GIB
    W, H = 1920, 1080
    step = 0.5
    t = time.time()
    vol = synth.make_cube(spec)
    log(f"cube {spec.shape} generated in {time.time() - t:.1f}s")
    cam = synth.orbit_camera(spec.shape, seed=2, w=W, h=H)
    lut = synth.lut_ramp()

    R = vr.Renderer(0)
    src = torch.from_numpy(vol).to(dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    R.load_volume(src, storage=args.storage, brick=args.brick)
    e1.record()
    torch.cuda.synchronize()
    load_ms = e0.elapsed_time(e1)
    store_bytes = R.storage.numel()
    load_gbs = (vol.nbytes + store_bytes) / (load_ms * 1e-3) / 1e9
    log(f"layout transcode {load_ms:.2f} ms ({load_gbs:.0f} GB/s moved)")
    del src
    torch.cuda.empty_cache()
    R.set_lut(lut)
    R.set_camera(cam)

    modes = [("composite", dict(mode="composite", filt="trilinear", step=step, ert=0.99)),
             ("mip", dict(mode="mip", filt="trilinear", step=step, ert=0.99))]
    outs = {"composite": torch.empty((H, W, 4), dtype=torch.float32, device=dev),
            "mip": torch.empty((H, W), dtype=torch.float32, device=dev)}

    # measurement passes (not timed): samples per frame and touched blocks
    samples, touched = {}, {}
    for name, kw in modes:
        c = R.count_samples(**{k: v for k, v in kw.items()})
        samples[name] = int(c.to(torch.int64).sum().item())
        touched[name] = R.touched_blocks(mode=kw["mode"], filt=kw["filt"], step=step, ert=kw["ert"])
        log(f"{name}: {samples[name] / 1e9:.3f} G samples/frame, {touched[name]} touched 8^3 blocks")

    esz = {"f32": 4, "f16": 2, "bf16": 2}[args.storage]
    out_bytes = {"composite": W * H * 16, "mip": W * H * 4}
    alg_bytes = {n: touched[n] * 512 * esz + out_bytes[n] + (lut.table.nbytes if n == "composite" else 0)
                 for n, _ in modes}

    def run_step(evs=None):
        for i, (name, kw) in enumerate(modes):
            if evs is not None:
                evs[name][0].record()
            R.render(out=outs[name], **kw)
            if evs is not None:
                evs[name][1].record()

    for _ in range(args.warmup):
        run_step()
    torch.cuda.synchronize()

    per_launch = {n: [] for n, _ in modes}
    ev_sets = [{n: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for n, _ in modes}
               for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        run_step(ev_sets[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for k in range(args.steps):
        for n, _ in modes:
            per_launch[n].append(ev_sets[k][n][0].elapsed_time(ev_sets[k][n][1]))
    ms_step = wall * 1e3 / args.steps
    total_samples = samples["composite"] + samples["mip"]
    value = total_samples / (ms_step * 1e-3) / 1e9
    mean_ms = {n: float(np.mean(v)) for n, v in per_launch.items()}
    fps = {n: 1e3 / mean_ms[n] for n in mean_ms}
    gsps = {n: samples[n] / (mean_ms[n] * 1e-3) / 1e9 for n in mean_ms}
    log(f"step {ms_step:.3f} ms; per launch {mean_ms}; fps {fps}")

    # roofline of the dominant kernel (the MIP march over the whole cube)
    dom = max(mean_ms, key=mean_ms.get)
    achieved = alg_bytes[dom] / (mean_ms[dom] * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            tr = json.load(open(tf))
            key = f"{dom}_{args.storage}_b{args.brick}"
            if key in tr and tr[key].get("kernel_rev") == kernel_revision():
                traffic = tr[key]["bytes_per_launch"]
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"k_march<{args.storage},{dom}>", "algorithmic_bytes": alg_bytes[dom]}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(vol, lut, cam, step, args.cpu_seconds)

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
        "config": {"workload": "1024x1024x2048 float32 cube (8 GiB), 1920x1080 perspective orbit (seed 2), "
                               "step 0.5; composite (ramp table, stop at alpha 0.99) + trilinear MIP",
                   "brick": args.brick, "storage": args.storage, "frames_per_step": 2},
        "fps": {k: round(v, 2) for k, v in fps.items()},
        "gsamples_per_s": {k: round(v, 2) for k, v in gsps.items()},
        "samples_per_frame": samples,
        "hbm_roofline_frac": {n: round(alg_bytes[n] / (mean_ms[n] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for n in mean_ms},
        "load_volume": {"ms": round(load_ms, 3), "GBps": round(load_gbs, 1)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    R.close()


def kernel_revision():
    """Hash of the march kernel's source; traffic counters are only valid for it."""
    import hashlib
    h = hashlib.sha1()
    for f in ("k_march.hip", "vr_common.h"):
        h.update(open(os.path.join(ROOT, "paper_1012_2909_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def cpu_baseline(vol, lut, cam, step, seconds):
    """The FP64 oracle on a bounded, seeded sample of the same frame's pixels
    (both modes), timed on the host cores."""
    import oracle
    threads = min(os.cpu_count() or 1, 64)
    rng = np.random.default_rng(12345)
    W, H = cam.tile[2], cam.tile[3]
    # probe on a small sample to size the real one
    n_probe = 400
    pix = np.stack([rng.integers(0, W, n_probe), rng.integers(0, H, n_probe)], 1).astype(np.int32)
    t = time.perf_counter()
    a = oracle.render(vol, lut, cam, mode="mip", pixels=pix, step=step, threads=threads)
    b = oracle.render(vol, lut, cam, pixels=pix, step=step, threads=threads)
    dt = time.perf_counter() - t
    per_px = max(dt / n_probe, 1e-7)
    n = int(min(W * H, max(1000, seconds / per_px)))
    pix = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], 1).astype(np.int32)
    log(f"cpu baseline: oracle on {n} sampled pixels x 2 modes, {threads} threads")
    t = time.perf_counter()
    a = oracle.render(vol, lut, cam, mode="mip", pixels=pix, step=step, threads=threads)
    b = oracle.render(vol, lut, cam, pixels=pix, step=step, threads=threads)
    dt = time.perf_counter() - t
    s = int(a["taken"].sum() + b["taken"].sum())
    return {"value": round(s / dt / 1e9, 5), "unit": "G ray-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} seeded pixels of the 1920x1080 frame, MIP + composite, {s} samples in {dt:.1f}s"}


if __name__ == "__main__":
    main()
