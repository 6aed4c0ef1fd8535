#!/usr/bin/env python3
"""Benchmark of the gfx950 normal bake.

Workload (one GPU): high-poly icosphere level 8 (1,310,720 triangles) displaced
by seeded 4-octave gradient noise, baked onto the level-5 icosphere (20,480
triangles) with a per-face grid atlas of 2048^2 texels, max_dist 0.12.  Inputs
are synthetic and resident in HBM before timing.

A step is one whole bake through the C ABI: low-poly prep, UV raster, LBVH
build over the high-poly, traversal + tangent-space encode, dilation, and the
backward pass of a squared-error loss when the library provides it.  value =
covered-texel rays per second of the full step.

Besides the JSON line's required fields it reports:
  roofline      the dominant kernel (traversal) against the VALU issue peak,
                with its duration from HIP events recorded on the bake stream
                over the timed steps, and the algorithmic op count from an
                instrumented bake (box and triangle tests);
  cpu_baseline  the FP64 brute-force oracle on a bounded sample of the same
                rays, on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 VALU operations per test, counted from the kernel source (traverse.hip):
#   box test (one child):   6 sub + 6 mul (slabs), 4 min/max, 2 mul (widening),
#                           2 min/max (clamp to the bound)              = 20
#   triangle test:          3 x (3 sub + 3 x 3 mul/fma) shear = 36,
#                           3 edge functions x 3 = 9, det 2, tolerance
#                           compare 4, T 3                              = 54
#   per ray (setup+encode): position, normal, frame, shear setup, hit
#                           normal and projection                        = 100
OPS_BOX, OPS_TRI, OPS_RAY = 20, 54, 100
# MI355X VALU issue rate: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed FP32)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

WORKLOAD = "noise4 icosphere L8 (1,310,720 tris) -> icosphere L5 (20,480 tris), 2048^2 atlas, max_dist 0.12"
METRIC = "baked rays/s (1.3M-tri→20k-tri, 2048² atlas); fwd+bwd ms; % HBM/VALU peak"


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2605_26137_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash):
    """HBM bytes per traversal launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic_traverse_noise4_L8_L5_2048.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_hash:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(asset, target_s):
    """The oracle as it stands (FP64 brute force over every triangle) on a
    seeded sample of the workload's covered texels."""
    import numpy as np
    import oracle
    cores = oracle.set_threads(0)
    face, _ = oracle.raster(asset.lo_UV, asset.res)
    cov = np.nonzero(face >= 0)[0]
    rng = np.random.default_rng(1234)

    def run(n):
        sample = np.sort(rng.choice(cov, size=n, replace=False))
        t0 = time.perf_counter()
        oracle.bake(asset, method="brute", texels=sample)
        return time.perf_counter() - t0

    t_small = run(64)
    n = int(max(64, min(cov.size, 64 * target_s / max(t_small, 1e-3))))
    dt = run(n)
    return {"value": n / dt, "unit": "rays/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} seeded covered texels of {cov.size}, FP64 brute force over all "
                      f"{asset.hi_F.shape[0]} triangles, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trav-block", type=int, default=0)
    ap.add_argument("--trav-stack", type=int, default=0)
    ap.add_argument("--trav-persist", type=int, default=-1)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build bakes on a single device "
              "(see DESIGN.md for how the bake would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2605_26137_amd.bake as B
    from synth import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # a plain copy kernel of known size: the reference for scaling the
        # FETCH_SIZE / WRITE_SIZE counters into bytes
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)
        return
    print(f"[bench] {B.version()} on {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)
    asset = make_config(2)
    t = B.to_device(asset, dev)
    res, md = asset.res, asset.max_dist
    kw = dict(trav_block=args.trav_block, trav_stack=args.trav_stack, trav_persist=args.trav_persist)
    first = B.bake_normals(*t, res, md, **kw)
    ws, out_map, out_hit = first.workspace, first.map, first.hit
    torch.cuda.synchronize()
    rays = first.ray_count()

    def step(timing):
        B.bake_normals(*t, res, md, timing=timing, workspace=ws, out_map=out_map,
                       out_hit=out_hit, **kw)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # timed region: whole steps back to back, stage events on the bake stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    hist = B.stage_history(min(args.steps, 64))
    stage_ms = {name: float(np.mean(hist[:, k])) for k, name in enumerate(B.STAGES)}
    print(f"[bench] {args.steps} steps, {ms_per_step:.3f} ms/step, stages {stage_ms}",
          file=sys.stderr, flush=True)

    # algorithmic op count of the traversal: one instrumented bake, untimed
    cnt = B.bake_normals(*t, res, md, count=True, workspace=ws, out_map=out_map, out_hit=out_hit)
    n_box, n_tri = cnt.test_counts()
    ops = n_box * OPS_BOX + n_tri * OPS_TRI + rays * OPS_RAY
    trav_s = stage_ms["traverse"] / 1e3
    achieved = ops / trav_s / 1e12
    khash = source_hash("traverse.hip", "lbvh.hip")
    roof = {"kernel": "traverse_kernel (traversal + encode)", "bound": "alu",
            "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(khash),
            "ops_per_launch": ops, "box_tests_per_ray": n_box / rays, "tri_tests_per_ray": n_tri / rays,
            "launch_ms": stage_ms["traverse"], "source_hash": khash}

    out = {
        "metric": METRIC,
        "value": rays / (ms_per_step / 1e3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "rays": rays, "texels": res * res,
                   "hi_tris": int(asset.hi_F.shape[0]), "lo_tris": int(asset.lo_F.shape[0]),
                   "step": "forward bake incl. BVH build"},
        "fwd_ms": stage_ms["forward"],
        "stages_ms": stage_ms,
        "texels_per_s": res * res / (ms_per_step / 1e3),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(asset, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
