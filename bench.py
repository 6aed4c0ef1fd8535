#!/usr/bin/env python3
"""Benchmark of the gfx950 normal bake.

Workload (one GPU): high-poly icosphere level 8 (1,310,720 triangles) displaced
by seeded 4-octave gradient noise, baked onto the level-5 icosphere (20,480
triangles) with a per-face grid atlas of 2048^2 texels, max_dist 0.12.  Inputs
are synthetic and resident in HBM before timing.

A step is one pass of the whole path through the C ABI: the forward bake
(low-poly prep, UV raster, LBVH build over the high-poly, traversal + tangent-
space encode, dilation) with its state saved, the squared-error loss against a
target map baked from a second noise seed, and the backward pass to dL/dlo_V
and dL/dhi_N.  value = covered-texel rays per second of the whole step.  The
step is first timed as plain API calls (which also gives the per-stage
times), then recorded once into a HIP graph and replayed K times; the replays
must reproduce the eager outputs bitwise, and their time is the reported one
(--eager reports the plain calls instead).

Besides the JSON line's required fields it reports:
  roofline      the dominant kernel (traversal) against the VALU issue peak,
                with its duration from HIP events recorded on the bake stream
                over the timed steps, and the algorithmic op count from an
                instrumented bake (box and triangle tests);
  cpu_baseline  the FP64 brute-force oracle on a bounded sample of the same
                rays, on this host's cores;
  batch         (--batch-assets N) N uneven assets (50k-2M triangles, 512^2-
                2048^2 atlases) baked forward + backward as one graph-recorded
                batch, against the same bakes as N sequential plain calls.
"""
import argparse
import hashlib
import json
import math
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
# closest-point query: point-to-box distance (3 x (2 sub + 2 max) + 3 mul/fma +
# compare = 16); nearest point on a triangle through the projection branch
# (edges 6, normal 9, |n|^2 3, signed distance 6, projection 4, corner
# offsets 9, three cross products 27, three weights 9, compare 2 = 75)
OPS_BOX_PT, OPS_TRI_PT = 16, 75
# MI355X VALU issue rate: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed FP32)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    1: "ripple icosphere L4 (5,120 tris) -> icosphere L1 (80 tris), 128^2 atlas, max_dist 0.1",
    2: "noise4 icosphere L8 (1,310,720 tris) -> icosphere L5 (20,480 tris), 2048^2 atlas, max_dist 0.12",
    3: "noise6+bumps icosphere L9 (5,242,880 tris) -> icosphere L6 (81,920 tris), 4096^2 atlas, max_dist 0.15",
}
WORKLOAD = WORKLOADS[2]
METRIC = "baked rays/s (1.3M-tri→20k-tri, 2048² atlas); fwd+bwd ms; % HBM/VALU peak"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_traverse_noise4_L8_L5_2048.json")


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2605_26137_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash):
    """HBM bytes per traversal launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_hash:
        return None
    return d.get("bytes_per_launch")


def sized_sample(run, pilot, limit, target_s):
    """Grow a sample until one run of the oracle takes about target_s seconds
    (a small pilot overstates the per-item time: fixed set-up cost, idle
    threads); returns (n, seconds) of the last run."""
    n, dt = pilot, run(pilot)
    for _ in range(3):
        if dt >= 0.6 * target_s or n >= limit:
            break
        n = int(min(limit, max(n + 1, n * target_s / max(dt, 1e-3))))
        dt = run(n)
    return n, dt


QEM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_qem_eval_noise4_L8_10k.json")


def measured_qem_traffic():
    """HBM bytes of the per-edge evaluation over one run, from the committed
    rocprofv3 counter runs, if taken on the current source; else None."""
    if not os.path.exists(QEM_TRAFFIC_FILE):
        return None
    with open(QEM_TRAFFIC_FILE) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash("qem.hip"):
        return None
    return d.get("bytes_per_run")


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it), for the CPU baselines."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(asset, target_s, max_dist, kind):
    """The oracle as it stands (FP64 brute force over every triangle) on a
    seeded sample of the workload's covered texels (forward query: the
    oracle's per-ray adjoint is negligible next to it)."""
    import numpy as np
    import oracle
    cores = oracle.set_threads(0)
    face, _ = oracle.raster(asset.lo_UV, asset.res)
    cov = np.nonzero(face >= 0)[0]
    rng = np.random.default_rng(1234)

    def run(n):
        sample = np.sort(rng.choice(cov, size=n, replace=False))
        t0 = time.perf_counter()
        oracle.bake(asset, method="brute", texels=sample, kind=kind, max_dist=max_dist)
        return time.perf_counter() - t0

    n, dt = sized_sample(run, 64, cov.size, target_s)
    return {"value": n / dt, "unit": "rays/s", "cores": cores, "cpu": cpu_model(), "kind": "oracle",
            "sample": f"{n} seeded covered texels of {cov.size}, FP64 brute-force {kind} query over all "
                      f"{asset.hi_F.shape[0]} triangles, {dt:.1f} s"}


VIS_WORKLOAD = ("hidden-face pass: noise-displaced shell (icosphere L5, 20,480 tris) around a hidden "
                "sphere (1,280 tris), 512 viewpoints on a sphere of radius 2.5, 1024^2 rays each, "
                "BVH build + first-hit rays + normal-gated flood fill")
# camera ray setup per ray (frame, pixel direction, ray-space shear): ~60 FP32 ops
OPS_CAM = 60


def bench_visibility(args, B, log):
    """The hidden-face pass (Sec. 6.2) at the paper's settings: one step is
    one whole call (BVH build over the mesh, 512 x 1024^2 camera rays, flood
    fill)."""
    import numpy as np
    import torch
    from synth import meshes as M
    dev = torch.device("cuda:0")
    V, F, n_out = M.hidden_face_mesh()
    n_views, res, t_far = 512, 1024, 4.0
    tan_half = math.tan(math.radians(30.0))
    eyes = M.sphere_viewpoints(n_views, [0, 0, 0], 2.5)
    Vd, Fd, Ed = (torch.from_numpy(x).to(dev) for x in (V, F, eyes))
    ws = torch.empty(B.visibility_workspace_size(V.shape[0], F.shape[0]), dtype=torch.uint8, device=dev)
    out = (torch.empty(F.shape[0], dtype=torch.uint8, device=dev), torch.empty(F.shape[0], dtype=torch.uint8,
                                                                               device=dev))
    rays = n_views * res * res

    def step(timing):
        return B.visibility(Vd, Fd, Ed, [0, 0, 0], tan_half, res, t_far, workspace=ws, out=out, timing=timing)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    hist = B.stage_history(min(args.steps, 64))
    stage_ms = {name: float(np.mean(hist[:, k])) for k, name in enumerate(B.VIS_STAGES) if name != "unused"}
    r = B.visibility(Vd, Fd, Ed, [0, 0, 0], tan_half, res, t_far, workspace=ws, out=out, count=True)
    n_box, n_tri, trips = r.counter(1), r.counter(2), r.counter(3)
    vis = r.visible.cpu().numpy()
    ext = r.exterior.cpu().numpy()
    assert r.status() == 0
    log(f"[bench] visibility: {ms:.3f} ms/step, stages {stage_ms}; shell visible {vis[:n_out].mean():.4f}, "
        f"exterior {ext[:n_out].mean():.4f}, inner visible {int(vis[n_out:].sum())}")
    ops = n_box * OPS_BOX + n_tri * OPS_TRI + rays * OPS_CAM
    achieved = ops / (stage_ms["rays"] / 1e3) / 1e12
    out_json = {
        "metric": "camera rays/s of the hidden-face pass (512 views x 1024^2, 21,760-tri mesh)",
        "value": rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": VIS_WORKLOAD, "rays": rays, "tris": int(F.shape[0]), "views": n_views, "res": res},
        "stages_ms": stage_ms,
        "roofline": {"kernel": "visibility_kernel (camera rays, first hit)", "bound": "alu", "achieved": achieved,
                     "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "box_tests_per_ray": n_box / rays, "tri_tests_per_ray": n_tri / rays,
                     "lane_utilisation": (n_box / 2 + n_tri) / (64 * trips) if trips else None,
                     "launch_ms": stage_ms["rays"]},
        "paper_context_s_per_mesh": 0.179,
    }
    if not args.no_cpu_baseline:
        import oracle
        cores = oracle.set_threads(0)
        rng = np.random.default_rng(1234)

        def run(n):
            which = np.sort(rng.choice(rays, size=n, replace=False))
            P, D = oracle.camera_rays(eyes, [0, 0, 0], tan_half, res, which=which)
            t1 = time.perf_counter()
            oracle.first_hit(V, F, P, D, t_far, "brute")
            return time.perf_counter() - t1

        n, dt = sized_sample(run, 256, rays, args.cpu_seconds)
        out_json["cpu_baseline"] = {"value": n / dt, "unit": "rays/s", "cores": cores, "cpu": cpu_model(), "kind": "oracle",
                                    "sample": f"{n} seeded camera rays of {rays}, FP64 brute-force first hit over "
                                              f"all {F.shape[0]} triangles, {dt:.1f} s"}
    return out_json


MAP_WORKLOAD = ("backprojection precompute: noise + bump displaced icosphere L5 (20,480 tris) with a 2048^2 "
                "per-face grid atlas, the ten texturing views at radius 2.5, 1024^2 depth buffers; G-buffer "
                "raster + BVH build + depth rays + per texel-view projection, incidence and visibility")


def bench_view_maps(args, B, log):
    """The backprojection precompute (Sec. 7.4, TextureGen Postprocessing) at the paper's scale: one step
    is one whole call; value = covered texel-views per second."""
    import numpy as np
    import torch
    from synth import meshes as M
    dev = torch.device("cuda:0")
    V, F, UV = M.textured_bumpy_mesh(level=5, res=2048)
    res, img, t_far, tol = 2048, 1024, 5.0, 2e-3
    tan_half = math.tan(math.radians(30.0))
    eyes = M.texture_views(2.5)
    Vd, Fd, UVd, Ed = (torch.from_numpy(x).to(dev) for x in (V, F, UV, eyes))
    K = eyes.shape[0]
    ws = torch.empty(B.view_maps_workspace_size(V.shape[0], F.shape[0], res, K, img), dtype=torch.uint8, device=dev)
    out = (torch.empty((K, res, res, 2), dtype=torch.float32, device=dev),
           torch.empty((K, res, res), dtype=torch.float32, device=dev))

    def step(timing, count=False):
        return B.view_maps(Vd, Fd, UVd, res, Ed, [0, 0, 0], tan_half, img, t_far, tol, workspace=ws, out=out,
                           timing=timing, count=count)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    hist = B.stage_history(min(args.steps, 64))
    stage_ms = {name: float(np.mean(hist[:, k])) for k, name in enumerate(B.MAP_STAGES) if name != "unused"}
    r = step(False, count=True)
    torch.cuda.synchronize()
    inc = out[1].cpu().numpy()
    n_box, n_tri, trips = r.counter(1), r.counter(2), r.counter(3)
    rays_depth = K * img * img
    covered = r.counter(0)
    tv = covered * K
    log(f"[bench] view maps: {ms:.3f} ms/step, stages {stage_ms}; {covered} covered texels, weight from some view "
        f"{(inc.reshape(K, -1).max(0) > 0).sum() / max(covered, 1):.4f}")
    ops = n_box * OPS_BOX + n_tri * OPS_TRI + rays_depth * OPS_CAM
    achieved = ops / (stage_ms["depth_rays"] / 1e3) / 1e12
    # the maps stage writes 12 B per texel-view (both outputs, every texel)
    # after reading the ray list (16 B per covered texel) and the depth buffers
    map_bytes = 12 * K * res * res + 16 * covered + 4 * rays_depth
    out_json = {
        "metric": "covered texel-views/s of the backprojection precompute (20,480-tri mesh, 2048^2 atlas, 10 views)",
        "value": tv / (ms / 1e3), "unit": "texel-views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": MAP_WORKLOAD, "covered_texels": covered, "views": K, "depth_res": img,
                   "tris": int(F.shape[0])},
        "stages_ms": stage_ms,
        "roofline": {"kernel": "visibility_kernel (depth rays, first hit)", "bound": "alu", "achieved": achieved,
                     "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "box_tests_per_ray": n_box / rays_depth, "tri_tests_per_ray": n_tri / rays_depth,
                     "lane_utilisation": (n_box / 2 + n_tri) / (64 * trips) if trips else None,
                     "launch_ms": stage_ms["depth_rays"]},
        "maps_stage": {"bound": "hbm", "bytes": map_bytes, "ms": stage_ms["maps"],
                       "achieved_GBps": map_bytes / (stage_ms["maps"] / 1e3) / 1e9, "peak_GBps": 8000.0},
        "paper_context_s": 1.455,
    }
    if not args.no_cpu_baseline:
        # the oracle on the whole workload (its own FP64 BVH for the depth
        # rays), repeated until about cpu_seconds have passed
        import oracle
        cores = oracle.set_threads(0)
        reps, t1 = 0, time.perf_counter()
        while reps == 0 or time.perf_counter() - t1 < args.cpu_seconds:
            vm = oracle.view_maps(V, F, UV, res, eyes, [0, 0, 0], tan_half, img, t_far, tol)
            reps += 1
        dt = time.perf_counter() - t1
        out_json["cpu_baseline"] = {"value": reps * vm.texels.size * K / dt, "unit": "texel-views/s",
                                    "cores": cores, "cpu": cpu_model(), "kind": "oracle",
                                    "sample": f"the whole workload x {reps} ({vm.texels.size} covered texels x {K} "
                                              f"views, {K} depth buffers of {img}^2 by the oracle's FP64 BVH), "
                                              f"{dt:.1f} s"}
    return out_json


def bench_simplify(args, B, log):
    """Quadric edge-collapse simplification (Sec. 6.1) of the bake's high-poly
    (1.31M faces) to 10,000 faces: one step is one whole blocking call (all
    rounds, inputs resident in HBM); value = faces removed per second."""
    import numpy as np
    import torch
    from synth import shapes as S
    V, F, target, name = S.simplify_input(2)
    Vd, Fd = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    ws = torch.empty(B.qem_workspace_size(V.shape[0], F.shape[0]), dtype=torch.uint8, device="cuda")
    out = (torch.empty_like(Vd), torch.empty_like(Fd))

    def step():
        return B.qem_simplify(Vd, Fd, target, workspace=ws, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eval_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = B.qem_simplify(Vd, Fd, target, workspace=ws, out=out, timing=True)
        eval_ms += r.times_ms[0]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    eval_ms /= args.steps
    removed = F.shape[0] - r.F.shape[0]
    # algorithmic bytes of the per-edge evaluation over the run: per round each
    # live vertex's position, quadric, list offsets and boundary flag (116 B),
    # each face and its three face-list entries (24 B), and per edge its ends,
    # two ring entries and the written cost bits, face count and placement
    # (45 B); live vertices from Euler's formula (closed genus-0 mesh)
    st = r.stats.astype(np.int64)
    faces_before = np.concatenate([[F.shape[0]], st[:-1, 3]])
    verts = 2 + st[:, 0] - faces_before
    algo = float(np.sum(116 * verts + 24 * faces_before + 45 * st[:, 0]))
    achieved = algo / (eval_ms / 1e3) / 1e9
    log(f"[bench] simplify: {ms:.3f} ms/step, {r.rounds} rounds, {r.F.shape[0]} faces; evaluation {eval_ms:.3f} ms, "
        f"{achieved:.0f} GB/s algorithmic")
    out_json = {
        "metric": "faces removed per second by QEM simplification (1.31M-face mesh -> 10,000 faces)",
        "value": removed / (ms / 1e3), "unit": "faces/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "QEM simplification with edge-constrained optimal placement: " + name +
                   ", rho 0.25 (cheapest quarter of the allowed edges eligible per round)",
                   "faces_in": int(F.shape[0]), "faces_out": int(r.F.shape[0]), "rounds": int(r.rounds),
                   "edges_evaluated": int(r.stats[:, 0].sum())},
        "roofline": {"kernel": "qem_eval_kernel (per-edge collapse evaluation, summed over the rounds of a run)",
                     "bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0, "traffic": measured_qem_traffic(),
                     "algorithmic_bytes_per_run": algo, "eval_ms_per_run": eval_ms,
                     "edges_evaluated_per_run": int(st[:, 0].sum())},
        "paper_context_s": 0.45,
    }
    if not args.no_cpu_baseline:
        # the oracle's round schedule on the same mesh, cut after as many rounds
        # as fit in about cpu_seconds (the first rounds are the largest)
        import oracle
        cores = 1
        n_rounds, dt, done = 1, 0.0, None
        while True:
            t1 = time.perf_counter()
            o = oracle.qem_simplify(V, F, target, method="rounds", max_rounds=n_rounds)
            dt = time.perf_counter() - t1
            done = F.shape[0] - o.F.shape[0]
            if dt >= 0.5 * args.cpu_seconds or o.rounds < n_rounds:
                break
            n_rounds = max(n_rounds + 1, int(n_rounds * args.cpu_seconds / max(dt, 1e-3)))
        out_json["cpu_baseline"] = {"value": done / dt, "unit": "faces/s", "cores": cores, "cpu": cpu_model(), "kind": "oracle",
                                    "sample": f"the oracle's first {o.rounds} rounds of the same workload "
                                              f"({F.shape[0]} -> {o.F.shape[0]} faces), {dt:.1f} s"}
    return out_json


def make_batch(n_assets, log):
    """The uneven batch's inputs, generated in a process pool (before this
    process touches the GPU)."""
    from synth import make_batch_assets
    t0 = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1))
    assets = make_batch_assets(n_assets, workers=workers)
    log(f"[bench] batch: {n_assets} assets generated in {time.perf_counter() - t0:.1f} s")
    return assets


def bench_batch(B, assets, steps, warmup, trav, log):
    """Uneven assets: forward + backward of the whole batch, recorded into one
    graph, against the same work as sequential per-asset plain calls."""
    import numpy as np
    import torch
    n_assets = len(assets)
    dev = torch.device("cuda:0")
    ins = [(*B.to_device(a, dev), a.res, a.max_dist) for a in assets]
    rng = np.random.default_rng(99)
    grads = [torch.from_numpy(rng.normal(size=(a.res, a.res, 3)).astype(np.float32)).to(dev) for a in assets]
    batch = B.BakeBatch(ins, save=True, **trav)
    for g, src in zip(batch.grad_maps, grads):
        g.copy_(src)
    tune = B.autotune(batch, reps=1)
    log(f"[bench] batch autotune: block {tune['block']} stack {tune['stack']} mode {tune['mode']}")
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    rays = int(sum(batch.ray_counts()))

    # sequential plain calls (each with its own BVH build), one shared workspace
    seq_opts = dict(trav_block=tune["block"], trav_stack=tune["stack"], trav_mode=tune["mode"])
    ws_bytes = max(B.workspace_size(x[0].shape[0], x[1].shape[0], x[3].shape[0], x[4].shape[0], x[6],
                                    B.make_options(save=True)) for x in ins)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    outs = [(torch.empty_like(batch.maps[i]), torch.empty_like(batch.hits[i]),
             torch.empty_like(batch.grad_lo_V[i]), torch.empty_like(batch.grad_hi_N[i]))
            for i in range(n_assets)]

    def seq_step():
        for i, x in enumerate(ins):
            om, oh, glo, ghi = outs[i]
            r = B.bake_normals(*x[:6], x[6], x[7], save=True, workspace=ws, out_map=om, out_hit=oh, **seq_opts)
            B.bake_normals_backward(r, x[:6], grads[i], out_lo=glo, out_hi=ghi)

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / k

    # the phases below are separated by idle gaps of 50 ms, so a kernel trace
    # of this run can be cut into them (outside every timed region)
    torch.cuda.synchronize()
    time.sleep(0.05)
    seq_ms = timed(seq_step, steps)
    time.sleep(0.05)
    # the sequential results equal the batch's, bitwise
    same = all(torch.equal(outs[i][0].view(torch.int32), batch.maps[i].view(torch.int32))
               and torch.equal(outs[i][1], batch.hits[i])
               and torch.equal(outs[i][2].view(torch.int32), batch.grad_lo_V[i].view(torch.int32))
               and torch.equal(outs[i][3].view(torch.int32), batch.grad_hi_N[i].view(torch.int32))
               for i in range(n_assets))

    def eager():
        batch.forward()
        batch.backward()

    eager_ms = timed(eager, steps)
    time.sleep(0.05)
    graph = batch.capture()
    torch.cuda.synchronize()
    time.sleep(0.05)
    graph_ms = timed(graph.replay, steps)
    log(f"[bench] batch: sequential {seq_ms:.2f} ms, batched eager {eager_ms:.2f} ms, graph {graph_ms:.2f} ms")
    return {"assets": n_assets, "hi_tris": int(sum(a.hi_F.shape[0] for a in assets)),
            "texels": int(sum(a.res * a.res for a in assets)), "rays": rays,
            "step": "forward (save) + backward from a fixed dL/dmap per asset",
            "sequential_ms": seq_ms, "batched_eager_ms": eager_ms, "batched_graph_ms": graph_ms,
            "speedup_graph_vs_sequential": seq_ms / graph_ms,
            "rays_per_s_graph": rays / (graph_ms / 1e3), "rays_per_s_sequential": rays / (seq_ms / 1e3),
            "bitwise_equal_to_sequential": bool(same),
            "tuned": {k: tune[k] for k in ("block", "stack", "mode")}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trav-block", type=int, default=0)
    ap.add_argument("--trav-stack", type=int, default=0)
    ap.add_argument("--trav-mode", type=int, default=-1)
    ap.add_argument("--one-queue", action="store_true",
                    help="traversal items from one work queue instead of one per XCD")
    ap.add_argument("--config", type=int, default=2, choices=(1, 2, 3),
                    help="workload: 2 = the headline 1.3M -> 20k triangle bake (default); 1 = the small "
                         "ripple bake; 3 = the large 5.2M-triangle bake")
    ap.add_argument("--query", choices=("ray", "closest", "visibility", "viewmaps", "simplify"), default="ray",
                    help="correspondence query (closest: the paper's closest-point form, forward only); "
                         "visibility: the hidden-face pass instead of the bake; viewmaps: the "
                         "backprojection precompute")
    ap.add_argument("--batch-assets", type=int, default=0, metavar="N",
                    help="also measure an N-asset batch (64 = the uneven batch workload)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-only", action="store_true",
                    help="with --batch-assets: measure only the batch (no headline step, no oracle baseline)")
    ap.add_argument("--eager", action="store_true",
                    help="time plain per-step API calls only (default: also record the step into a HIP graph "
                         "and report the replayed step)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the bake runs on a single device here "
              "(forward shards by rays or assets with no exchange; the backward reduces the "
              "per-GPU gradients in a fixed rank order); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2605_26137_amd.bake as B
    from synth import make_config

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    batch_assets = make_batch(args.batch_assets, log) if args.batch_assets > 0 else None
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
    log(f"[bench] {B.version()} on {torch.cuda.get_device_name(0)}")
    if args.query == "visibility":
        print(json.dumps(bench_visibility(args, B, log)), flush=True)
        return
    if args.query == "simplify":
        print(json.dumps(bench_simplify(args, B, log)), flush=True)
        return
    if args.query == "viewmaps":
        print(json.dumps(bench_view_maps(args, B, log)), flush=True)
        return
    if args.batch_only and batch_assets:
        trav = dict(trav_block=args.trav_block, trav_stack=args.trav_stack, trav_mode=args.trav_mode,
                    one_queue=args.one_queue)
        print(json.dumps({"batch": bench_batch(B, batch_assets, args.batch_steps, 1, trav, log)}), flush=True)
        return
    asset = make_config(args.config)
    t = B.to_device(asset, dev)
    res, md = asset.res, asset.max_dist
    closest = args.query == "closest"
    if closest:  # the paper's distance filter: 1% of the high-poly bounding-box diagonal
        V = np.asarray(asset.hi_V, np.float64)
        md = 0.01 * float(np.linalg.norm(V.max(0) - V.min(0)))
    trav = dict(trav_block=args.trav_block, trav_stack=args.trav_stack, trav_mode=args.trav_mode,
                query=args.query, one_queue=args.one_queue)
    # loss target: the map baked (by this library, untimed) from a second noise seed
    tgt_asset = make_config(args.config, seed=1)
    target = B.bake_normals(*B.to_device(tgt_asset, dev), res, md).map.clone()
    first = B.bake_normals(*t, res, md, save=not closest, **trav)
    ws, out_map, out_hit = first.workspace, first.map, first.hit
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gmap = torch.empty_like(out_map)
    scratch = torch.empty(4 * ((out_map.numel() + 255) // 256 + 1), dtype=torch.uint8, device=dev)
    glo = torch.empty_like(t[3])
    ghi = torch.empty_like(t[2])
    torch.cuda.synchronize()
    rays = first.ray_count()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]

    def step(timing, k=None):
        r = B.bake_normals(*t, res, md, save=not closest, timing=timing, workspace=ws, out_map=out_map,
                           out_hit=out_hit, **trav)
        if k is not None:
            ev[2 * k].record()
        if not closest:  # the closest-point query is forward only
            B.sq_loss(out_map, target, out_loss=loss, out_grad=gmap, scratch=scratch)
            B.bake_normals_backward(r, t, gmap, out_lo=glo, out_hi=ghi)
        if k is not None:
            ev[2 * k + 1].record()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # timed region: whole steps back to back; stage events on the bake stream
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True, k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eager_ms = (t1 - t0) * 1e3 / args.steps
    graph_ms, graph_equal = None, None
    if not args.eager:
        # the same step recorded once into a HIP graph and replayed (no host
        # work per kernel); the replays must reproduce the eager outputs
        ref = [x.clone() for x in ((out_map, glo, ghi) if not closest else (out_map,))]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step(False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            step(False)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - tg) * 1e3 / args.steps
        got = (out_map, glo, ghi) if not closest else (out_map,)
        graph_equal = all(torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(ref, got))
        log(f"[bench] graph-replayed step: {graph_ms:.3f} ms (outputs equal to the eager step: {graph_equal})")
        assert graph_equal, "graph replay changed the results"
    ms_per_step = graph_ms if graph_ms is not None else eager_ms
    hist = B.stage_history(min(args.steps, 64))
    stage_ms = {name: float(np.mean(hist[:, k])) for k, name in enumerate(B.STAGES)}
    bwd_ms = float(np.mean([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)]))
    log(f"[bench] {args.steps} eager steps, {eager_ms:.3f} ms/step, stages {stage_ms}, loss+backward {bwd_ms:.3f} ms")

    # algorithmic op count of the traversal: one instrumented bake, untimed
    cnt = B.bake_normals(*t, res, md, count=True, workspace=ws, out_map=out_map, out_hit=out_hit, **trav)
    n_box, n_tri = cnt.test_counts()
    trips = cnt.wave_trips()
    if closest:
        ops = n_box * OPS_BOX_PT + n_tri * OPS_TRI_PT + rays * OPS_RAY
    else:
        ops = n_box * OPS_BOX + n_tri * OPS_TRI + rays * OPS_RAY
    trav_s = stage_ms["traverse"] / 1e3
    achieved = ops / trav_s / 1e12
    khash = source_hash("traverse.hip", "lbvh.hip", "internal.h")
    # the counters were taken on the headline workload with the default launch
    # configuration: another workload or configuration reports none
    headline = (args.config == 2 and not closest and args.trav_block == 0 and args.trav_stack == 0
                and args.trav_mode == -1)
    roof = {"kernel": "traverse_batch_kernel (" + ("closest-point query" if closest else "traversal") + " + encode)",
            "bound": "alu",
            "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(khash) if headline else None,
            "ops_per_launch": ops, "box_tests_per_ray": n_box / rays, "tri_tests_per_ray": n_tri / rays,
            # lanes of a wave that advance a ray in an average trip of its
            # traversal loop (one trip: an internal node, two box tests, or a leaf)
            "lane_utilisation": (n_box / 2 + n_tri) / (64 * trips) if trips else None,
            "wave_trips_per_ray_batch": trips / ((rays + 63) // 64),
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
        "config": {"workload": WORKLOADS[args.config] + (f", closest-point query (max_dist {md:.4f})" if closest else ""),
                   "rays": rays, "texels": res * res,
                   "hi_tris": int(asset.hi_F.shape[0]), "lo_tris": int(asset.lo_F.shape[0]),
                   "step": ("forward bake incl. BVH build (closest-point query: no backward)" if closest else
                            "forward bake incl. BVH build + squared-error loss + backward"),
                   "launch": ("the whole step recorded once into a HIP graph and replayed" if graph_ms is not None
                              else "plain API calls per step")},
        "fwd_bwd_ms": ms_per_step,
        "eager_ms_per_step": eager_ms,
        "graph_equal_to_eager": graph_equal,
        "fwd_ms": stage_ms["forward"],
        "loss_bwd_ms": bwd_ms,
        "fwd_rays_per_s": rays / (stage_ms["forward"] / 1e3),
        "stages_ms": stage_ms,
        "roofline": roof,
    }
    if batch_assets:
        out["batch"] = bench_batch(B, batch_assets, args.batch_steps, 1, trav, log)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(asset, args.cpu_seconds, md, args.query)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
