"""Benchmark: path vertices/s of the fluorescent path tracer on one MI355X.

Headline workload: the Cornell-style scene (three dye spheres in a diffuse
box, 128x128 pinhole, 64 spp = 2^20 light paths, 101 bins).  One step = one
full forward render of that job (fpt_render: every per-vertex stage of the
walk plus the film splat), inputs resident on the device.  Vertices are
counted exactly by the device tallies.

The JSON line also carries the roofline of the render's two launches (the
transport kernel and the deferred-connection kernel): algorithmic ALU lane
operations per render, from the exact event tallies and a per-event
operation table, divided by the two launches' mean durations measured with
HIP events on the render stream, against the MI355X vector issue rate; the
CPU oracle timed on the host; and the other forms (large scene, plain slab,
forward+adjoint, batched) as extra fields.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X vector ALU issue rate: 256 CUs x 64 lanes x 2.4 GHz, one 32-bit lane
# operation per lane per clock (an FMA is one operation; packed FP32 is not
# used by these kernels)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Lane operations per event (FMA, add, compare, logic, conversion and
# transcendental = 1; a 32x32->64 product = 2).
PHILOX = 92            # ten rounds of 2 products + 4 xors, four 24-bit conversions
STEP = PHILOX + 6      # free flight: log, scale, position update
START = 2 * PHILOX + 25  # light vertex: line choice, point and direction on the quad
EMISSION = PHILOX + 17   # quantum-yield test, emission CDF inversion
CAM_START = PHILOX + 90  # camera-side path: pixel of the path index, pixel sample, eye ray, box entry


def ops_model(t, n_spheres, geometry, refractive=False):
    """Algorithmic ALU lane operations of one render from its event tallies."""
    open_geo = geometry in ("slab", "halfspace", "infinite", "sphere")
    medium = 14 if geometry in ("slab", "halfspace", "infinite") else 25   # boundary distance, event, direction
    surface = 4 if open_geo else 55 + 15 * n_spheres   # walls, light quad, sphere entries
    if open_geo and refractive:
        surface += 30   # boundary normal, Fresnel reflectance, mirror
    conn = 118 + 21 * n_spheres                          # camera connection and transmittance
    return (START * t["paths"]
            + (STEP + medium) * (t["scatters"] + t["dye_abs"] + t["exit_bg"])
            + (STEP + surface) * (t["crossings"] + t["wall_reflect"] + t["exit_wall"] + t["exit_light"]
                                  + t["exit_esc_r"] + t["exit_esc_t"])
            + EMISSION * (t["emissions"] + t["exit_nonrad"])
            + conn * (t["splat_hit"] + t["splat_miss"] + t["splat_rr_kill"]))


def camera_ops(t, n_spheres, n_lines):
    """Algorithmic ALU lane operations of one camera-side render (eq. 12
    estimator) from its event tallies: the forward walk's per-vertex costs,
    and per light connection a Philox call, the light point, distance and
    emitter cosine, one chord per sphere and one transmittance per line."""
    medium = 25
    surface = 55 + 15 * n_spheres
    conn = PHILOX + 29 + 22 * n_spheres + n_lines * (n_spheres + 5)
    return (CAM_START * t["paths"]
            + (STEP + medium) * (t["scatters"] + t["dye_abs"] + t["exit_bg"])
            + (STEP + surface) * (t["crossings"] + t["wall_reflect"] + t["exit_wall"] + t["exit_light"]
                                  + t["exit_esc_r"])
            + conn * (t["splat_hit"] + t["splat_miss"]))


def time_renders(sc, run, steps, warmup, film, camera=False):
    """Wall time per render over `steps` renders, and the mean durations of
    its transport and deferred-connection launches from the HIP events the
    library records around them on the render stream in the same renders."""
    import torch
    render = sc.render_camera if camera else sc.render
    for _ in range(warmup):
        render(run, film=film)
    torch.cuda.synchronize()
    sc.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        render(run, film=film)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n, t_ms, d_ms = sc.timing()
    sc.set_timing(False)
    assert n == steps
    return wall / steps * 1e3, t_ms, d_ms


def count_vertices(sc, run):
    import torch
    import paper_1706_03024_amd as fpt
    t = fpt.new_tallies()
    sc.render(run, tallies=t)
    torch.cuda.synchronize()
    return fpt.tallies_dict(t)


def forward_form(scene, run, steps, warmup, tune_name=None):
    import paper_1706_03024_amd as fpt
    from paper_1706_03024_amd import autotune
    sc = fpt.Scene(scene)
    tune = autotune.autotune(tune_name, scene=sc, run=run) if tune_name else None
    film = sc.new_film()
    tal = count_vertices(sc, run)
    ms, t_ms, d_ms = time_renders(sc, run, steps, warmup, film)
    geo = scene["geometry"]["kind"]
    nsph = len(scene["geometry"].get("spheres", [])) if geo == "box" else 0
    ops = ops_model(tal, nsph, geo, refractive=scene["media"][scene["geometry"].get("medium", 0)].get("ior", 1.0) != 1.0)
    sc.close()
    return {"vertices": tal["vertices"], "ms_per_step": ms, "transport_ms": t_ms, "deferred_ms": d_ms,
            "kernel_ms": t_ms + d_ms, "vertices_per_s": tal["vertices"] / (ms / 1e3), "ops": ops,
            "tallies": tal, "tune": tune}


def camera_form(steps, warmup, cpu=False):
    """The camera-side estimator (eq. 12, sec. 4.1) on the Cornell scene:
    128x128 pixels x 101 emission bins x 8 samples, paths from the eye with a
    light connection at every collision in a dye sphere."""
    import torch
    import paper_1706_03024_amd as fpt
    import workloads
    scene, run = workloads.camera_config()
    sc = fpt.Scene(scene)
    film = sc.new_film()
    t = fpt.new_tallies()
    sc.render_camera(run, tallies=t)
    torch.cuda.synchronize()
    tal = fpt.tallies_dict(t)
    ms, k_ms, _ = time_renders(sc, run, steps, warmup, film, camera=True)
    sc.close()
    ops = camera_ops(tal, len(scene["geometry"]["spheres"]), len(scene["light"]["lines"]))
    out = {"vertices": tal["vertices"], "paths": run["path_count"], "ms_per_step": ms,
           "kernel_ms": k_ms, "vertices_per_s": tal["vertices"] / (ms / 1e3),
           "light_connections": tal["splat_hit"] + tal["splat_miss"],
           "alu_frac": ops / (k_ms / 1e3) / 1e12 / ALU_PEAK_TOPS}
    if cpu:
        out["cpu_oracle"] = camera_cpu_sample(scene, run)
    return out


def camera_cpu_sample(scene, run, chunks=256, chunk=8192):
    """The camera-side oracle (1 thread, fp64) on a bounded sample of the
    same job: `chunks` runs of `chunk` consecutive paths spread evenly over the
    path index range (pixels top to bottom, all samples)."""
    import oracle
    n = run["path_count"]
    verts, dt = 0, 0.0
    for i in range(chunks):
        begin = (n - chunk) * i // max(1, chunks - 1)
        t0 = time.perf_counter()
        o = oracle.render_camera(scene, dict(run, path_begin=begin, path_count=chunk), film=False)
        dt += time.perf_counter() - t0
        verts += int(o["tallies"][1])
    return {"value": verts / dt, "unit": "path vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"{chunks} ranges of {chunk} paths spread over the {n}-path job "
                      f"({verts} vertices, {dt:.1f} s, fp64, 1 thread)"}


def oracle_sample(scene, run, target_s=2.0, grad=False):
    """The oracle (1 thread, fp64) on the first paths of a job, doubled until
    one render takes about target_s/2 (path ids are independent, so the first
    ones are a fair sample); with grad, the path-replay gradient too."""
    import numpy as np
    import oracle
    n, dt, verts = 1024, 0.0, 0
    g = np.ones(oracle.film_shape(scene, run.get("parity_batches", 1))) if grad else None
    while True:
        t0 = time.perf_counter()
        o = oracle.render(scene, dict(run, path_count=n), film=grad, grad_film=g)
        dt = time.perf_counter() - t0
        verts = int(o["tallies"][1])
        if dt >= target_s / 2 or n >= run["path_count"]:
            break
        n = min(run["path_count"], 2 * n)
    return {"value": verts / dt, "unit": "path vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {run['path_count']} paths of the same job ({verts} vertices, "
                      f"{dt:.1f} s, fp64, 1 thread{', with the gradient' if grad else ''})"}


def batch_oracle_sample(scenes, runs, every=16, paths=2048):
    """The oracle (1 thread, fp64) on every `every`-th instance of a batch, the
    first `paths` paths of each."""
    import oracle
    verts, dt, k = 0, 0.0, 0
    for s, r in list(zip(scenes, runs))[::every]:
        n = min(paths, r["path_count"])
        t0 = time.perf_counter()
        o = oracle.render(s, dict(r, path_count=n), film=False)
        dt += time.perf_counter() - t0
        verts += int(o["tallies"][1])
        k += 1
    return {"value": verts / dt, "unit": "path vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} of {len(scenes)} instances (every {every}th), the first {paths} paths of each "
                      f"({verts} vertices, {dt:.1f} s, fp64, 1 thread)"}


def alu_frac(form):
    return form["ops"] / (form["kernel_ms"] / 1e3) / 1e12 / ALU_PEAK_TOPS


def adjoint_form(steps, warmup):
    """Forward + path-replay adjoint on the 256x256, 256 spp Cornell job:
    forward vertices / (t_fwd + t_adj)."""
    import torch
    import paper_1706_03024_amd as fpt
    import workloads
    scene, run, target, trun = workloads.adjoint_config()
    sc = fpt.Scene(scene)
    film = sc.new_film()
    tal = count_vertices(sc, run)
    g = torch.ones_like(film)
    grad = torch.zeros(sc.n_params, device="cuda")
    for _ in range(warmup):
        sc.render(run, film=film)
        sc.render_adjoint(run, g, grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sc.render(run, film=film)
        sc.render_adjoint(run, g, grad)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    sc.close()
    # the adjoint replays the forward walk event for event (same random
    # numbers, same connections): both launches do at least the forward's
    # operations; the gradient arithmetic on top of them is not counted
    ops = 2 * ops_model(tal, len(scene["geometry"]["spheres"]), "box")
    return {"vertices": tal["vertices"], "ms_per_step": ms,
            "vertices_per_s": tal["vertices"] / (ms / 1e3),
            "alu_frac": ops / (ms / 1e3) / 1e12 / ALU_PEAK_TOPS,
            "alu_frac_counts": "the replayed walk in both launches; gradient arithmetic not counted"}


def batched_form(steps, warmup):
    import torch
    import paper_1706_03024_amd as fpt
    import workloads
    if not hasattr(fpt, "Batch"):
        return None
    from paper_1706_03024_amd import autotune
    scenes, runs = workloads.batch_config()
    b = fpt.Batch(scenes, runs)
    tune = autotune.autotune("batched-1024", batch=b)
    b.close()
    b = fpt.Batch(scenes, runs, tune={k: v for k, v in tune.items() if k != "ms"})
    films = b.new_films()
    ops, tal = batch_ops(b, scenes)
    for _ in range(warmup):
        b.render(films)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.render(films)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    b.close()
    return {"vertices": tal, "ms_per_step": ms, "vertices_per_s": tal / (ms / 1e3),
            "instances": len(scenes), "tune": tune,
            "alu_frac": ops / (ms / 1e3) / 1e12 / ALU_PEAK_TOPS}


def batch_ops(b, scenes):
    """Lane operations and vertices of one batched render, from every
    instance's own event tallies and geometry."""
    import torch
    import paper_1706_03024_amd as fpt
    t = fpt.new_tallies(len(scenes))
    b.render(b.new_films(), t)
    torch.cuda.synchronize()
    ops = verts = 0
    for i, s in enumerate(scenes):
        ti = fpt.tallies_dict(t[i])
        geo = s["geometry"]
        refr = s["media"][geo.get("medium", 0)].get("ior", 1.0) != 1.0
        ops += ops_model(ti, 0, geo["kind"], refractive=refr)
        verts += ti["vertices"]
    return ops, verts


def sweep_form(steps, warmup):
    """The excitation scan of the paper's experiments: 81 dye-slab instances
    (300-700 nm, 2^18 paths each) in one batched launch."""
    import torch
    import paper_1706_03024_amd as fpt
    import workloads
    from paper_1706_03024_amd import autotune
    scenes, runs = workloads.excitation_scan()
    b = fpt.Batch(scenes, runs)
    tune = autotune.autotune("excitation-scan-81", batch=b)
    b.close()
    b = fpt.Batch(scenes, runs, tune={k: v for k, v in tune.items() if k != "ms"})
    films = b.new_films()
    ops, tal = batch_ops(b, scenes)
    for _ in range(warmup):
        b.render(films)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.render(films)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    b.close()
    return {"vertices": tal, "ms_per_step": ms, "vertices_per_s": tal / (ms / 1e3),
            "instances": len(scenes), "tune": tune,
            "alu_frac": ops / (ms / 1e3) / 1e12 / ALU_PEAK_TOPS}


def cpu_baseline(scene, run, target_s=12.0):
    """The oracle as it stands (single thread, fp64) on a bounded sample of the
    workload: the first paths of the same job, sized to roughly target_s; a
    job that takes less is rendered whole, repeatedly, until target_s."""
    import oracle
    n = 1 << 14
    t0 = time.perf_counter()
    o = oracle.render(scene, dict(run, path_count=n))
    dt = time.perf_counter() - t0
    n2 = int(min(run["path_count"], max(n, n * target_s / max(dt, 1e-3))))
    reps, verts, dt = 0, 0, 0.0
    while dt < 0.8 * target_s or reps == 0:
        t0 = time.perf_counter()
        o = oracle.render(scene, dict(run, path_count=n2))
        dt += time.perf_counter() - t0
        verts += int(o["tallies"][1])
        reps += 1
    return {"value": verts / dt, "unit": "path vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n2} of {run['total_paths']} light paths of the same job, {reps} time(s) "
                      f"({verts} vertices, {dt:.1f} s, fp64, 1 thread)"}


def _oracle_worker(task):
    """One host process of the all-cores oracle figure: renders consecutive
    chunks of its own path range (from its start again once done) until its
    time budget is spent; returns vertices, paths and its busy time."""
    scene, run, begin, count, budget = task
    import oracle
    t0 = time.perf_counter()
    verts = done = 0
    while time.perf_counter() - t0 < budget:
        k = done % count
        n = count - k   # whole ranges: each call also allocates the film
        o = oracle.render(scene, dict(run, path_begin=begin + k, path_count=n))
        verts += int(o["tallies"][1])
        done += n
    return verts, done, time.perf_counter() - t0


def cpu_all_cores(scene, run, budget_s=8.0):
    """The oracle on every host core the job may use (at most 16): one fresh
    process per core on disjoint path ranges of the same job, aggregate
    vertices per second of wall time.  Run before the GPU is touched."""
    import multiprocessing as mp
    P = max(1, min(16, os.cpu_count() or 1))
    span = run["path_count"] // P
    ctx = mp.get_context("spawn")
    with ctx.Pool(P) as pool:
        res = pool.map(_oracle_worker, [(scene, run, i * span, span, budget_s) for i in range(P)])
    verts = sum(r[0] for r in res)
    paths = sum(r[1] for r in res)
    # the processes run concurrently: the aggregate rate is the sum of theirs
    rate = sum(r[0] / r[2] for r in res)
    return {"value": rate, "unit": "path vertices/s", "cores": P, "kind": "oracle",
            "sample": f"{P} concurrent processes, each on its own 1/{P} of the same job's light paths "
                      f"(repeated until ~{budget_s:.0f} s): {paths} paths, {verts} vertices, fp64"}


COPY_BYTES = 256 << 20
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("fpt_kernels.hip", "fpt_internal.h"):
        with open(os.path.join(ROOT, "paper_1706_03024_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the transport kernel from the recorded
    FETCH_SIZE / WRITE_SIZE counter runs, or None when the kernel source has
    changed since they were taken."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source") != kernel_source_hash():
        return None
    w = rec.get("workloads", {}).get(workload)
    return None if w is None else w.get("bytes_per_launch")


FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (packed FMA)


def measured_fp32(workload):
    """FP32 FLOPs issued per launch (per step for the forward+adjoint pair)
    from the recorded SQ_INSTS_VALU_FLOPS_FP32 counter runs (wave instructions,
    FMA = 2, x 64 lanes: every lane of an issued instruction is counted), or
    None when the kernel source has changed since they were taken."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source") != kernel_source_hash():
        return None
    w = rec.get("workloads", {}).get(workload)
    return None if w is None else w.get("fp32_flops_per_launch")


def fp32_rate(form, workload, ms):
    """Issued FP32 FLOP rate over the launch time and its fraction of the
    MI355X FP32 vector peak."""
    f = measured_fp32(workload)
    if f and ms > 0:
        form["fp32_tflops"] = f / (ms / 1e3) / 1e12
        form["fp32_frac"] = form["fp32_tflops"] / FP32_PEAK_TFLOPS


def hbm_rate(form, workload, ms):
    """HBM bytes per launch from the recorded counter runs (while the kernel
    source matches them) over the launch time, in GB/s; 8000 GB/s is the peak."""
    t = measured_traffic(workload)
    if t is not None and ms > 0:
        form["hbm_gb_per_s"] = t / (ms / 1e3) / 1e9


def profile_run(name, steps):
    """Kernels for a profiler: a plain device copy of COPY_BYTES (reads and
    writes that many bytes; calibrates FETCH_SIZE / WRITE_SIZE) and `steps`
    renders of one workload."""
    import torch
    import paper_1706_03024_amd as fpt
    import workloads
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    from paper_1706_03024_amd import autotune
    if name == "batched":
        scenes, runs = workloads.batch_config()
        bt = fpt.Batch(scenes, runs)
        tune = autotune.autotune("batched-1024", batch=bt, measure=False)
        print(f"launch shape: {tune} (device {autotune.device_tag()})", flush=True)
        if tune is not None:
            bt.close()
            bt = fpt.Batch(scenes, runs, tune={k: v for k, v in tune.items() if k != "ms"})
        films = bt.new_films()
        for _ in range(steps):
            bt.render(films)
        torch.cuda.synchronize()
        bt.close()
        print(f"profiled {steps} batched renders", flush=True)
        return
    scene, run = {"cornell": workloads.cornell_config, "large": workloads.large_config,
                  "slab": workloads.slab_config, "camera": workloads.camera_config,
                  "adjoint": lambda: workloads.adjoint_config()[:2]}[name]()
    if name == "slab":
        run = dict(run, path_count=1 << 22, total_paths=1 << 22)
    sc = fpt.Scene(scene)
    tune_name = {"cornell": "cornell-128-64spp", "slab": "slab-2^22", "large": "large-512-1024spp"}.get(name)
    if tune_name:
        print(f"launch shape: {autotune.autotune(tune_name, scene=sc, run=run, measure=False)} "
              f"(device {autotune.device_tag()})", flush=True)
    film = sc.new_film()
    g = torch.ones_like(film) if name == "adjoint" else None
    for _ in range(steps):
        if name == "camera":
            sc.render_camera(run, film=film)
            continue
        sc.render(run, film=film)
        if g is not None:
            sc.render_adjoint(run, g)
    torch.cuda.synchronize()
    sc.close()
    print(f"profiled {steps} {name} renders", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline render (for profiler runs)")
    ap.add_argument("--profile", choices=["cornell", "large", "slab", "batched", "adjoint",
                                          "camera"],
                    help="profiler run: one 256 MiB device copy (traffic calibration) and "
                         "--steps renders of the named workload, nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)
    import workloads
    all_cores = None
    if not (args.profile or args.only_headline or args.no_cpu_baseline):
        # host processes start before anything touches the GPU
        all_cores = cpu_all_cores(*workloads.cornell_config())
    import torch
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", 0)))
    if args.profile:
        profile_run(args.profile, args.steps)
        return
    scene, run = workloads.cornell_config()
    head = forward_form(scene, run, args.steps, args.warmup, tune_name="cornell-128-64spp")
    if args.only_headline:
        print(json.dumps({"headline": head}, default=float), flush=True)
        return
    value = head["vertices_per_s"]
    achieved = head["ops"] / (head["kernel_ms"] / 1e3) / 1e12
    line = {
        "metric": "path vertices/s on 1 MI355X (fwd, batched, fwd+adjoint) at <=3 s.e. vs oracle",
        "value": value,
        "unit": "path vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cornell box, 3 Gaussian dye spheres, 128x128 pinhole, 64 spp "
                               "(2^20 light paths), 101 bins, fwd",
                   "paths": run["path_count"], "vertices_per_step": head["vertices"],
                   "launch": head["tune"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                     "unit": "Tops/s", "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": measured_traffic("cornell"),
                     "kernel": "fpt::k_transport<BOX, FWD> + fpt::k_splat_jobs",
                     "kernel_ms": head["kernel_ms"], "transport_ms": head["transport_ms"],
                     "deferred_ms": head["deferred_ms"], "ops_per_launch": head["ops"]},
    }
    fp32_rate(line["roofline"], "cornell", head["kernel_ms"])
    extra = {}
    if not args.no_extra:
        s3, r3 = workloads.large_config()
        big = forward_form(s3, r3, max(2, args.steps // 25), 1, tune_name="large-512-1024spp")
        extra["fwd_large"] = {k: big[k] for k in ("vertices", "ms_per_step", "vertices_per_s")}
        if not args.no_cpu_baseline:
            extra["fwd_large"]["cpu_oracle"] = oracle_sample(s3, r3)
        extra["fwd_large"]["alu_frac"] = alu_frac(big)
        hbm_rate(extra["fwd_large"], "large", big["kernel_ms"])
        fp32_rate(extra["fwd_large"], "large", big["kernel_ms"])
        s1, r1 = workloads.slab_config()
        r1 = dict(r1, path_count=1 << 22, total_paths=1 << 22)
        sl = forward_form(s1, r1, max(5, args.steps // 5), 2, tune_name="slab-2^22")
        extra["fwd_slab_2^22"] = {k: sl[k] for k in ("vertices", "ms_per_step", "vertices_per_s")}
        if not args.no_cpu_baseline:
            extra["fwd_slab_2^22"]["cpu_oracle"] = oracle_sample(s1, r1)
        extra["fwd_slab_2^22"]["alu_frac"] = alu_frac(sl)
        hbm_rate(extra["fwd_slab_2^22"], "slab", sl["kernel_ms"])
        fp32_rate(extra["fwd_slab_2^22"], "slab", sl["kernel_ms"])
        # the same slab behind a water boundary (n = 1.33): Fresnel reflection
        # and total internal reflection at both faces
        s1w = workloads.deepcopy(s1)
        s1w["media"][0]["ior"] = 1.33
        sw = forward_form(s1w, r1, max(5, args.steps // 5), 2, tune_name="slab-2^22")
        extra["fwd_slab_water_2^22"] = {k: sw[k] for k in ("vertices", "ms_per_step", "vertices_per_s")}
        extra["fwd_slab_water_2^22"]["alu_frac"] = alu_frac(sw)
        extra["fwd_slab_water_2^22"]["boundary_reflections"] = sw["tallies"]["wall_reflect"]
        try:
            extra["fwd_adjoint"] = adjoint_form(max(3, args.steps // 10), 1)
            fp32_rate(extra["fwd_adjoint"], "adjoint", extra["fwd_adjoint"]["ms_per_step"])
            if not args.no_cpu_baseline:
                sa, ra = workloads.adjoint_config()[:2]
                extra["fwd_adjoint"]["cpu_oracle"] = oracle_sample(sa, ra, grad=True)
        except Exception as e:  # reported, not hidden
            extra["fwd_adjoint"] = {"error": str(e)}
        b = batched_form(max(3, args.steps // 10), 1)
        if b is not None:
            extra["batched"] = b
            if not args.no_cpu_baseline:
                b["cpu_oracle"] = batch_oracle_sample(*workloads.batch_config())
            hbm_rate(b, "batched", b["ms_per_step"])
            fp32_rate(b, "batched", b["ms_per_step"])
        extra["excitation_scan"] = sweep_form(max(3, args.steps // 5), 1)
        extra["camera_side"] = camera_form(max(3, args.steps // 5), 1, cpu=not args.no_cpu_baseline)
        hbm_rate(extra["camera_side"], "camera", extra["camera_side"]["kernel_ms"])
        fp32_rate(extra["camera_side"], "camera", extra["camera_side"]["kernel_ms"])
    line["forms"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, run)
        line["cpu_baseline_all_cores"] = all_cores
    print(json.dumps(line, default=float), flush=True)


if __name__ == "__main__":
    main()
