"""Benchmark: path vertices/s of the fluorescent path tracer on one MI355X.

Headline workload: the large highly scattering scene (five bimodal dye
spheres, sigma_s up to 1000/mm, in a diffuse box; 512x512 pinhole, 1024 spp
= 2^28 light paths, 301 bins, scatter cap 1e4), the largest single-GPU
configuration.  One step = one full forward render of that job (fpt_render:
every per-vertex stage of the walk plus the film splat), inputs resident on
the device.  Vertices are counted exactly by the device tallies.

The JSON line also carries the roofline of the render's two launches (the
transport kernel and the deferred-connection kernel): algorithmic FP32 FLOPs
per render, from the exact event tallies and a per-event FLOP table, divided
by the two launches' durations measured with HIP events on the render stream
(mean and median over the timed renders), against the MI355X FP32 vector
peak; beside it, labelled separately, the same renders' algorithmic ALU lane
operations against the vector issue rate; the CPU oracle timed on the host;
and the other forms (Cornell scene, plain slab, forward+adjoint, batched,
excitation scan, camera-side estimator) as extra fields.
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
OPAQUE = 32              # connection opaque in its own sphere: eye direction, sphere exit, test


# Algorithmic FP32 work per event (an FMA counts 2, a transcendental, compare
# or conversion 1): the per-vertex arithmetic the walk cannot avoid, whatever
# the implementation (no random-number generation, addressing or control).
FL_SOURCE = 19            # line choice, point on the quad, cosine-weighted direction
FL_COLLIDE_SPHERE = 45    # flight (log, scale), sphere exit distance, advance, event, new direction
FL_COLLIDE_PLANE = 30     # the same with a plane distance (slab, half-space, unbounded)
FL_EMIT = 23              # quantum-yield test, emission CDF search, emitted direction
FL_NONRAD = 1             # quantum-yield test
FL_SURFACE = 17           # reaching an interface, wall, the light or the open face
FL_REFLECT = 19           # wall or Fresnel reflection: hit plus a new direction
FL_CONN = 38              # camera connection: distance, projection, cosines, exp
FL_CONN_SPHERE = 20       # + one chord per sphere
FL_CONN_OPAQUE = 30       # a connection opaque inside the vertex's own sphere: direction
                          # to the eye and that sphere's exit distance (no image tests,
                          # other chords or exp: the kernel resolves it with these)


def flops_model(t, n_spheres, geometry):
    """Algorithmic FP32 FLOPs of one render from its event tallies."""
    collide = FL_COLLIDE_PLANE if geometry in ("slab", "halfspace", "infinite") else FL_COLLIDE_SPHERE
    return (FL_SOURCE * t["paths"]
            + collide * (t["scatters"] + t["dye_abs"] + t["exit_bg"])
            + FL_EMIT * t["emissions"] + FL_NONRAD * t["exit_nonrad"]
            + FL_SURFACE * (t["crossings"] + t["exit_wall"] + t["exit_light"] + t["exit_esc_r"]
                            + t["exit_esc_t"])
            + FL_REFLECT * t["wall_reflect"]
            + (FL_CONN + FL_CONN_SPHERE * n_spheres) * (t["splat_hit"] + t["splat_miss"]
                                                        + t["splat_rr_kill"] - t.get("splat_opaque", 0))
            + FL_CONN_OPAQUE * t.get("splat_opaque", 0))


def ops_model(t, n_spheres, geometry, refractive=False):
    """Algorithmic ALU lane operations of one render from its event tallies."""
    open_geo = geometry in ("slab", "halfspace", "infinite", "sphere")
    medium = 14 if geometry in ("slab", "halfspace", "infinite") else 25   # boundary distance, event, direction
    surface = 4 if open_geo else 55 + 15 * n_spheres   # walls, light quad, sphere entries
    if open_geo and refractive:
        surface += 30   # boundary normal, Fresnel reflectance, mirror
    conn = 118 + 21 * n_spheres                          # camera connection and transmittance
    opaque = t.get("splat_opaque", 0)                    # resolved inside the own sphere
    return (START * t["paths"]
            + (STEP + medium) * (t["scatters"] + t["dye_abs"] + t["exit_bg"])
            + (STEP + surface) * (t["crossings"] + t["wall_reflect"] + t["exit_wall"] + t["exit_light"]
                                  + t["exit_esc_r"] + t["exit_esc_t"])
            + EMISSION * (t["emissions"] + t["exit_nonrad"])
            + conn * (t["splat_hit"] + t["splat_miss"] + t["splat_rr_kill"] - opaque)
            + OPAQUE * opaque)


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


def time_renders(sc, run, steps, warmup, film, camera=False, each=False):
    """Wall time per render over `steps` renders, and the mean durations of
    its transport and deferred-connection launches from the HIP events the
    library records around them on the render stream in the same renders
    (with each=True also the per-render launch durations)."""
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
    if each:
        t, d = sc.timing_each()
        sc.set_timing(False)
        assert len(t) == steps
        return wall / steps * 1e3, float(t.mean()), float(d.mean()), t + d
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
    ms, t_ms, d_ms, each = time_renders(sc, run, steps, warmup, film, each=True)
    geo = scene["geometry"]["kind"]
    nsph = len(scene["geometry"].get("spheres", [])) if geo == "box" else 0
    ops = ops_model(tal, nsph, geo, refractive=scene["media"][scene["geometry"].get("medium", 0)].get("ior", 1.0) != 1.0)
    flops = flops_model(tal, nsph, geo)
    sc.close()
    return {"vertices": tal["vertices"], "ms_per_step": ms, "transport_ms": t_ms, "deferred_ms": d_ms,
            "kernel_ms": t_ms + d_ms, "kernel_ms_median": float(sorted(each)[len(each) // 2]),
            "vertices_per_s": tal["vertices"] / (ms / 1e3), "ops": ops, "flops": flops,
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
    workload: the first paths of the same job, in chunks accumulated into one
    film, until about target_s of rendering (a job that takes less is rendered
    whole, repeatedly)."""
    import numpy as np
    import oracle
    film = np.zeros(oracle.film_shape(scene, max(1, run.get("parity_batches", 1))))
    chunk = min(run["path_count"], 1 << 14)
    done = verts = 0
    dt = 0.0
    while dt < target_s:
        begin = done % run["path_count"]
        n = min(chunk, run["path_count"] - begin)
        t0 = time.perf_counter()
        o = oracle.render(scene, dict(run, path_begin=run["path_begin"] + begin, path_count=n),
                          film_out=film)
        dt += time.perf_counter() - t0
        verts += int(o["tallies"][1])
        done += n
    return {"value": verts / dt, "unit": "path vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"first {min(done, run['path_count'])} of {run['total_paths']} light paths of "
                      f"the same job ({done} paths rendered, {verts} vertices, {dt:.1f} s, fp64, "
                      f"1 thread)"}


def _oracle_worker(task):
    """One host process of the all-cores oracle figure: renders consecutive
    chunks of its own path range into one film (from its start again once
    done) until its time budget is spent; returns vertices, paths and its
    busy time."""
    scene, run, begin, count, budget = task
    import numpy as np
    import oracle
    film = np.zeros(oracle.film_shape(scene, max(1, run.get("parity_batches", 1))))
    chunk = min(count, 1 << 14)
    t0 = time.perf_counter()
    verts = done = 0
    while time.perf_counter() - t0 < budget:
        k = done % count
        n = min(chunk, count - k)
        o = oracle.render(scene, dict(run, path_begin=begin + k, path_count=n), film_out=film)
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
                      f"(in chunks of up to 2^14, until ~{budget_s:.0f} s): {paths} paths, "
                      f"{verts} vertices, fp64"}


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


HEADLINE_TUNE = "large-512-1024spp"

# main kernel(s) of each profiled workload (name prefixes in rocprofv3's output)
PROFILED_KERNELS = {
    "cornell": ("void fpt::k_transport<4, 0,",), "large": ("void fpt::k_transport<4, 0,",),
    "slab": ("void fpt::k_transport<0, 0,",), "batched": ("void fpt::k_batch<",),
    "camera": ("void fpt::k_camera<",),
    "adjoint": ("void fpt::k_transport<4, 0,", "void fpt::k_transport<4, 1,"),
}


def record_counters(workload, csv_paths):
    """Writes profiles/traffic.json's entry for `workload` from rocprofv3
    counter-collection CSVs of `bench.py --profile <workload>` runs (one pass
    per counter set): FETCH_SIZE / WRITE_SIZE per dispatch of the workload's
    kernel(s) and of k_splat_jobs, scaled by what the same counters read for
    the run's 256 MiB device copy, and SQ_INSTS_VALU_FLOPS_FP32 (wave
    instructions x 64 lanes, FMA = 2).  The entry is keyed by the kernel
    source hash, so it is ignored once the kernels change."""
    import collections
    import csv
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in csv_paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                if name.startswith("__amd_rocclr_copyBuffer"):
                    key = "copy"
                elif name.startswith("fpt::k_splat_jobs"):
                    key = "deferred"
                elif any(name.startswith(k) for k in PROFILED_KERNELS[workload]):
                    key = "main"
                else:
                    continue
                per[key][(r["Counter_Name"], r["Dispatch_Id"])].append(float(r["Counter_Value"]))

    def mean(key, counter):
        v = [sum(x) for (c, _), x in per[key].items() if c == counter]
        return sum(v) / len(v) if v else None

    def largest(key, counter):  # the calibration copy (other small copies may run too)
        v = [sum(x) for (c, _), x in per[key].items() if c == counter]
        return max(v) if v else None

    launches = len(PROFILED_KERNELS[workload])  # kernels per step
    entry = {}
    copy_kib = COPY_BYTES / 1024.0
    f_copy, w_copy = largest("copy", "FETCH_SIZE"), largest("copy", "WRITE_SIZE")
    f_main, w_main = mean("main", "FETCH_SIZE"), mean("main", "WRITE_SIZE")
    if None not in (f_copy, w_copy, f_main, w_main):
        ff, wf_ = copy_kib / f_copy, copy_kib / w_copy
        f_def, w_def = mean("deferred", "FETCH_SIZE") or 0.0, mean("deferred", "WRITE_SIZE") or 0.0
        tb = (f_main * ff + w_main * wf_) * 1024.0 * launches
        db = (f_def * ff + w_def * wf_) * 1024.0
        entry.update({"bytes_per_launch": tb + db, "transport_bytes": tb, "deferred_bytes": db,
                      "fetch_kib_raw": f_main, "write_kib_raw": w_main,
                      "deferred_fetch_kib_raw": f_def, "deferred_write_kib_raw": w_def,
                      "fetch_factor": ff, "write_factor": wf_})
    fl = mean("main", "SQ_INSTS_VALU_FLOPS_FP32")
    if fl is not None:
        entry["fp32_flops_per_launch"] = fl * 64.0 * launches
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    if rec.get("kernel_source") != kernel_source_hash():
        rec = {"kernel_source": kernel_source_hash(), "copy_bytes": COPY_BYTES, "workloads": {}}
    rec["workloads"][workload] = entry
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps({workload: entry}), flush=True)


def form_summary(f, workload):
    """The per-form fields of a forward render: throughput, the algorithmic
    FP32 rate against the FP32 peak, the ALU issue fraction (lane-operation
    model) and, while the recorded counters match the kernel source, HBM
    bytes per second and the issued FP32 fraction."""
    out = {k: f[k] for k in ("vertices", "ms_per_step", "vertices_per_s", "kernel_ms",
                             "kernel_ms_median")}
    out["fp32_algorithmic_frac"] = f["flops"] / (f["kernel_ms"] / 1e3) / 1e12 / FP32_PEAK_TFLOPS
    out["alu_frac"] = alu_frac(f)
    hbm_rate(out, workload, f["kernel_ms"])
    fp32_rate(out, workload, f["kernel_ms"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline render (for profiler runs)")
    ap.add_argument("--profile", choices=["cornell", "large", "slab", "batched", "adjoint",
                                          "camera"],
                    help="profiler run: one 256 MiB device copy (traffic calibration) and "
                         "--steps renders of the named workload, nothing else")
    ap.add_argument("--record-counters", nargs="+", metavar=("WORKLOAD", "CSV"),
                    help="write profiles/traffic.json's entry for WORKLOAD from the rocprofv3 "
                         "counter CSVs of its --profile runs (no GPU work)")
    args = ap.parse_args()
    if args.record_counters:
        record_counters(args.record_counters[0], args.record_counters[1:])
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)
    import workloads
    all_cores = None
    if not (args.profile or args.only_headline or args.no_cpu_baseline):
        # host processes start before anything touches the GPU
        all_cores = cpu_all_cores(*workloads.large_config())
    import torch
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", 0)))
    if args.profile:
        profile_run(args.profile, args.steps)
        return
    scene, run = workloads.large_config()
    head = forward_form(scene, run, args.steps, args.warmup, tune_name=HEADLINE_TUNE)
    if args.only_headline:
        print(json.dumps({"headline": {k: v for k, v in head.items() if k != "tallies"}},
                         default=float), flush=True)
        return
    value = head["vertices_per_s"]
    flop_rate = head["flops"] / (head["kernel_ms"] / 1e3) / 1e12
    ops_rate = head["ops"] / (head["kernel_ms"] / 1e3) / 1e12
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
        "config": {"workload": "large highly scattering scene: box, 5 bimodal Gaussian dye spheres "
                               "(sigma_s 200-1000/mm), 512x512 pinhole, 1024 spp (2^28 light "
                               "paths), 301 bins, scatter cap 1e4, fwd",
                   "paths": run["path_count"], "vertices_per_step": head["vertices"],
                   "launch": head["tune"]},
        "roofline": {"bound": "alu", "achieved": flop_rate, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flop_rate / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic("large"),
                     "work": "algorithmic FP32 FLOPs per render from the event tallies x the "
                             "per-event FLOP table (FMA = 2)",
                     "kernel": "fpt::k_transport<BOX, FWD> + fpt::k_splat_jobs",
                     "kernel_ms": head["kernel_ms"], "kernel_ms_median": head["kernel_ms_median"],
                     "transport_ms": head["transport_ms"], "deferred_ms": head["deferred_ms"],
                     "flops_per_launch": head["flops"]},
        "alu_issue": {"achieved": ops_rate, "peak": ALU_PEAK_TOPS, "unit": "T lane-ops/s",
                      "frac": ops_rate / ALU_PEAK_TOPS, "ops_per_launch": head["ops"],
                      "work": "algorithmic 32-bit lane operations per render (Philox, flight, "
                              "geometry, connections) from the event tallies x the per-event "
                              "operation table, against 256 CUs x 64 lanes x 2.4 GHz"},
    }
    fp32_rate(line["roofline"], "large", head["kernel_ms"])
    extra = {}
    if not args.no_extra:
        s2, r2 = workloads.cornell_config()
        co = forward_form(s2, r2, max(20, args.steps * 5), 5, tune_name="cornell-128-64spp")
        extra["fwd_cornell"] = form_summary(co, "cornell")
        if not args.no_cpu_baseline:
            extra["fwd_cornell"]["cpu_oracle"] = oracle_sample(s2, r2)
        s1, r1 = workloads.slab_config()
        r1 = dict(r1, path_count=1 << 22, total_paths=1 << 22)
        sl = forward_form(s1, r1, max(10, args.steps * 2), 2, tune_name="slab-2^22")
        extra["fwd_slab_2^22"] = form_summary(sl, "slab")
        if not args.no_cpu_baseline:
            extra["fwd_slab_2^22"]["cpu_oracle"] = oracle_sample(s1, r1)
        # the same slab behind a water boundary (n = 1.33): Fresnel reflection
        # and total internal reflection at both faces
        s1w = workloads.deepcopy(s1)
        s1w["media"][0]["ior"] = 1.33
        sw = forward_form(s1w, r1, max(10, args.steps * 2), 2, tune_name="slab-2^22")
        extra["fwd_slab_water_2^22"] = form_summary(sw, "slab_water")
        extra["fwd_slab_water_2^22"]["boundary_reflections"] = sw["tallies"]["wall_reflect"]
        try:
            extra["fwd_adjoint"] = adjoint_form(max(3, args.steps), 1)
            fp32_rate(extra["fwd_adjoint"], "adjoint", extra["fwd_adjoint"]["ms_per_step"])
            if not args.no_cpu_baseline:
                sa, ra = workloads.adjoint_config()[:2]
                extra["fwd_adjoint"]["cpu_oracle"] = oracle_sample(sa, ra, grad=True)
        except Exception as e:  # reported, not hidden
            extra["fwd_adjoint"] = {"error": str(e)}
        b = batched_form(max(3, args.steps), 1)
        if b is not None:
            extra["batched"] = b
            if not args.no_cpu_baseline:
                b["cpu_oracle"] = batch_oracle_sample(*workloads.batch_config())
            hbm_rate(b, "batched", b["ms_per_step"])
            fp32_rate(b, "batched", b["ms_per_step"])
        extra["excitation_scan"] = sweep_form(max(3, args.steps * 2), 1)
        extra["camera_side"] = camera_form(max(3, args.steps * 2), 1, cpu=not args.no_cpu_baseline)
        hbm_rate(extra["camera_side"], "camera", extra["camera_side"]["kernel_ms"])
        fp32_rate(extra["camera_side"], "camera", extra["camera_side"]["kernel_ms"])
    line["forms"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, run)
        line["cpu_baseline_all_cores"] = all_cores
    print(json.dumps(line, default=float), flush=True)


if __name__ == "__main__":
    main()
