"""Benchmark of the synchronized tracer on one MI355X.

A step is one frame of the hot path on resident inputs: volumes of interest,
tile A-buffer build (project, count, scan, scatter, sort) and synchronized
tracing of every pixel, for the 1920x1080, 4096-primitive workload.  Flatten
(tree preprocessing, needed only when the tree structure changes) runs once
before timing and is reported separately, like the paper's preprocessing.

Prints ONE JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

# FP32 FLOPs per node evaluation (FMA = 2; add, sub, mul, min, max, sqrt,
# reciprocal = 1; compares, selects, abs/neg modifiers = 0), counted from the
# device formulas: sphere, box, capsule, operator on its sharp branch; the
# smooth branch of a compact operator adds SMOOTH_EXTRA.
FLOPS_PRIM = {"sphere": 10, "box": 34, "capsule": 24}
FLOPS_OP_SHARP = 1
SMOOTH_EXTRA = 20
PEAK_FP32 = 157.3e12     # MI355X FP32 vector, packed
PEAK_FP32_NONPACKED = 78.6e12

# FP32 FLOPs of one ray / volume-of-interest test in the binning's tile test
# (same counting rules; only the work that depends on the ray direction: the
# per-candidate terms are computed once per candidate), including the update
# of the interval (clamp, two depth products, min, max): sphere, box (three
# slabs), capsule (two end spheres and the cylinder).
FLOPS_TEST = {"sphere": 25, "box": 38, "capsule": 96}

# HBM traffic of a kernel, measured with rocprofv3 FETCH_SIZE and WRITE_SIZE
# counters and calibrated against a copy kernel of known size; it is reported
# only while the kernel's sources hash to what was measured.
TRAFFIC = {
    "trace": (ROOT / "profiles" / "trace_c3_traffic.md",
              ["trace.hip", "st_trace.h", "st_field.h", "st_internal.h", "st_prune.h", "st_common.h", "st_mlp.h"]),
    "tile_test": (ROOT / "profiles" / "tile_test_c3_traffic.md",
                  ["binning.hip", "st_internal.h", "st_prune.h", "st_voi.h", "st_common.h"]),
}


def source_hash(names) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update((ROOT / "paper_2304_09673_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """Bytes per launch of the kernel from its committed counter summary, or None."""
    path, sources = TRAFFIC[kernel]
    if not path.exists():
        return None
    kv = {}
    for line in path.read_text().splitlines():
        line = line.strip().lstrip("-* ")
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip().strip("`")] = v.strip().strip("`")
    if kv.get("source_sha256") != source_hash(sources):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calib_copy(mib: int, reps: int = 5):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": n * 4, "calib_copy_bytes_written": n * 4, "reps": reps}), flush=True)


def algorithmic_flops(stats) -> float:
    ne = stats["node_evals"]
    return (ne[0] * FLOPS_PRIM["sphere"] + ne[1] * FLOPS_PRIM["box"] + ne[2] * FLOPS_PRIM["capsule"]
            + ne[3] * FLOPS_OP_SHARP + stats.get("smooth_evals", 0) * SMOOTH_EXTRA)


def _oracle_rate(config: int, seed: int, n_rays: int, sample_seed: int):
    """Oracle Mrays/s on n_rays seeded random pixels of a workload's frame (this process's threads)."""
    import oracle
    import scenegen as sg
    oracle.build(force=False)
    sc = sg.by_config(config, seed=seed)
    osc = oracle.OracleScene(sc)
    rng = np.random.default_rng(sample_seed)
    px = rng.integers(0, sc.camera.width, n_rays) + 0.5
    py = rng.integers(0, sc.camera.height, n_rays) + 0.5
    t0 = time.perf_counter()
    _, _, flag, ev = osc.trace(sc.camera, px, py)
    dt = time.perf_counter() - t0
    return {"mrays_s": n_rays / dt / 1e6, "seconds": dt, "evals": int(ev.sum()), "threads": oracle.num_threads()}


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, config: int, seed: int, n_rays: int, n_rays_1core: int = 1024):
    """The oracle on the host's cores and, in a child process, on one core."""
    r = _oracle_rate(config, seed, n_rays, 1234)
    one = None
    env = dict(os.environ, OMP_NUM_THREADS="1")
    import subprocess
    code = (f"import sys, json; sys.path.insert(0, {str(ROOT)!r}); import bench; "
            f"print(json.dumps(bench._oracle_rate({config}, {seed}, {n_rays_1core}, 4321)))")
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        if res.returncode == 0:
            one = json.loads(res.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    out = {"value": r["mrays_s"], "unit": "Mrays/s", "cores": r["threads"], "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"{n_rays} seeded random pixels of the same {sc.camera.width}x{sc.camera.height} frame, "
                     f"full-tree FP64 first-root tracing (no pruning, no A-buffer); {r['seconds']:.1f} s, "
                     f"{r['evals']} full-tree evaluations"}
    if one is not None:
        out["single_core"] = {"value": one["mrays_s"], "unit": "Mrays/s", "cores": one["threads"],
                              "sample": f"{n_rays_1core} other seeded random pixels of the same frame; "
                                        f"{one['seconds']:.1f} s"}
    return out


def bench_batch(args):
    """The 64-scene batch: one graph launch per frame (replayed A-buffer builds
    of every scene + persistent trace kernels over a shared job queue)."""
    import torch
    import scenegen as sg
    from paper_2304_09673_amd import st

    scs = sg.config4(args.n_scenes)
    handles = [st.Scene(sc) for sc in scs]
    cams = [sc.camera for sc in scs]
    t0 = time.perf_counter()
    if args.no_autotune:
        b = st.Batch(handles, cams, tuning=st.default_tuning(tile=args.tile, max_new=args.max_new,
                                                             sub_depth=args.sub_depth))
        tuned = "fixed"
    else:
        b = st.Batch(handles, cams, autotune=True, reps=1)
        tuned = "autotuned"
    setup_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        b.render()
    torch.cuda.synchronize()
    stats = b.stats()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        b.render()
        evs[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    frame_ms = float(np.median([a.elapsed_time(c) for a, c in evs]))
    rays = sum(c.width * c.height for c in cams)
    evals = sum(x["field_evals"] for x in stats)
    flops = sum(algorithmic_flops(x) for x in stats)
    line = {
        "metric": "Mrays/s + field evals/s at 1080p, 4096 prims; learned vs plain step at equal depth err",
        "value": round(rays / (ms_per_step * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(scs)} scenes (primitives log-uniform in [32, 8192], resolutions "
                               f"from 256x256 to 1920x1080), one graph launch per frame, plain sphere tracing",
                   "rays": rays, "tuning": {"source": tuned, "tile": b.tuning.tile, "max_new": b.tuning.max_new,
                                            "sub_depth": round(b.tuning.sub_depth, 4)}},
        "frame_ms_device": round(frame_ms, 4),
        "field_evals_per_s": evals / (frame_ms * 1e-3),
        "setup_s": round(setup_s, 2),
        "roofline": {"bound": "alu", "kernel": "batch (binning replay + batch_fast_kernel + batch_wide_kernel)",
                     "achieved": flops / (frame_ms * 1e-3) / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": flops / (frame_ms * 1e-3) / PEAK_FP32, "traffic": None},
    }
    print(json.dumps(line), flush=True)
    b.close()


def bench_batch_streams(args):
    """The 64-scene batch without the persistent batch kernel (switched off):
    every scene's A-buffer build (replayed) and trace per frame, the scenes
    spread round-robin over `frames_in_flight` streams so that their
    latency-bound kernels run side by side; the same frame on one stream is
    reported beside it."""
    import torch
    import scenegen as sg
    from paper_2304_09673_amd import st

    scs = sg.config4(args.n_scenes)
    F = max(1, args.frames_in_flight)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(F - 1)]
    tune = st.default_tuning(tile=args.tile, max_new=args.max_new, sub_depth=args.sub_depth)
    scenes, outs = [], []
    for sc in scs:
        cam = sc.camera
        scenes.append(st.Scene(sc))
        outs.append((torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda"),
                     torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")))

    def frame(nstreams, stats=False):
        res = []
        for i, (sc, s_) in enumerate(zip(scs, scenes)):
            stv = streams[i % nstreams]
            s_.build_abuffer(sc.camera, tune, stream=stv)
            res.append(s_.trace(sc.camera, *outs[i], stats=stats, stream=stv)[2])
        return res

    progress(f"batch of {len(scs)} scenes: sizing builds")
    stats = frame(1, stats=True)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        frame(F)
    torch.cuda.synchronize()
    ref = [o[0].clone() for o in outs]

    def timed(nstreams):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            frame(nstreams)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3

    ms_serial = timed(1)
    ms = timed(F)
    for o, r in zip(outs, ref):
        assert torch.equal(o[0], r), "batch frames differ"
    rays = sum(sc.camera.width * sc.camera.height for sc in scs)
    evals = sum(x["field_evals"] for x in stats)
    flops = sum(algorithmic_flops(x) for x in stats)
    line = {
        "metric": "Mrays/s + field evals/s at 1080p, 4096 prims; learned vs plain step at equal depth err",
        "value": round(rays / (ms * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(scs)} scenes (primitives log-uniform in [32, 8192], resolutions "
                               f"from 256x256 to 1920x1080), every scene built and traced per frame, plain sphere "
                               f"tracing; scenes round-robin over {F} streams (the persistent batch kernel is "
                               f"switched off)",
                   "rays": rays, "streams": F,
                   "tuning": {"source": "fixed", "tile": tune.tile, "max_new": tune.max_new,
                              "sub_depth": round(tune.sub_depth, 4)}},
        "serial": {"ms_per_frame": round(ms_serial, 4), "mrays_s": round(rays / (ms_serial * 1e-3) / 1e6, 3)},
        "field_evals_per_s": evals / (ms * 1e-3),
        "frame_roofline": {"bound": "alu", "note": "algorithmic FLOPs of all traces of a frame over the frame's "
                                                   "wall time (not one kernel's launch)",
                           "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                           "frac": flops / (ms * 1e-3) / PEAK_FP32},
    }
    print(json.dumps(line), flush=True)
    for s_ in scenes:
        s_.close()


def progress(msg: str):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# loss weight of over-predicted step factors (an over-relaxed step that fails
# the overlap test costs an evaluation)
OVER_WEIGHT = 64.0


def learned_vs_plain(args):
    """16384 primitives of the second workload's laws at 3840x2160: plain,
    over-relaxed (factor 1.7) and learned step, with one tuning (the
    autotuner's choice for the plain step).  The step model is trained first
    (outside the timed region) on dumps of the plain tracer over scenes of the
    first two workloads.  Hit masks must agree; depth
    differences between the learned and the plain image are reported (the
    oracle comparison is in the tests)."""
    import torch
    import scenegen as sg
    from paper_2304_09673_amd import st, stepmodel

    sc = sg.config5()
    cam = sc.camera
    # one tuning for all three modes: the autotuner's choice for the plain step
    progress("learned step: autotuning the plain step")
    s = st.Scene(sc)
    tuned, _ = s.autotune(cam, reps=5)
    s.close()
    kw = {"tile": tuned.tile, "max_new": tuned.max_new, "sub_depth": tuned.sub_depth}
    # training scenes: the first two workloads (16 spheres at 256x256, seeds
    # 0-9; 142 primitives at 512x512, seeds 0-4)
    t0 = time.perf_counter()
    train = [sg.config1(seed=k, width=256, height=256) for k in range(10)] + \
            [sg.config2(seed=k, width=512, height=512) for k in range(5)]
    progress("learned step: collecting training samples")
    X, T = stepmodel.collect(train, cap_per_scene=1 << 20, tuning=st.default_tuning(**kw))
    progress(f"learned step: training on {X.shape[0]} samples")
    w, norm, losses = stepmodel.fit(X, T, epochs=10, batch=8192, lr=3e-3, seed=0, over_weight=OVER_WEIGHT)
    train_s = time.perf_counter() - t0
    out = {}
    imgs = {}
    for name, mode in (("plain", st.ST_STEP_PLAIN), ("overrelax", st.ST_STEP_OVERRELAX),
                       ("learned", st.ST_STEP_LEARNED)):
        progress(f"learned step: {name} at {cam.width}x{cam.height}")
        s = st.Scene(sc)
        if mode == st.ST_STEP_LEARNED:
            s.set_step_model(w, norm)
        tune = st.default_tuning(step_mode=mode, **kw)
        s.build_abuffer(cam, tune)
        _, _, stats = s.trace()
        ts = []
        for _ in range(args.c5_reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            d, n, _ = s.trace(stats=False)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        rays = cam.width * cam.height
        imgs[name] = d.cpu().numpy()
        out[name] = {"trace_ms": round(ms, 2), "mrays_s": round(rays / ms / 1e3, 3),
                     "field_evals_per_s": stats["field_evals"] / (ms * 1e-3),
                     "steps_per_ray": stats["steps"] / rays, "evals_per_ray": stats["field_evals"] / rays,
                     "relaxed_accepted": stats["learned_accepted"], "relaxed_rejected": stats["learned_rejected"],
                     "unconverged": stats["unconverged"], "hits": stats["hits"]}
        ext = s.info()["extent"]
        s.close()
    hit = np.isfinite(imgs["plain"])
    for name in ("overrelax", "learned"):
        hn = np.isfinite(imgs[name])
        both = hit & hn
        dd = np.abs(imgs[name][both].astype(np.float64) - imgs["plain"][both]) / ext if both.any() else np.zeros(1)
        out[name]["hit_miss_differs_from_plain"] = int((hn != hit).sum())
        out[name]["depth_diff_vs_plain_rel"] = {"p99": float(np.percentile(dd, 99)), "max": float(dd.max())}
        out[name]["speedup_vs_plain"] = round(out["plain"]["trace_ms"] / out[name]["trace_ms"], 4)
    return {"workload": f"{sc.name}: 16384 primitives, depth<=24, {cam.width}x{cam.height}, autotuned tile "
                        f"{kw['tile']}, max_new {kw['max_new']}, sub_depth {kw['sub_depth']:.3g}; median of "
                        f"{args.c5_reps} traces",
            "train": {"scenes": "first workload seeds 0-9 at 256x256, second workload seeds 0-4 at 512x512",
                      "samples": int(X.shape[0]),
                      "epochs": 10, "over_weight": OVER_WEIGHT, "final_loss": losses[-1],
                      "seconds": round(train_s, 1)},
            **out}


def _wall_ms(fn, reps):
    """Median wall time of fn() over reps calls, each ended by a device synchronization."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def dense_and_ablation(args):
    """The second workload (142 primitives, mixed compact operators) at
    1024x1024 with 16x16 tiles, where about a third of the pixels hit: the
    synchronized frame with the trace kernel's roofline on a frame whose
    field evaluations are dense, and the paper's Table 1 ablation on the same
    frame: ParentPtr/Full and FastPtr/Full (A-buffer of 8x8 tiles with every
    entry kept, per-pixel dexel buffer, every ray traced on its own with the
    field evaluated by Algorithm 1 over parent or fast ancestor pointers).
    Frame times are wall times of build + trace with a synchronization."""
    import torch
    import scenegen as sg
    from paper_2304_09673_amd import st

    sc = sg.config2(0)
    cam = sc.camera
    rays = cam.width * cam.height
    depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda")
    normal = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")
    progress("dense frame: synchronized")
    s = st.Scene(sc)
    tune = st.default_tuning(tile=16)
    s.build_abuffer(cam, tune)
    _, _, stats = s.trace(cam, depth, normal)
    tr = []
    for _ in range(args.c5_reps + 2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        s.trace(cam, depth, normal, stats=False)
        b.record()
        torch.cuda.synchronize()
        tr.append(a.elapsed_time(b))
    trace_ms = float(np.median(tr))
    frame_ms = _wall_ms(lambda: (s.build_abuffer(cam, tune), s.trace(cam, depth, normal, stats=False)),
                        args.c5_reps + 2)
    flops = algorithmic_flops(stats)
    out = {"workload": f"{sc.name}: 142 primitives, random tree depth<=10, compact smooth union/intersection/"
                       f"difference 60/20/20%, {cam.width}x{cam.height}, 16x16 tiles, plain sphere tracing",
           "synchronized": {"frame_ms": round(frame_ms, 3), "mrays_s": round(rays / frame_ms / 1e3, 2),
                            "trace_ms": round(trace_ms, 3), "hits": stats["hits"],
                            "evals_per_ray": stats["field_evals"] / rays,
                            "field_evals_per_s": stats["field_evals"] / (trace_ms * 1e-3)},
           "trace_roofline": {"bound": "alu", "kernel": "trace (trace_fast_kernel + trace_wide_kernel)",
                              "achieved": flops / (trace_ms * 1e-3) / 1e12, "peak": PEAK_FP32 / 1e12,
                              "unit": "TFLOP/s", "frac": flops / (trace_ms * 1e-3) / PEAK_FP32,
                              "frac_nonpacked": flops / (trace_ms * 1e-3) / PEAK_FP32_NONPACKED,
                              "flops_per_launch": flops, "launch_ms": trace_ms, "traffic": None}}
    s.close()
    s = st.Scene(sc)
    full = st.default_tuning(tile=8, keep_all_entries=1)
    for name, variant in (("parent_ptr_full", st.ST_ABLATION_PARENT_PTR), ("fast_ptr_full", st.ST_ABLATION_FAST_PTR)):
        progress(f"dense frame: ablation {name}")
        s.build_abuffer(cam, full)
        _, _, ast = s.trace_ablation(variant, cam, depth, normal)
        ms = _wall_ms(lambda: (s.build_abuffer(cam, full), s.trace_ablation(variant, cam, depth, normal, stats=False)),
                      args.c5_reps)
        out[name] = {"frame_ms": round(ms, 3), "mrays_s": round(rays / ms / 1e3, 2),
                     "dexel_entries": ast["abuffer_entries"], "evals_per_ray": ast["field_evals"] / rays,
                     "operators_visited": ast["view_nodes"], "hits": ast["hits"],
                     "slowdown_vs_synchronized": round(ms / frame_ms, 2)}
    s.close()
    return out


def segment_vs_plain(sc, tune, reps):
    """Plain and segment tracing of the same frame and A-buffer tuning
    (trace-only device time, median of reps)."""
    import torch
    from paper_2304_09673_amd import st
    cam = sc.camera
    rays = cam.width * cam.height
    out = {}
    for name, mode in (("plain", st.ST_STEP_PLAIN), ("segment", st.ST_STEP_SEGMENT)):
        s = st.Scene(sc)
        t = st.default_tuning(tile=tune.tile, max_new=tune.max_new, sub_depth=tune.sub_depth, step_mode=mode)
        s.build_abuffer(cam, t)
        _, _, stats = s.trace()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            s.trace(stats=False)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        out[name] = {"trace_ms": round(ms, 4), "trace_only_mrays_s": round(rays / ms / 1e3, 2),
                     "steps_per_ray": stats["steps"] / rays, "evals_per_ray": stats["field_evals"] / rays}
        s.close()
    out["speedup"] = round(out["plain"]["trace_ms"] / out["segment"]["trace_ms"], 4)
    return out


def tune_in_flight(st, scenes, streams, outs, cam, F, reps=3):
    """The tuning grid of st_autotune (tile 8/16/32, fetch cap 6/16/64/256,
    fetch-ahead depth 1/20 and 1/4 of the scene depth), each setting timed as
    the bench runs its frames: F in flight, every frame a replayed build and a
    trace without statistics.  Returns the fastest setting."""
    import torch

    best = None
    for tile in (8, 16, 32):
        for max_new in (6, 16, 64, 256):
            for sub_depth in (0.05, 0.25):
                t = st.default_tuning(tile=tile, max_new=max_new, sub_depth=sub_depth)
                for i in range(F):   # sizing builds, then one frame per slot
                    scenes[i].build_abuffer(cam, t, stream=streams[i])
                    scenes[i].trace(cam, *outs[i], stats=False, stream=streams[i])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for k in range(reps * F):
                    i = k % F
                    scenes[i].build_abuffer(cam, t, stream=streams[i])
                    scenes[i].trace(cam, *outs[i], stats=False, stream=streams[i])
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if best is None or dt < best[0]:
                    best = (dt, t)
    return best[1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 100 frames of ~0.12 ms: the start (an idle chip) and the drain (the last
    # frames' tails) of the timed region weigh little against them
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--max-new", type=int, default=64)
    ap.add_argument("--sub-depth", type=float, default=0.25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=24576)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB")
    ap.add_argument("--n-scenes", type=int, default=64)
    ap.add_argument("--no-c5", action="store_true", help="skip the learned-vs-plain comparison")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the 1024x1024 second-workload frame (dense roofline, ablation variants)")
    ap.add_argument("--c5-reps", type=int, default=3)
    ap.add_argument("--frames-in-flight", type=int, default=4,
                    help="frames rendered concurrently (one scene, output pair and stream each; the "
                         "default, 4, is one per hardware queue HIP gives a process)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU design (screen tiles sharded "
              "across GPUs, no exchange during a frame) is described but not built.", file=sys.stderr)
        sys.exit(2)

    if args.calib_copy:
        calib_copy(args.calib_copy)
        return

    if args.config == 4:
        try:
            bench_batch(args)
        except Exception as exc:   # the batch entry points refuse while switched off
            progress(f"persistent batch unavailable ({exc}); scenes on streams instead")
            bench_batch_streams(args)
        return

    import torch
    import scenegen as sg
    from paper_2304_09673_amd import st

    sc = sg.by_config(args.config, seed=args.seed)
    cam = sc.camera
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    scene = st.Scene(sc)
    flatten_ms = (time.perf_counter() - t0) * 1e3
    F = max(1, args.frames_in_flight)
    # F frames in flight: one scene (its own A-buffer), output pair and
    # stream per slot; frame k runs on slot k mod F, so frame k+1's build
    # overlaps frame k's trace.  Streams keep the default priority.
    scenes = [scene] + [st.Scene(sc) for _ in range(F - 1)]
    streams = [stream] + [torch.cuda.Stream() for _ in range(F - 1)]
    outs = [(torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda"),
             torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")) for _ in range(F)]
    depth, normal = outs[0]
    library_choice = None
    if args.no_autotune:
        tune = st.default_tuning(tile=args.tile, max_new=args.max_new, sub_depth=args.sub_depth)
        tuned = "fixed"
    else:
        # set-up, outside the timed region: grid search of tile size, fetch
        # cap and fetch-ahead depth with device timing (the library's
        # autotuner, one frame at a time), then the same grid timed the way
        # the frames run below, F in flight
        tune, _ = scene.autotune(cam, reps=3)
        library_choice = {"tile": tune.tile, "max_new": tune.max_new, "sub_depth": round(tune.sub_depth, 4)}
        if F > 1:
            tune = tune_in_flight(st, scenes, streams, outs, cam, F)
            tuned = "autotuned, frames in flight"
        else:
            tuned = "autotuned"

    def step(slot=0, stats=False, ev=None):
        sc_, st_ = scenes[slot], streams[slot]
        sc_.build_abuffer(cam, tune, stream=st_)
        if ev is not None:
            ev[0].record(st_)
        out = sc_.trace(cam, *outs[slot], stats=stats, stream=st_)
        if ev is not None:
            ev[1].record(st_)
        return out[2]

    for _ in range(args.warmup):
        for i in range(F):
            step(i)
    torch.cuda.synchronize()
    stats = step(stats=True)
    torch.cuda.synchronize()

    # one frame at a time on one stream (per-frame latency, build and trace
    # split); not the reported value when F > 1
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(0, ev=evs[k])
    torch.cuda.synchronize()
    serial_ms = (time.perf_counter() - t0) / args.steps * 1e3
    serial_trace_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    build_ms = serial_ms - serial_trace_ms

    # the timed region: exactly `steps` frames, F in flight
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    # the library records a HIP event pair around every tile-test launch, on
    # the build stream
    for s_ in scenes:
        s_.kernel_timing(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k % F, ev=evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    test_total_ms, test_launches = 0.0, 0
    for s_ in scenes:
        a, b = s_.kernel_timing(False)
        test_total_ms += a
        test_launches += b
    test_ms_avg = test_total_ms / max(test_launches, 1)
    ms_per_step = wall / args.steps * 1e3
    trace_ms = [a.elapsed_time(b) for a, b in evs]
    trace_ms_avg = float(np.mean(trace_ms))
    # every slot renders the same image
    for d_, n_ in outs[1:]:
        assert torch.equal(d_, depth) and torch.equal(n_, normal), "frames in flight differ"

    rays = cam.width * cam.height
    value = rays / (ms_per_step * 1e-3) / 1e6
    evals_per_s = stats["field_evals"] / (trace_ms_avg * 1e-3)
    flops = algorithmic_flops(stats)
    achieved = flops / (trace_ms_avg * 1e-3)
    pix = stats["candidate_pixels"]
    test_flops = pix[0] * FLOPS_TEST["sphere"] + pix[1] * FLOPS_TEST["box"] + pix[2] * FLOPS_TEST["capsule"]
    test_achieved = test_flops / (test_ms_avg * 1e-3)
    roof_trace = {"bound": "alu", "kernel": "trace (trace_fast_kernel + trace_wide_kernel)",
                  "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                  "frac": achieved / PEAK_FP32, "frac_nonpacked": achieved / PEAK_FP32_NONPACKED,
                  "flops_per_launch": flops, "launch_ms": trace_ms_avg, "traffic": measured_traffic("trace")}
    roof_test = {"bound": "alu", "kernel": "binning tile test (tile_test_kernel)",
                 "achieved": test_achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                 "frac": test_achieved / PEAK_FP32, "frac_nonpacked": test_achieved / PEAK_FP32_NONPACKED,
                 "flops_per_launch": test_flops, "launch_ms": test_ms_avg, "launches_timed": test_launches,
                 "tested_pixels": {"sphere": pix[0], "box": pix[1], "capsule": pix[2]},
                 "traffic": measured_traffic("tile_test")}
    # the roofline of the kernel that takes longest per frame
    dominant, other = (roof_test, roof_trace) if test_ms_avg >= trace_ms_avg else (roof_trace, roof_test)

    line = {
        "metric": "Mrays/s + field evals/s at 1080p, 4096 prims; learned vs plain step at equal depth err",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{sc.name} seed {args.seed}: {sc.n_prims} primitives (spheres, boxes, capsules; "
                               f"32-cluster Gaussian mixture), random tree depth<=16, compact smooth "
                               f"union/intersection/difference 60/20/20%, {cam.width}x{cam.height}, "
                               f"plain sphere tracing",
                   "rays": rays, "tuning": {"source": tuned, "tile": tune.tile, "max_new": tune.max_new,
                                            "sub_depth": round(tune.sub_depth, 4), "eps": tune.eps,
                                            **({"library_autotune": library_choice} if library_choice else {})},
                   "frames_in_flight": F},
        "field_evals_per_s": evals_per_s,
        "trace_ms": round(trace_ms_avg, 4),
        "serial": {"note": "one frame at a time on one stream: build (replayed, no host synchronization) "
                           "then trace; ms_per_frame is the frame's latency",
                   "ms_per_frame": round(serial_ms, 4), "mrays_s": round(rays / (serial_ms * 1e-3) / 1e6, 3),
                   "trace_ms": round(serial_trace_ms, 4), "build_ms": round(build_ms, 4)},
        "build_ms": round(build_ms, 4),
        "flatten_ms": round(flatten_ms, 3),
        "trace_only_mrays_s": round(rays / (trace_ms_avg * 1e-3) / 1e6, 3),
        "evals_per_ray": stats["field_evals"] / rays,
        "hits": stats["hits"],
        "unconverged": stats["unconverged"],
        "abuffer_entries": stats["abuffer_entries"],
        "abuffer_binned": stats["abuffer_binned"],
        "max_overlap": stats["max_overlap"],
        "max_active": stats["max_active"],
        "block_cycles": {"note": "8x8 blocks of the statistics frame, shader clock cycles from the start to the end "
                                 "of each block (the trace launch lasts at least the longest)",
                         "max": stats["block_cycles_max"],
                         "mean": stats["block_cycles_sum"] / max(1, -(-cam.width // 8) * -(-cam.height // 8)),
                         "blocks": -(-cam.width // 8) * -(-cam.height // 8)},
        "subfrustums": stats["subfrustums"],
        "empty_views": stats["empty_views"],
        "view_nodes": stats["view_nodes"],
        "wide_tiles": stats["wide_tiles"],
        "abuffer_candidates": stats["abuffer_candidates"],
        "abuffer_tested": stats["abuffer_tested"],
        "roofline": dominant,
        "roofline_other_kernel": other,
    }
    # binning (HBM-bound by design): algorithmic bytes = VOI reads (2 passes,
    # 48 B/primitive each), tile count/scan/offsets (12 B/tile), per candidate
    # the scatter write, the pre-test pruning's read and primitive-to-node
    # lookup (12 B), per tested candidate the pruning's write, the test's read
    # and write (4 + 4 + 12 B) and the post-test pruning's read (12 B), per
    # kept entry the pruning's write and the per-tile sort's read + write
    # (12 + 24 B)
    n_tiles = -(-cam.width // tune.tile) * -(-cam.height // tune.tile)
    e = stats["abuffer_entries"]
    ec = stats["abuffer_candidates"]
    et = stats["abuffer_tested"]
    bin_bytes = 96 * sc.n_prims + 12 * n_tiles + 12 * ec + 32 * et + 36 * e
    line["binning"] = {"bound": "hbm", "algorithmic_bytes": bin_bytes, "ms_wall": round(build_ms, 4),
                       "achieved_GBps": bin_bytes / (build_ms * 1e-3) / 1e9,
                       "frac": bin_bytes / (build_ms * 1e-3) / 8e12,
                       "note": "serial frame wall time minus the trace's device time: the build replayed "
                               "with the sizes of the valid A-buffer (no host synchronization), launch gaps "
                               "included"}
    progress(f"frame: {value:.1f} Mrays/s")
    progress("segment tracing on the same frame")
    line["segment_vs_plain"] = segment_vs_plain(sc, tune, 5)
    if not args.no_dense:
        line["dense_frame"] = dense_and_ablation(args)
    if not args.no_c5:
        line["learned_vs_plain"] = learned_vs_plain(args)
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(sc, args.config, args.seed, args.cpu_rays)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
