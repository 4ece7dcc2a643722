#!/usr/bin/env python3
"""Benchmark of the VBD hot path on one MI355X.

Headline: vertex-updates/s of the 65^3-vertex tet cube (274,625 vertices,
1,572,864 stable Neo-Hookean tets, per-tet E log-uniform in [1e4, 1e6] Pa,
h = 1/60 s, 100 VBD iterations per frame, greedy coloring, adaptive init),
FP32 state on the GPU, inputs resident in HBM.  A vertex update is one local
solve of a free vertex; value = free vertices x iterations x frames / time.

Also measured in the same run (JSON "extra"): every launch mode on the cube,
the batched 512-mesh workload (persistent hipGraph launch vs the plain kernel
mesh by mesh), the adjoint (forward + backward of the 33^3 differentiable
workload), the 1024^2 mass-spring cloth with contacts, a STREAM-like copy
probe, and the paper's own timings with their hardware, as context.  "roofline" is the color-solve kernel's algorithmic HBM bytes per
launch over its average launch time (HIP events on the launch stream);
"cpu_baseline" is the FP64 oracle timed on a bounded sample of the cube.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
       [--no-cpu-baseline] [--mode auto|plain|graph|persistent|persistent_graph]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
MODES = {"plain": 0, "graph": 1, "persistent": 2, "persistent_graph": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="auto", choices=["auto"] + list(MODES))
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=50)
    ap.add_argument("--profile-only", default="",
                    help="run only one workload for a profiler: cube|batch|copy|stack|adjoint|floor")
    ap.add_argument("--lanes", type=int, default=8, help="--profile-only: lanes per vertex")
    ap.add_argument("--block", type=int, default=128, help="--profile-only: block size")
    ap.add_argument("--remap", type=int, default=1, help="--profile-only: XCD remap")
    ap.add_argument("--unroll", type=int, default=3, help="--profile-only: tet entries per lane")
    ap.add_argument("--compact", type=int, default=0, help="--profile-only: 32-B pair records")
    return ap.parse_args()


def state(w, dev):
    import torch
    x = torch.tensor(w.x0, dtype=torch.float32, device=dev).contiguous()
    v = torch.tensor(w.v0, dtype=torch.float32, device=dev).contiguous()
    E = torch.tensor(w.tet_E, dtype=torch.float32, device=dev).contiguous()
    return x, v, v.clone(), E


def time_frames(topo, w, mode, steps, warmup, dev, autotune=True):
    """Time `steps` frames after `warmup` frames; returns (seconds, updates/frame)."""
    import torch
    x, v, vp, E = state(w, dev)
    if autotune:
        topo.autotune(x, v, vp, E, w.params, mode)
    for _ in range(warmup):
        topo.step(x, v, vp, E, w.params, mode)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        topo.step(x, v, vp, E, w.params, mode)
    b.record()
    torch.cuda.synchronize()
    topo.check()
    if not bool(torch.isfinite(x).all()):
        raise RuntimeError("non-finite positions after the timed frames")
    free = int((w.pinned == 0).sum())
    return a.elapsed_time(b) / 1e3, free * w.params.n_iters


def kernel_roofline(topo, w, dev, frames=3):
    """Average color-solve launch time and algorithmic bytes (plain launches)."""
    import torch
    x, v, vp, E = state(w, dev)
    topo.step(x, v, vp, E, w.params, MODES["plain"])
    topo.profile_enable(True)
    topo.profile_read(reset=True)
    for _ in range(frames):
        topo.step(x, v, vp, E, w.params, MODES["plain"])
    torch.cuda.synchronize()
    st = topo.profile_read(reset=True)
    topo.profile_enable(False)
    avg_ms = st["total_ms"] / st["n_launches"]
    avg_bytes = st["total_bytes"] / st["n_launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    return dict(avg_ms=avg_ms, avg_bytes=avg_bytes, achieved_gbs=achieved,
                launches=st["n_launches"],
                updates_per_s=st["n_vertex_updates"] / (st["total_ms"] * 1e-3))


def adjoint_phases(topo, w, dev, frames=2):
    """Average reverse color-phase time and algorithmic bytes: plain backward
    launches of recorded frames, timed by the library's profiler."""
    import torch
    from paper_2403_06321_amd import _native as N
    x, v, vp, E = state(w, dev)
    g = [torch.full_like(x, 1e-3) for _ in range(3)]
    o = [torch.zeros_like(x) for _ in range(3)]
    gE = torch.zeros_like(E)
    tot = None
    for f in range(frames + 1):
        xs = (x.clone(), v.clone(), vp.clone())
        topo.step_record(x, v, vp, E, w.params, N.LAUNCH_PLAIN)
        if f == 1:
            topo.profile_enable(True)
            topo.profile_read(reset=True)
        topo.step_backward(*xs, E, *g, *o, gE, w.params, N.LAUNCH_PLAIN, recorded=True)
    torch.cuda.synchronize()
    st = topo.profile_read(reset=True)
    topo.profile_enable(False)
    avg_ms = st["total_ms"] / st["n_launches"]
    avg_bytes = st["total_bytes"] / st["n_launches"]
    return dict(avg_ms=avg_ms, avg_bytes=avg_bytes, achieved_gbs=avg_bytes / (avg_ms * 1e-3) / 1e9)


def read_probe(dev):
    """Best read-only streaming rate over a 2 GiB buffer (the library's probe,
    a few grid sizes)."""
    import torch
    from paper_2403_06321_amd.api import probe_read
    n = 1 << 29
    src = torch.ones(n, device=dev)
    best = 0.0
    for blocks in (256, 512, 1024, 8192):
        part = torch.zeros(blocks, device=dev)
        probe_read(src, part)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            probe_read(src, part)
        b.record()
        torch.cuda.synchronize()
        best = max(best, 5 * 4 * n / (a.elapsed_time(b) * 1e-3) / 1e9)
    del src
    torch.cuda.empty_cache()
    return best


# The paper's own timings (Table 1: average time per step on its scenes),
# turned into vertex-updates/s as vertices x iterations / step time; its
# hardware, meshes and contact work differ from these workloads, so they are
# context, not a target.
PAPER_CONTEXT = {
    "source": "Table 1 (average time per step), vertices x iterations / step time",
    "hardware": "NVIDIA RTX 4090, FP32; collision detection on the CPU (Embree) where contacts are active",
    "scenes": [
        {"scene": "squishy ball drop", "vertices": 230000, "tets": 700000, "iterations": 120,
         "ms_per_step": 15.0, "vertex_updates_per_s": 1.8e9, "contacts": True},
        {"scene": "216 squishy balls into a teapot", "vertices": 48000000, "tets": 151000000,
         "iterations": 40, "ms_per_step": 3600.0, "vertex_updates_per_s": 5.3e8, "contacts": True},
        {"scene": "10,368 models dropping", "vertices": 36000000, "tets": 124000000, "iterations": 60,
         "ms_per_step": 4200.0, "vertex_updates_per_s": 5.1e8, "contacts": True},
        {"scene": "flattening initialization", "vertices": 15000, "tets": 50000, "iterations": 100,
         "ms_per_step": 3.3, "vertex_updates_per_s": 4.5e8, "contacts": False},
    ],
}


def kernel_traffic(cfg):
    """Measured HBM bytes per launch of the color-solve kernel in launch
    configuration cfg, from committed rocprofv3 counter runs (one record per
    configuration taken); None when cfg was not measured or the kernel source
    has changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_solve_tet_cube65.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2403_06321_amd", "csrc", "vbd_kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernel_sha256"):
        return None
    keys = ("lanes_per_vertex", "block_size", "xcd_remap", "blocks_per_cu", "tet_unroll", "compact_records")
    for r in rec.get("configs", []):
        if all(r["launch_config"].get(k) == cfg.get(k) for k in keys):
            return r["bytes_per_launch"]
    return None


def host_threads():
    """The host's CPU share: the affinity mask, capped by OMP_NUM_THREADS when
    the environment sets it."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(omp))) if omp.isdigit() else n


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, iters):
    """The FP64 oracle (plain loops, OpenMP within a color) on bounded samples
    of the benchmarked workloads, on the host's CPU share and on one thread."""
    import dataclasses
    import oracle as O
    threads = host_threads()
    res = {}

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    # the headline cube: one frame x `iters` iterations on all threads, 2 on one
    w = W.config_large_cube(coloring="smallest_last")
    m = O.Model.from_workload(w)
    free = int((w.pinned == 0).sum())
    O.set_threads(threads)
    p = dataclasses.replace(w.params, n_iters=iters)
    dt = timed(lambda: O.step(m, p, w.x0, w.v0, w.v0, w.tet_E))
    O.set_threads(1)
    p1 = dataclasses.replace(w.params, n_iters=1)
    dt1 = timed(lambda: O.step(m, p1, w.x0, w.v0, w.v0, w.tet_E))
    res.update(value=free * iters / dt, unit="vertex-updates/s", cores=threads, kind="oracle",
               sample=f"65^3 cube, 1 frame x {iters} iterations, FP64, {threads} threads, "
                      f"{dt:.1f} s; single thread: 1 frame x 1 iteration, {dt1:.1f} s",
               single_thread=free / dt1, cpu_model=cpu_model(),
               host_cpus=os.cpu_count())
    del m
    O.set_threads(threads)
    # the batch: 8 seeded sample meshes of the 512, one frame of 40 iterations
    wb = W.config_batch(frames=1, coloring="smallest_last")
    import numpy as np
    ids = sorted(np.random.default_rng(3).choice(wb.n_meshes, 8, replace=False).tolist())
    sub = W.subset_meshes(wb, ids)
    ms = O.Model.from_workload(sub)
    dtb = timed(lambda: O.step(ms, sub.params, sub.x0, sub.v0, sub.v0, sub.tet_E))
    res["batch_8_meshes"] = dict(value=sub.n_verts * sub.params.n_iters / dtb, unit="vertex-updates/s",
                                 seconds=dtb, sample=f"8 of the 512 meshes ({sub.n_verts} vertices), "
                                                     f"1 frame x {sub.params.n_iters} iterations")
    # the differentiable cube: one frame of 5 iterations forward and its adjoint
    wd = W.config_differentiable(coloring="smallest_last")
    wd = dataclasses.replace(wd, params=dataclasses.replace(wd.params, n_iters=5))
    md = O.Model.from_workload(wd)
    st = {}

    def fwd():
        st["x"] = O.step(md, wd.params, wd.x0, wd.v0, wd.v0, wd.tet_E)[0]
    dtf = timed(fwd)
    g = np.ones_like(wd.x0) * 1e-3
    dtg = timed(lambda: O.step_backward(md, wd.params, wd.x0, wd.v0, wd.v0, wd.tet_E, g, g * 0, g * 0))
    freed = int((wd.pinned == 0).sum())
    res["adjoint_one_frame"] = dict(forward_s=dtf, backward_s=dtg,
                                    updates_per_s_forward_backward=freed * wd.params.n_iters / (dtf + dtg),
                                    sample=f"33^3 cube, 1 frame x {wd.params.n_iters} iterations, "
                                           "forward then adjoint")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_06321_amd import workloads as W
    from paper_2403_06321_amd.api import Topology, probe_copy
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.profile_only == "copy":
        n = 1 << 28   # 1 GiB of float32
        src = torch.ones(n, device=dev); dst = torch.empty_like(src)
        for _ in range(5):
            probe_copy(dst, src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * 4 * n}))
        return

    if args.profile_only == "floor":
        print(json.dumps(phase_floor(dev, W, Topology)))
        return

    if args.profile_only == "stack":
        # mesh-mesh contacts: 4 levels of 8x8 stacked 9^3 cubes, plain launches
        ws = W.config_block_stack(cols=8, levels=4, n=9, coloring="smallest_last")
        ts = Topology.from_workload(ws)
        secs, upd = time_frames(ts, ws, MODES["plain"], args.steps, args.warmup, dev, autotune=False)
        print(json.dumps({"profile": "stack", "ms_per_frame": secs / args.steps * 1e3}))
        return

    if args.profile_only == "batch":
        # the 512-mesh batch, plain launches in the given launch configuration
        wb = W.config_batch(coloring="smallest_last")
        tb = Topology.from_workload(wb)
        tb.launch_config = dict(lanes_per_vertex=args.lanes, block_size=args.block,
                                xcd_remap=args.remap, tet_unroll=args.unroll,
                                compact_records=args.compact)
        secs, upd = time_frames(tb, wb, MODES["plain"], args.steps, args.warmup, dev, autotune=False)
        print(json.dumps({"profile": "batch", "ms_per_frame": secs / args.steps * 1e3}))
        return

    if args.profile_only == "adjoint":
        # forward + backward through the 33^3 differentiable workload
        from paper_2403_06321_amd.api import Rollout
        wd = W.config_differentiable(coloring="smallest_last")
        td = Topology.from_workload(wd, max_backward_iters=wd.params.n_iters)
        x0, v0, _, E = state(wd, dev)
        # the launch configuration given (the reverse phases take its block
        # size and XCD mapping), so that counter runs are reproducible
        td.launch_config = dict(lanes_per_vertex=args.lanes, block_size=args.block, xcd_remap=args.remap,
                                blocks_per_cu=0, tet_unroll=args.unroll, compact_records=args.compact)
        v0.requires_grad_(True); E.requires_grad_(True)
        target = torch.tensor(wd.target, dtype=torch.float32, device=dev)
        for _ in range(args.steps):
            xT, _ = Rollout.apply(x0, v0, E, td, wd.params, wd.frames)
            ((xT.mean(0) - target) ** 2).sum().backward()
        torch.cuda.synchronize()
        print(json.dumps({"profile": "adjoint", "launch_config": td.launch_config}))
        return

    # ---------------------------------------------------------- headline ----
    w = W.config_large_cube(coloring="smallest_last")
    log(f"[bench] building topology: {w.name}, {w.n_verts} verts, {w.n_tets} tets")
    t0 = time.perf_counter()
    topo = Topology.from_workload(w)
    log(f"[bench] topology built in {time.perf_counter() - t0:.1f} s, {topo.n_colors} colors")
    if args.profile_only == "cube":
        topo.launch_config = dict(lanes_per_vertex=args.lanes, block_size=args.block,
                                  xcd_remap=args.remap, tet_unroll=args.unroll,
                                  compact_records=args.compact)
        secs, upd = time_frames(topo, w, MODES["plain"], args.steps, args.warmup, dev, autotune=False)
        print(json.dumps({"profile": "cube", "ms_per_frame": secs / args.steps * 1e3}))
        return
    modes = list(MODES) if args.mode == "auto" else [args.mode]
    per_mode = {}
    for name in modes:
        secs, upd = time_frames(topo, w, MODES[name], min(args.steps, 20) if args.mode == "auto" else args.steps,
                                args.warmup, dev)
        n = min(args.steps, 20) if args.mode == "auto" else args.steps
        per_mode[name] = dict(updates_per_s=upd * n / secs, ms_per_frame=secs / n * 1e3,
                              config=topo.launch_config)
        log(f"[bench] cube mode {name}: {per_mode[name]['updates_per_s']:.3e} v-upd/s, "
            f"{per_mode[name]['ms_per_frame']:.2f} ms/frame, cfg {topo.launch_config}")
    best = max(per_mode, key=lambda k: per_mode[k]["updates_per_s"])
    # the timed run of the headline, in the best mode
    topo.autotune(*state(w, dev), w.params, MODES[best])
    secs, upd = time_frames(topo, w, MODES[best], args.steps, args.warmup, dev, autotune=False)
    value = upd * args.steps / secs
    ms_per_step = secs / args.steps * 1e3
    log(f"[bench] headline ({best}): {value:.3e} v-upd/s, {ms_per_step:.3f} ms/frame")
    # two more runs of the same frames, for the median and minimum of three
    runs = [value]
    for _ in range(2):
        s2, _ = time_frames(topo, w, MODES[best], args.steps, args.warmup, dev, autotune=False)
        runs.append(upd * args.steps / s2)
    headline_runs = dict(updates_per_s=runs, median=float(sorted(runs)[1]), min=float(min(runs)))
    log(f"[bench] three runs: median {headline_runs['median']:.3e}, min {headline_runs['min']:.3e}")
    roof = kernel_roofline(topo, w, dev)
    log(f"[bench] solve kernel: {roof['avg_ms'] * 1e3:.1f} us/launch, "
        f"{roof['avg_bytes'] / 1e6:.2f} MB/launch, {roof['achieved_gbs']:.0f} GB/s")
    traffic = kernel_traffic(topo.launch_config)
    read_gbs = read_probe(dev)
    # the cache-ideal byte model (every array once per iteration: 60 B per tet,
    # 4 B per tet-vertex pair, 52 B per vertex), shared by the iteration's
    # color phases
    model_a = (60.0 * w.n_tets + 4.0 * 4 * w.n_tets + 52.0 * w.n_verts) / topo.n_colors
    log(f"[bench] read probe {read_gbs:.0f} GB/s; cache-ideal model {model_a / 1e6:.2f} MB/launch "
        f"-> {model_a / (roof['avg_ms'] * 1e-3) / 1e9:.0f} GB/s")

    out = {
        "metric": "VBD vertex-updates/s + HBM GB/s, 64³ tet cube; batched & adjoint vs plain",
        "value": value,
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tet cube 65x65x65 vertices (274,625 verts, 1,572,864 tets), "
                               "per-tet E log-uniform [1e4,1e6] Pa, nu 0.3, h 1/60 s, 100 iterations x "
                               "frames, greedy vertex coloring (first fit in smallest-last order, "
                               f"{topo.n_colors} colors), bottom face pinned",
                   "launch_mode": best, "launch_config": topo.launch_config,
                   "free_vertices": int((w.pinned == 0).sum()), "iterations": w.params.n_iters},
        "roofline": {"bound": "hbm", "achieved": roof["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": roof["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "k_solve<tets> (one color phase per launch)",
                     "avg_launch_us": roof["avg_ms"] * 1e3,
                     "algorithmic_bytes_per_launch": roof["avg_bytes"],
                     "read_probe_gbs": read_gbs, "frac_of_read_probe": roof["achieved_gbs"] / read_gbs,
                     "cache_ideal_bytes_per_launch": model_a,
                     "cache_ideal_frac": model_a / (roof["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "measured_traffic_frac": (None if traffic is None else
                                               traffic / (roof["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)},
    }
    del topo
    torch.cuda.empty_cache()

    extra = {"cube_modes": per_mode, "headline_runs": headline_runs}
    if not args.no_extras:
        # the same cube and iterations with other colorings: greedy first fit in
        # vertex-id order (8 colors) and the caller-supplied lattice coloring
        for name, coloring in (("cube_greedy_id_order", "id"), ("cube_lattice_4_colors", "lattice4")):
            w4 = W.config_large_cube(coloring=coloring)
            t4 = Topology.from_workload(w4)
            n = min(args.steps, 20)
            secs, upd = time_frames(t4, w4, MODES["graph"], n, args.warmup, dev)
            r4 = kernel_roofline(t4, w4, dev)
            extra[name] = dict(updates_per_s=upd * n / secs, ms_per_frame=secs / n * 1e3,
                               colors=t4.n_colors, config=t4.launch_config,
                               solve_kernel=dict(avg_launch_us=r4["avg_ms"] * 1e3,
                                                 achieved_gbs=r4["achieved_gbs"],
                                                 frac=r4["achieved_gbs"] / HBM_PEAK_GBS))
            log(f"[bench] 65^3, {coloring} coloring ({t4.n_colors} colors): "
                f"{extra[name]['updates_per_s']:.3e} v-upd/s, {r4['avg_ms'] * 1e3:.1f} us/launch, "
                f"{r4['achieved_gbs']:.0f} GB/s")
            del t4
            torch.cuda.empty_cache()
    if not args.no_extras:
        # copy probe: achievable streaming bandwidth
        n = 1 << 28
        src = torch.ones(n, device=dev); dst = torch.empty_like(src)
        probe_copy(dst, src); torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            probe_copy(dst, src)
        b.record(); torch.cuda.synchronize()
        extra["copy_probe_gbs"] = 10 * 8 * n / (a.elapsed_time(b) * 1e-3) / 1e9
        del src, dst
        log(f"[bench] copy probe {extra['copy_probe_gbs']:.0f} GB/s")
        extra.update(extras(dev, W, Topology))
    extra["paper_context"] = PAPER_CONTEXT
    out["extra"] = extra
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_iters)
        log(f"[bench] oracle {out['cpu_baseline']['value']:.3e} v-upd/s ({out['cpu_baseline']['sample']})")
    print(json.dumps(out))


def phase_floor(dev, W, Topology):
    """Cost of one color phase with (almost) no work: a 2x2x2 cube (8 colors
    of one vertex) stepped with 2000 iterations, per-color kernels replayed
    from a hipGraph against the persistent kernel's grid barrier (the
    autotuned grid of the 65^3 cube: the barrier's cost depends on the grid,
    not on the work)."""
    import dataclasses
    import torch
    w = W.tet_cube(2, 0, n_iters=2000, pin_bottom=False)
    t = Topology.from_workload(w)
    res = {}
    for name, mode, cfg in (("graph_us", MODES["graph"], dict(block_size=64)),
                            ("persistent_256_blocks_us", MODES["persistent_graph"],
                             dict(block_size=512, blocks_per_cu=1)),
                            ("persistent_1024_blocks_us", MODES["persistent_graph"],
                             dict(block_size=256, blocks_per_cu=4))):
        t.launch_config = cfg
        secs, _ = time_frames(t, w, mode, 5, 2, dev, autotune=False)
        res[name] = secs / 5 / (w.params.n_iters * t.n_colors) * 1e6
    res["workload"] = (f"2x2x2 cube, {t.n_colors} colors of one vertex, 2000 iterations; "
                       "per color phase")
    return res


def extras(dev, W, Topology):
    import torch
    res = {}
    res["phase_floor"] = phase_floor(dev, W, Topology)
    log(f"[bench] empty color phase: graph {res['phase_floor']['graph_us']:.2f} us, persistent "
        f"{res['phase_floor']['persistent_256_blocks_us']:.2f} us (256 blocks), "
        f"{res['phase_floor']['persistent_1024_blocks_us']:.2f} us (1024 blocks)")
    # batched: 512 meshes, persistent hipGraph vs the plain kernel mesh by mesh
    wb = W.config_batch(coloring="smallest_last")
    log(f"[bench] batch: {wb.n_meshes} meshes, {wb.n_verts} verts, {wb.n_tets} tets")
    t0 = time.perf_counter()
    tb = Topology.from_workload(wb)
    log(f"[bench] batch topology {time.perf_counter() - t0:.1f} s, {tb.n_colors} colors")
    secs, upd = time_frames(tb, wb, MODES["persistent_graph"], 10, 2, dev)
    res["batched_persistent_graph"] = dict(updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100,
                                           config=tb.launch_config)
    secs, upd = time_frames(tb, wb, MODES["graph"], 10, 2, dev)
    res["batched_graph"] = dict(updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100,
                                config=tb.launch_config)
    log(f"[bench] batched persistent graph {res['batched_persistent_graph']['updates_per_s']:.3e}, "
        f"graph {res['batched_graph']['updates_per_s']:.3e} v-upd/s")
    roof = kernel_roofline(tb, wb, dev, frames=1)
    res["batched_solve_kernel"] = dict(avg_launch_us=roof["avg_ms"] * 1e3,
                                       achieved_gbs=roof["achieved_gbs"],
                                       frac=roof["achieved_gbs"] / HBM_PEAK_GBS)
    del tb
    # plain kernel, mesh by mesh (one topology per mesh, plain launches), 1 frame
    vo, to = wb.offsets()
    tops, sts = [], []
    for k in range(wb.n_meshes):
        sub = W.subset_meshes(wb, [k])
        tops.append(Topology.from_workload(sub))
        sts.append(state(sub, dev))
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for t, (x, v, vp, E) in zip(tops, sts):
        t.step(x, v, vp, E, wb.params, MODES["plain"])
    b.record(); torch.cuda.synchronize()
    upd = int(wb.n_verts) * wb.params.n_iters
    res["batched_plain_mesh_by_mesh"] = dict(updates_per_s=upd / (a.elapsed_time(b) * 1e-3),
                                             ms_per_frame=a.elapsed_time(b))
    log(f"[bench] plain mesh by mesh {res['batched_plain_mesh_by_mesh']['updates_per_s']:.3e} v-upd/s")
    del tops, sts
    torch.cuda.empty_cache()
    # adjoint: differentiable 33^3 workload, forward + backward through 30 frames
    from paper_2403_06321_amd.api import Rollout
    wd = W.config_differentiable(coloring="smallest_last")
    td = Topology.from_workload(wd, max_backward_iters=wd.params.n_iters)
    x0, v0, _, E = state(wd, dev)
    td.autotune(x0, v0, v0.clone(), E, wd.params, MODES["graph"])
    v0.requires_grad_(True); E.requires_grad_(True)
    target = torch.tensor(wd.target, dtype=torch.float32, device=dev)

    def fwd_bwd():
        xT, _ = Rollout.apply(x0, v0, E, td, wd.params, wd.frames)
        loss = ((xT.mean(0) - target) ** 2).sum()
        loss.backward()
        return loss

    fwd_bwd(); torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    for _ in range(3):
        fwd_bwd()
    b.record(); torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 3
    free = int((wd.pinned == 0).sum())
    upd = free * wd.params.n_iters * wd.frames
    x, v, vp, E2 = state(wd, dev)
    a.record()
    for _ in range(wd.frames):
        td.step(x, v, vp, E2, wd.params, MODES["plain"])
    b.record(); torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b)
    # the reverse color phases alone (plain launches, HIP events around the
    # sweep) against the forward color phases of the same topology
    adj = adjoint_phases(td, wd, dev)
    fwd_k = kernel_roofline(td, wd, dev, frames=2)
    res["adjoint"] = dict(forward_backward_ms=ms, forward_only_ms=ms_fwd,
                          updates_per_s_forward_backward=upd / (ms * 1e-3),
                          updates_per_s_forward=upd / (ms_fwd * 1e-3),
                          reverse_phase=dict(avg_launch_us=adj["avg_ms"] * 1e3,
                                             algorithmic_bytes_per_launch=adj["avg_bytes"],
                                             achieved_gbs=adj["achieved_gbs"],
                                             frac=adj["achieved_gbs"] / HBM_PEAK_GBS),
                          forward_phase=dict(avg_launch_us=fwd_k["avg_ms"] * 1e3,
                                             algorithmic_bytes_per_launch=fwd_k["avg_bytes"],
                                             achieved_gbs=fwd_k["achieved_gbs"],
                                             frac=fwd_k["achieved_gbs"] / HBM_PEAK_GBS),
                          reverse_over_forward_phase=adj["avg_ms"] / fwd_k["avg_ms"],
                          workload="33^3 cube, 30 frames x 20 iterations, loss on final centroid, "
                                   f"smallest-last coloring ({td.n_colors} colors)",
                          config=td.launch_config)
    log(f"[bench] adjoint fwd+bwd {ms:.1f} ms, forward {ms_fwd:.1f} ms; reverse phase "
        f"{adj['avg_ms'] * 1e3:.2f} us ({adj['achieved_gbs']:.0f} GB/s), forward phase "
        f"{fwd_k['avg_ms'] * 1e3:.2f} us ({fwd_k['achieved_gbs']:.0f} GB/s)")
    del td
    # mesh-mesh contacts: 4 levels of 8x8 stacked 9^3 cubes, graph launches
    ws = W.config_block_stack(cols=8, levels=4, n=9, coloring="smallest_last")
    ts = Topology.from_workload(ws)
    secs, upd = time_frames(ts, ws, MODES["graph"], 10, 2, dev)
    xs = state(ws, dev)[0]
    ts.detect_contacts(xs, ws.params)
    torch.cuda.synchronize()
    a.record()
    for _ in range(10):
        tri = ts.detect_contacts(xs, ws.params)
    b.record(); torch.cuda.synchronize()
    res["block_stack_contacts_graph"] = dict(
        updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100,
        detection_ms=a.elapsed_time(b) / 10, contacts_at_rest=int((tri >= 0).sum().item()),
        workload=f"{ws.name}: {ws.n_verts} vertices, {ws.n_tets} tets, {ws.params.n_iters} iterations, "
                 f"smallest-last coloring ({ts.n_colors} colors)")
    log(f"[bench] block stack {res['block_stack_contacts_graph']['updates_per_s']:.3e} v-upd/s, "
        f"detection {res['block_stack_contacts_graph']['detection_ms']:.3f} ms")
    del ts
    # cloth
    wc = W.config_cloth()
    tc = Topology.from_workload(wc)
    secs, upd = time_frames(tc, wc, MODES["persistent_graph"], 10, 3, dev)
    res["cloth_persistent_graph"] = dict(updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100)
    secs, upd = time_frames(tc, wc, MODES["graph"], 10, 3, dev)
    res["cloth_graph"] = dict(updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100)
    # the whole drop (frames 0-119, plain launches: no graph capture inside the
    # timed frames), and frames 30-39 alone, when the cloth drapes over the
    # sphere with most of its contacts active
    secs, upd = time_frames(tc, wc, MODES["plain"], wc.frames, 0, dev, autotune=False)
    res["cloth_plain_all_frames"] = dict(updates_per_s=upd * wc.frames / secs,
                                         ms_per_frame=secs / wc.frames * 1e3, frames=wc.frames)
    secs, upd = time_frames(tc, wc, MODES["graph"], 10, 30, dev, autotune=False)
    res["cloth_graph_frames_30_39"] = dict(updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100)
    log(f"[bench] cloth all {wc.frames} frames {res['cloth_plain_all_frames']['updates_per_s']:.3e}, "
        f"frames 30-39 {res['cloth_graph_frames_30_39']['updates_per_s']:.3e} v-upd/s")
    roof = kernel_roofline(tc, wc, dev, frames=2)
    res["cloth_solve_kernel"] = dict(avg_launch_us=roof["avg_ms"] * 1e3,
                                     achieved_gbs=roof["achieved_gbs"],
                                     frac=roof["achieved_gbs"] / HBM_PEAK_GBS)
    log(f"[bench] cloth {res['cloth_persistent_graph']['updates_per_s']:.3e} / "
        f"{res['cloth_graph']['updates_per_s']:.3e} v-upd/s")
    del tc
    # the same cloth colored by DSATUR: 5 colors instead of 7
    wd = W.config_cloth(coloring="dsatur")
    td = Topology.from_workload(wd)
    secs, upd = time_frames(td, wd, MODES["persistent_graph"], 10, 3, dev)
    res["cloth_dsatur_persistent_graph"] = dict(updates_per_s=upd * 10 / secs,
                                                ms_per_frame=secs * 100, n_colors=td.n_colors)
    secs, upd = time_frames(td, wd, MODES["graph"], 10, 3, dev)
    res["cloth_dsatur_graph"] = dict(updates_per_s=upd * 10 / secs, ms_per_frame=secs * 100,
                                     n_colors=td.n_colors)
    log(f"[bench] cloth dsatur ({td.n_colors} colors) "
        f"{res['cloth_dsatur_persistent_graph']['updates_per_s']:.3e} / "
        f"{res['cloth_dsatur_graph']['updates_per_s']:.3e} v-upd/s")
    return res


if __name__ == "__main__":
    main()
