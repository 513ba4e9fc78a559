"""Benchmark of the shift-and-stack search on one MI355X.

One step = one sst_detect call over the full synthetic field (64 frames of
1024x1024 float32, an 81x81 grid of trial velocities at 1 px/h, S/N 5 cut,
top-64 candidates per velocity): frame statistics, padded background-
subtracted copy, coverage intervals, the stacking kernel with S/N and peak
extraction, and the per-velocity merge.  Frames are resident in HBM before the
timed region.  The metric is frame*pixel*velocity updates per second
(N*H*W*N_vel per step / step time).

The JSON line also carries the roofline position of the dominant kernel
(the stacking kernel, timed with HIP events on its launch stream inside the
library) and the float64 CPU oracle timed on a bounded sample of the same
workload.
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

# MI355X published FP32 vector peak: 157.3 TFLOP/s (256 CUs x 2.4 GHz x 128
# lanes x 2 flops of an FMA).  One update of the search is one FP32 add, counted
# as one flop.  The FP32 add rate itself is 256 x 128 x 2.4 GHz = 78.6 T adds/s
# (a plain v_add_f32 loop measures 112 adds/clk/CU, 88 % of it).
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_ADD_T = 78.6
HBM_PEAK_GBS = 8000.0


# Profile summary of the stacking kernel on the full field, holding the HBM
# bytes per launch measured with the profiler's FETCH_SIZE / WRITE_SIZE
# counters (each scaled by what the counter reads for a plain 1 GiB copy) and
# a hash of the kernel sources it was taken on.
PROFILE = os.path.join(ROOT, "profiles", "k_stack_detect_64x1024x1024_grid81x81.md")
KERNEL_SOURCES = ("paper_2303_07293_amd/csrc/sst_kernels.hip", "paper_2303_07293_amd/csrc/sst_internal.h",
                  "paper_2303_07293_amd/csrc/sst_api.cpp")


def measured_traffic():
    """HBM bytes per launch of the stacking kernel from the committed profile,
    or None if the kernel sources changed since the counters were taken."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256_16") != h.hexdigest()[:16] or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


_ORACLE_FIELD = None


def _oracle_share(ks):
    """One worker's share of the oracle sample (velocity indices ks); the
    field is inherited from the parent process (fork)."""
    import oracle
    f = _ORACLE_FIELD
    t0 = time.perf_counter()
    oracle.detect(f.frames, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max, velocities=ks)
    return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(f, per_core: int, max_workers: int = 16, seed: int = 0):
    """The float64 oracle as written, timed on the host cores: velocity
    indices of the same field spread over worker processes (fork; the frames
    are shared copy-on-write), each worker running oracle.detect on its share
    (its own frame statistics included, as the GPU step includes them).
    Value: updates of the sample / wall time.  Also a single-core run."""
    import multiprocessing as mp
    global _ORACLE_FIELD
    _ORACLE_FIELD = f
    cores = max(1, min(os.cpu_count() or 1, max_workers))
    rng = np.random.default_rng(seed)
    nk = len(f.vx) * len(f.vy)
    n_vel = min(nk, cores * per_core)
    ks = sorted(rng.choice(nk, size=n_vel, replace=False).tolist())
    shares = [ks[j::cores] for j in range(cores)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        busy = pool.map(_oracle_share, shares)
        wall = time.perf_counter() - t0
    one = ks[:per_core]
    t1 = _oracle_share(one)
    px = f.n * f.h * f.w
    return {"value": n_vel * px / wall, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "single_core_value": len(one) * px / t1,
            "sample": f"{n_vel} of {nk} velocities of the same field (all {f.n} frames of {f.w}x{f.h}) in "
                      f"{cores} worker processes, numpy float64 oracle incl. frame statistics; wall {wall:.1f} s, "
                      f"{sum(busy):.1f} s of worker time; single core: {len(one)} velocities in {t1:.1f} s"}


def copy_reference(torch, mib: int):
    """A plain copy of known size on the device (read mib MiB, write mib MiB)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read": n * 4, "bytes_written": n * 4, "repeats": 3}), flush=True)


def prep_bench(torch, sst, args):
    """The steps the paper runs before the search, on survey-shaped frames:
    64 raw 2048x2048 frames binned 2x2, then static-source removal by the
    per-pixel median and co-adding of 13-frame groups on the binned frames.
    Each is HBM-bound: reported as algorithmic bytes (read once + written
    once) per kernel time against the HBM peak."""
    import synth
    n, side, group = 64, 2048, 13
    rng = np.random.default_rng(synth.SEED_BASE + 5)
    raw = torch.from_numpy(rng.normal(100.0, 10.0, size=(n, side, side)).astype(np.float32)).to("cuda:0")
    binned = sst.sst_bin2x2(raw)
    torch.cuda.synchronize()
    h = w = side // 2
    ng = n // group
    cases = {
        "bin2x2": (lambda: sst.sst_bin2x2(raw), 4 * n * side * side + 4 * n * h * w),
        "median_subtract": (lambda: sst.sst_median_subtract(binned), 4 * n * h * w * 2),
        "coadd13": (lambda: sst.sst_coadd(binned, group), 4 * ng * group * h * w + 4 * ng * h * w),
    }
    res = {}
    for name, (fn, nbytes) in cases.items():
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "bytes": nbytes, "GB/s": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    print(json.dumps({"metric": "preprocessing HBM throughput", "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"prep {n}x{side}x{side} -> bin 2x2 -> median, co-add {group}"},
                      "kernels": res}), flush=True)


def refine_bench(torch, sst, args):
    """4096 candidates drawn (with replacement, seeded) from the full field's
    detections, jittered by up to 0.5 px and 0.5 px/h, refined with 33x33
    bilinear cutouts over the 64 frames and 20 gradient-ascent steps in one
    call.  Reported: candidates x steps per second and bilinear samples per
    second (21 evaluations per candidate, each 64 x 33 x 33 samples)."""
    import synth
    f = synth.full_field()
    fr = torch.from_numpy(f.frames).to("cuda:0")
    cand, count = sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max)
    g = sst.candidates_to_numpy(cand)
    cnt = count.cpu().numpy()
    pool = [(g[k]["x"][j], g[k]["y"][j], f.vx[g[k]["ivx"][j]], f.vy[g[k]["ivy"][j]])
            for k in range(len(cnt)) for j in range(min(int(cnt[k]), f.k_max))]
    pool = np.array(pool, np.float64)
    rng = np.random.default_rng(synth.SEED_BASE + 5)
    nc, steps, cut = 4096, 20, 33
    pick = pool[rng.integers(0, len(pool), nc)]
    th = pick + np.concatenate([rng.uniform(-0.5, 0.5, (nc, 2)), rng.uniform(-0.5, 0.5, (nc, 2))], axis=1)
    tht = torch.from_numpy(th.astype(np.float32)).to("cuda:0")
    for _ in range(args.warmup):
        sst.sst_refine(fr, f.t, f.t_ref, tht, cutout=cut, steps=steps, lr=0.002)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        _, sn, _ = sst.sst_refine(fr, f.t, f.t_ref, tht, cutout=cut, steps=steps, lr=0.002)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    samples = nc * (steps + 1) * f.n * cut * cut
    print(json.dumps({"metric": "refinement candidate-steps/s", "value": nc * steps / (ms * 1e-3),
                      "unit": "candidate-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_call": ms, "bilinear_samples_per_s": samples / (ms * 1e-3), "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": f"refine {nc} detections of {f.name}, cutout {cut}, {steps} steps",
                                 "detections_pool": len(pool), "mean_snr_after": float(sn.mean())}}), flush=True)


def batch_bench(torch, sst, args):
    """Many fields per call.  batch: the 16 uneven fields of the batching
    workload (24-160 frames, 512^2-2048^2, grids 41^2-121^2); tinybatch: 64
    fields of the small field's shape (32 x 128^2, 21^2 grid).  Each field is
    prepared once, with the velocity-block shape the tuner picks for its
    geometry (tune_plan); timed are (a) plain sst_detect calls, one
    per field, (b) the prepared runs enqueued back to back, (c) the same runs
    captured in one graph and replayed, (d) the runs spread over 4 streams,
    (e) (d) captured in one graph, (f) one persistent stacking launch per
    round for all fields (SstBatch), (g) (f) captured in one graph.  Value:
    updates/s of the faster of (e) and (g)."""
    import synth
    dev = torch.device("cuda:0")
    if args.workload == "batch":
        specs = synth.uneven_batch()
    else:
        base = synth.tiny_field(noise=False)
        specs = [synth.FieldSpec(f"tiny{k}", synth.SEED_BASE + 400 + k, base.n, base.h, len(base.vx), base.t, 3)
                 for k in range(64)]
    fields = []
    for sp in sorted(specs, key=lambda s: -s.updates):  # largest first
        f = sp.make()
        fr = torch.from_numpy(f.frames).to(dev)
        # the velocity-block shape is picked per geometry by the tuner
        plan = sst.tune_plan(fr, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max)
        out = (torch.empty((plan.nk, f.k_max, 8), dtype=torch.int32, device=dev),
               torch.empty((plan.nk,), dtype=torch.int32, device=dev))
        # the one-shot calls use the default shape: a workspace of their own
        ews = torch.empty(sst.sst_workspace_bytes(sst.SST_OP_DETECT, f.n, f.h, f.w, f.t, f.t_ref, f.vx, f.vy,
                                                  f.k_max), dtype=torch.uint8, device=dev)
        fields.append((f.name, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max, fr, plan, out,
                       ews, sp.updates))
        del f
        if args.workload == "batch":
            print(f"prepared {sp.name}", file=sys.stderr, flush=True)
    total = sum(x[-1] for x in fields)

    def eager():
        for (_, t, t_ref, vx, vy, thr, cmin, kmax, fr, plan, (c, n), ews, _) in fields:
            sst.sst_detect(fr, t, t_ref, vx, vy, thr, cmin, kmax, ws=ews, cand=c, count=n)

    def runs():
        for (*_, fr, plan, (c, n), _ews, _) in fields:
            plan.run(fr, cand=c, count=n)

    # the same runs spread over 4 streams (fields round-robin, default
    # priority): independent fields can then share the GPU
    streams = [torch.cuda.Stream() for _ in range(4)]

    def runs_parallel():
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for k, (*_, fr, plan, (c, n), _ews, _) in enumerate(fields):
            with torch.cuda.stream(streams[k % len(streams)]):
                plan.run(fr, cand=c, count=n)
        for st in streams:
            cur.wait_stream(st)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    reps = max(1, args.steps // (5 if args.workload == "batch" else 1))
    t_runs = timed(runs, reps)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        runs()
    torch.cuda.synchronize()
    t_graph = timed(graph.replay, reps)
    t_par = timed(runs_parallel, reps)
    graph4 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph4):
        runs_parallel()
    torch.cuda.synchronize()
    t_graph4 = timed(graph4.replay, reps)
    # (f) one persistent stacking launch per round for all fields, (g) (f)
    # captured in one graph
    batch = sst.SstBatch([x[9] for x in fields])
    bframes = [x[8] for x in fields]
    bc, bn = [x[10][0] for x in fields], [x[10][1] for x in fields]

    def batched():
        batch.run(bframes, cands=bc, counts=bn)

    t_batch = timed(batched, reps)
    graphb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graphb):
        batched()
    torch.cuda.synchronize()
    t_graphb = timed(graphb.replay, reps)
    # the eager path re-uploads the tables into the plans' workspaces: last
    t_eager = timed(eager, reps)
    best = min(t_graph4, t_graphb)
    print(json.dumps({"metric": "frame*pixel*velocity updates/s", "value": total / best, "unit": "updates/s",
                      "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": best * 1e3, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"{args.workload}: {len(fields)} fields, {total:.3g} updates",
                                 "fields": [x[0] for x in fields],
                                 "shapes": [sst.sst_shapes()[x[9].shape] for x in fields]},
                      "ms_eager_calls": t_eager * 1e3, "ms_prepared_runs": t_runs * 1e3,
                      "ms_graph_replay": t_graph * 1e3, "ms_prepared_runs_4_streams": t_par * 1e3,
                      "ms_graph_replay_4_streams": t_graph4 * 1e3, "ms_persistent_batch": t_batch * 1e3,
                      "ms_graph_replay_persistent_batch": t_graphb * 1e3}), flush=True)


def roofline(updates: float, kern_ms: float, launches: float, traffic=None, kernel="k_stack<detect>"):
    """Roofline position of the stacking kernel: one FP32 add (one flop) per
    update over the kernel's event-timed duration, against the published
    FP32 vector peak; the FP32 add rate is a separate, labelled ceiling."""
    achieved = updates / (kern_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic, "traffic_unit": "B/launch",
            "kernel": kernel, "kernel_ms_per_step": round(kern_ms, 4), "launches_per_step": launches,
            "add_rate_ceiling": {"peak": PEAK_FP32_ADD_T, "unit": "T adds/s",
                                 "frac": round(achieved / PEAK_FP32_ADD_T, 4)}}


def time_plain_stack(torch, sst, f, steps: int, warmup: int):
    """sst_stack (SUM, every [vy][vx][h][w] float32 stack written to HBM) on
    field f: step time, kernel time and the compulsory HBM bytes (frames read
    once, stacks written once) per step against the HBM peak."""
    dev = torch.device("cuda:0")
    frames = torch.from_numpy(f.frames).to(dev)
    n, h, w = f.frames.shape
    nvx, nvy = len(f.vx), len(f.vy)
    nb = sst.sst_workspace_bytes(sst.SST_OP_STACK, n, h, w, f.t, f.t_ref, f.vx, f.vy)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = torch.empty((nvy, nvx, h, w), dtype=torch.float32, device=dev)

    def step():
        sst.sst_stack(frames, f.t, f.t_ref, f.vx, f.vy, out=out, ws=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    sst.sst_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kern_ms, launches = sst.sst_profile_end()
    kern_ms /= steps
    updates = n * h * w * nvx * nvy
    nbytes = 4 * n * h * w + 4 * nvx * nvy * h * w
    del out, ws, frames
    torch.cuda.empty_cache()
    return {"workload": f.name, "ms_per_step": round(dt * 1e3, 4), "updates_per_s": updates / dt,
            "compulsory_bytes": nbytes, "GB/s": round(nbytes / dt / 1e9, 1),
            "frac_hbm": round(nbytes / dt / 1e9 / HBM_PEAK_GBS, 4),
            "roofline": roofline(updates, kern_ms, launches / steps, None, "k_stack<stack>")}


def stack_bench(torch, sst, args):
    """The plain float32 stack (`sst_stack`, SUM, every [vy][vx][h][w] stack
    written to HBM) on the full field's grid: 32 frames (the diagnostic shape,
    where the written stacks make HBM a co-binding roof) or all 64.  Reported
    as updates/s, and as compulsory HBM bytes (frames read once, stacks
    written once) per step time against the HBM peak."""
    import synth
    f = synth.diagnostic_field() if args.workload == "stack" else synth.full_field()
    r = time_plain_stack(torch, sst, f, args.steps, args.warmup)
    print(json.dumps({
        "metric": "frame*pixel*velocity updates/s", "value": r["updates_per_s"], "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"plain stack {f.n}x{f.h}x{f.w} grid{len(f.vx)}x{len(f.vy)}, SUM, stacks written",
                   "output_bytes": 4 * len(f.vx) * len(f.vy) * f.h * f.w},
        "hbm": {"compulsory_bytes": r["compulsory_bytes"], "GB/s": r["GB/s"], "frac": r["frac_hbm"]},
        "roofline": r["roofline"],
    }), flush=True)


def time_detect(torch, sst, f, frames, scale, steps: int, warmup: int):
    """sst_detect on field f (frames already on the device): seconds per
    step, stacking-kernel ms per step, launches per step, candidates."""
    dev = frames.device
    n, h, w = f.frames.shape
    nk = len(f.vx) * len(f.vy)
    nb = sst.sst_workspace_bytes(sst.SST_OP_DETECT, n, h, w, f.t, f.t_ref, f.vx, f.vy, f.k_max)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    cand = torch.empty((nk, f.k_max, 8), dtype=torch.int32, device=dev)
    count = torch.empty((nk,), dtype=torch.int32, device=dev)

    def step():
        sst.sst_detect(frames, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max,
                       scale=scale, ws=ws, cand=cand, count=count)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    sst.sst_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kern_ms, launches = sst.sst_profile_end()
    cands = int(count.sum().item())
    del ws, cand, count
    return dt, kern_ms / steps, launches / steps, cands


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["full", "tiny", "prep", "refine", "batch", "tinybatch", "stack", "stackfull"],
                    default="full",
                    help="full: the search on the full field; tiny: the small field; prep: the steps before the "
                         "search (2x2 binning, median removal, co-adding) timed on their own; refine: sub-pixel "
                         "refinement of 4096 full-field detections (33x33 cutouts, 20 ascent steps); batch: 16 "
                         "uneven fields as prepared runs, back to back and as one graph; tinybatch: 64 small "
                         "fields likewise; stack / stackfull: the plain float32 stacks written to HBM, 32 or 64 "
                         "frames of the full field")
    ap.add_argument("--storage", choices=["f32", "bf16", "f16"], default="f32",
                    help="frame storage: 16-bit frames with per-frame scales (quantised on the GPU before the "
                         "timed region); arithmetic stays float32")
    ap.add_argument("--cpu-velocities", type=int, default=8,
                    help="oracle sample: velocities per host core (a few seconds per core at the full field; "
                         "0: skip)")
    ap.add_argument("--half-search", action="store_true",
                    help="with --storage f16: search the 16-bit samples themselves (sst_set_half_search)")
    ap.add_argument("--no-extras", action="store_true",
                    help="full workload: skip the 16-bit storage and plain-stack measurements")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (three times) and exit: "
                         "the reference point that scales the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the search shards by field or velocity block with no exchange between GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_mib > 0:
        copy_reference(torch, args.copy_mib)
        return
    import synth
    import paper_2303_07293_amd as sst
    if args.workload == "prep":
        prep_bench(torch, sst, args)
        return
    if args.workload == "refine":
        refine_bench(torch, sst, args)
        return
    if args.workload in ("batch", "tinybatch"):
        batch_bench(torch, sst, args)
        return
    if args.workload in ("stack", "stackfull"):
        stack_bench(torch, sst, args)
        return

    f = synth.full_field() if args.workload == "full" else synth.tiny_field()
    dev = torch.device("cuda:0")
    frames = torch.from_numpy(f.frames).to(dev)
    scale = None
    if args.storage != "f32":
        # centred storage: each frame's mean removed before rounding (S/N unchanged)
        frames, scale, _ = sst.sst_quantize(frames, torch.bfloat16 if args.storage == "bf16" else torch.float16,
                                            center=True)
        torch.cuda.synchronize()
    if args.half_search:
        if args.storage != "f16":
            print("--half-search needs --storage f16", file=sys.stderr)
            sys.exit(2)
        sst.sst_set_half_search(True)
    n, h, w = f.frames.shape
    nk = len(f.vx) * len(f.vy)
    dt, kern_ms_step, launches, cands = time_detect(torch, sst, f, frames, scale, args.steps, args.warmup)
    updates = f.updates
    value = updates / dt
    # the counters were taken on float32 frames of the full field
    traffic = measured_traffic() if args.workload == "full" and args.storage == "f32" else None
    out = {
        "metric": "frame*pixel*velocity updates/s", "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f.name, "storage": args.storage + ("-searched-16bit" if args.half_search else ""),
                   "frames": n, "height": h, "width": w, "velocities": nk,
                   "threshold": f.threshold, "k_max": f.k_max, "candidates_last_step": cands},
        "roofline": roofline(updates, kern_ms_step, launches, traffic),
    }
    if args.workload == "full" and args.storage == "f32" and not args.no_extras:
        # the rest of the metric: 16-bit storage against float32 on the same
        # field, and the plain stacks' HBM fraction
        del frames
        torch.cuda.empty_cache()
        fr32 = torch.from_numpy(f.frames).to(dev)
        ratio = {"f32_ms_per_step": round(dt * 1e3, 4)}
        # bf16 and f16 searched on a float32 copy (the default), and f16
        # searched on its 16-bit samples (mixed-precision FMA, opt-in)
        for name, tdt, direct in (("bf16", torch.bfloat16, False), ("f16", torch.float16, False),
                                  ("f16_direct", torch.float16, True)):
            q, sc, _ = sst.sst_quantize(fr32, tdt, center=True)
            torch.cuda.synchronize()
            prev = sst.sst_set_half_search(direct)
            try:
                d16, k16, _, c16 = time_detect(torch, sst, f, q, sc, max(3, args.steps // 2), 2)
            finally:
                sst.sst_set_half_search(prev)
            ratio[f"{name}_ms_per_step"] = round(d16 * 1e3, 4)
            ratio[f"speedup_{name}_vs_f32"] = round(dt / d16, 4)
            ratio[f"{name}_candidates"] = c16
            del q, sc
        del fr32
        torch.cuda.empty_cache()
        out["storage_16bit_vs_f32"] = ratio
        ps = max(2, args.steps // 5)
        out["plain_stack_hbm"] = [time_plain_stack(torch, sst, synth.diagnostic_field(), ps, 1),
                                  time_plain_stack(torch, sst, f, ps, 1)]
    if args.cpu_velocities > 0:
        out["cpu_baseline"] = cpu_baseline(f, args.cpu_velocities)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
