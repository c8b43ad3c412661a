#!/usr/bin/env python3
"""Throughput benchmark of GPU block matching (selection + exhaustive NCC search).

One step = one pass of the whole hot path over one volume pair already
resident in HBM: variance-ranked selection of the blocks of `ref`, the
per-voxel window statistics of `flt` (the two are independent and run on two
streams; launched eagerly, or captured once as a HIP graph and replayed,
whichever is faster), and the exhaustive NCC search of every selected block.
The step time is taken by the host clock over steps with no timing events;
the kernel times come from a second run of the same steps with HIP events.  The default workload is the MRI-shaped pair (256x256x124
uint16, 12-bit, blocks 7^3 on a stride-7 grid, top 25% by variance = 5508
blocks, window +-10).

Prints one JSON line: whole-step throughput in evaluated NCC voxel-pairs per
second, ms per step, p50/p99 latency of one registration call (selection +
matching, enqueue to stream sync), the roofline position of the search
kernel (timed with HIP events on its stream) and the oracle's CPU
throughput on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (generator kwargs, block, stride, fraction, window)
    "mri_256x256x124_u16": ("mri", 7, 7, 0.25, 10),
    "translation_64_f32": ("translation", 7, 7, 0.20, 5),
    "blobs_512x512x256_u16": ("blobs", 9, 5, 0.70, 12),
}
# the batched parametric search: the 64^3 float pair with 32 parameter sets
BATCHED = "batched_64_f32_32sets"
# the registration server: Poisson arrivals of mixed-size requests
SERVING = "serving_poisson_4hz"
# selection inside a region mask with a connectivity pattern, on the MRI pair
# (one-workgroup path) and on the dense 512x512x256 grid (round launches)
SELECT_EX = "mri_select_ex_u16"
SELECT_EX_DENSE = "blobs_select_ex_u16"
SELECT_EX_CFG = {SELECT_EX: ("mri", 7, 7, 0.25, 6), SELECT_EX_DENSE: ("blobs", 9, 5, 0.70, 6)}
# per-axis sizes on the MRI pair: blocks thinner along z (slice axis)
ANISO = "mri_aniso_256x256x124_u16"
ANISO_CFG = {"block": (7, 7, 3), "stride": (7, 7, 3), "fraction": 0.25, "window": (10, 10, 4)}

# MI355X: 256 CUs x 2.4 GHz x 256 ops/clk/CU (2 multiply-adds per lane per
# clock: packed FP32 FMA, or v_dot2_i32_i16) = the FP32 vector peak.
PEAK_TOPS = 157.3
# MI355X dense fp16 matrix-core peak (the matrix-core search's own dtype)
PEAK_MFMA_F16_TFLOPS = 2500.0
OPS_PER_PAIR = 2  # one multiply-add per (block voxel, displacement) pair


# HBM traffic of the search kernels, measured with rocprofv3 counters and kept
# in profiles/ (one summary per workload); reported only while the kernel's
# sources are unchanged.
TRAFFIC_FILES = {
    ("mri_256x256x124_u16", "dot2"): ("k_match_u16_mri_256x256x124_traffic.json",
                                      ["paper_2308_10868_amd/csrc/match.hip",
                                       "paper_2308_10868_amd/csrc/nrr_internal.h"]),
    ("blobs_512x512x256_u16", "dot2"): ("k_match_u16_blobs_512x512x256_traffic.json",
                                        ["paper_2308_10868_amd/csrc/match.hip",
                                         "paper_2308_10868_amd/csrc/nrr_internal.h"]),
    ("mri_256x256x124_u16", "mfma"): ("k_match_mfma_mri_256x256x124_traffic.json",
                                      ["paper_2308_10868_amd/csrc/match_mfma.hip",
                                       "paper_2308_10868_amd/csrc/nrr_internal.h"]),
    ("blobs_512x512x256_u16", "mfma"): ("k_match_mfma_blobs_512x512x256_traffic.json",
                                        ["paper_2308_10868_amd/csrc/match_mfma.hip",
                                         "paper_2308_10868_amd/csrc/nrr_internal.h"]),
    ("mri_aniso_256x256x124_u16", "fma"): ("k_match_aniso_u16_mri_256x256x124_traffic.json",
                                           ["paper_2308_10868_amd/csrc/match_aniso.hip",
                                            "paper_2308_10868_amd/csrc/nrr_internal.h"]),
}


def kernel_source_hash(sources) -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, arith: str):
    """Bytes per search launch from the committed counter summary, or None
    when it was taken on other sources or there is none for the workload and
    arithmetic form."""
    if (workload, arith) not in TRAFFIC_FILES:
        return None
    name, sources = TRAFFIC_FILES[(workload, arith)]
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("workload") != workload or t.get("source_sha256") != kernel_source_hash(sources):
        return None
    return t.get("traffic_bytes")


def make_pair(kind: str, seed: int):
    from paper_2308_10868_amd import synth

    if kind == "mri":
        return synth.gen_mri_u16(seed=seed)
    if kind == "translation":
        return synth.gen_translation_f32(seed=seed)
    return synth.gen_blobs_u16(seed=seed)


def evaluated_pairs(centers: np.ndarray, dims, b, w) -> int:
    """sum over blocks of the block's voxel count x (number of displacements
    whose displaced block stays inside the volume); b and w are numbers or
    per-axis (x, y, z) triples."""
    b = np.broadcast_to(np.asarray(b, dtype=np.int64), (3,))
    w = np.broadcast_to(np.asarray(w, dtype=np.int64), (3,))
    h = (b - 1) // 2
    c = centers.astype(np.int64)
    n = np.asarray(dims, dtype=np.int64)
    lo = np.maximum(-w, h - c)
    hi = np.minimum(w, n - 1 - h - c)
    cnt = np.prod(np.maximum(hi - lo + 1, 0), axis=1)
    return int(cnt.sum()) * int(np.prod(b))


def to_dev(a: np.ndarray, torch):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(a).cuda()


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the CPU baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own block-matching timings, as context (another machine, other
# data; none is this metric): its GPU block matching ran about 10x faster
# than its CPU code, and tuning the GPU launch configuration gained about 30x,
# on a GeForce 8800 GT beside two Core2 Duo CPUs at 3.16 GHz, where the
# time-critical registration (block matching and the FEM solve) took under a
# minute; the cluster version answered in 30-42 s (240 + 29 processors).
PAPER_CONTEXT = {
    "gpu_vs_cpu_block_matching": "about 10x (NVIDIA GeForce 8800 GT vs 2x Intel Core2 Duo "
                                 "3.16 GHz; clinical MRI, block sizes not stated)",
    "tuned_vs_untuned_launch": "about 30x on the same GPU",
    "time_critical_registration": "under 1 min on that workstation; 30-42 s on a 269-processor "
                                  "cluster (7 clinical cases)",
}


def cpu_baseline(pair, centers: np.ndarray, b, w, budget_s: float):
    """Time the FP64 oracle on a bounded, seeded sample of the selected blocks
    (per-axis search when b is a triple): on all host threads with about
    two thirds of the budget, then on one thread with the rest."""
    import oracle

    oracle.build()
    search = oracle.match if np.ndim(b) == 0 else oracle.match_aniso
    rng = np.random.default_rng(1)
    order = rng.permutation(len(centers))

    def timed(n_probe, budget):
        probe = centers[order[:n_probe]]
        t = time.perf_counter()
        search(pair.ref, pair.flt, probe, b, w)
        per_block = max(time.perf_counter() - t, 1e-6) / len(probe)
        n = int(min(len(centers), max(n_probe, budget / per_block)))
        sample = centers[order[:n]]
        t = time.perf_counter()
        search(pair.ref, pair.flt, sample, b, w)
        dt = time.perf_counter() - t
        return evaluated_pairs(sample, pair.dims, b, w), dt, n

    cores = oracle.threads()
    pairs, dt, n = timed(32, budget_s * 2 / 3)
    oracle.set_threads(1)
    pairs1, dt1, n1 = timed(4, budget_s / 3)
    oracle.set_threads(cores)
    return {"value": pairs / dt, "unit": "voxel-pairs/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d of %d selected blocks (seeded), %.3g pairs, %.1f s"
            % (n, len(centers), pairs, dt),
            "value_1core": pairs1 / dt1,
            "sample_1core": "%d blocks, %.3g pairs, %.1f s" % (n1, pairs1, dt1)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mri_256x256x124_u16",
                    choices=sorted(WORKLOADS) + [BATCHED, SERVING, ANISO, SELECT_EX,
                                                 SELECT_EX_DENSE])
    ap.add_argument("--requests", type=int, default=48,
                    help="requests of the serving workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device-to-device copy 3 times (the reference "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the selection and statistics eagerly every step")
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 = skip)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        n = 256 << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: every box here has a single MI355X and the "
              "block-matching path is built and timed per GPU (multi-GPU sharding is a design "
              "note, not a measured path). Run with --gpus 1.", file=sys.stderr)
        return 2

    if args.workload == BATCHED:
        return bench_batched(args)
    if args.workload == SERVING:
        return bench_serving(args)
    if args.workload == ANISO:
        return bench_aniso(args)
    if args.workload in SELECT_EX_CFG:
        return bench_select_ex(args)

    import torch

    import paper_2308_10868_amd as nrr

    kind, b, stride, frac, w = WORKLOADS[args.workload]
    t0 = time.time()
    pair = make_pair(kind, args.seed)
    print("# generated %s in %.1f s" % (args.workload, time.time() - t0), file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ref = to_dev(pair.ref, torch)
    flt = to_dev(pair.flt, torch)
    dt_code, dims = (nrr.U16 if pair.ref.dtype == np.uint16 else nrr.F32), pair.dims
    k = nrr.select_count(dims, b, stride, frac)
    sel_ws = torch.empty(nrr.select_workspace_bytes(dims, b, stride), dtype=torch.uint8, device=dev)
    mat_ws = torch.empty(nrr.match_workspace_bytes(dt_code, dims, b), dtype=torch.uint8, device=dev)
    disp = torch.empty((k, 3), dtype=torch.int32, device=dev)
    ncc = torch.empty(k, dtype=torch.float32, device=dev)
    conf = torch.empty(k, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        # selection (reads ref) and the window statistics (read flt) are
        # independent: one library call runs the statistics on its second
        # stream beside the selection, forked after the keys kernel (so the
        # selection's one-workgroup kernel is placed first) and joined back
        # before the search; being on this stream, they follow the previous
        # step's search, which releases the table.  ev: events around the
        # selection + statistics and around the search, on this stream.
        if ev is not None:
            ev[0].record(stream)
        centers, _ = nrr.select_and_window_stats(ref, flt, b, stride, frac, w,
                                                 select_workspace=sel_ws, match_workspace=mat_ws)
        if ev is not None:
            ev[1].record(stream)
            ev[2].record(stream)
        nrr.block_match(ref, flt, centers, b, w, workspace=mat_ws, out=(disp, ncc, conf),
                        prepared=True)
        if ev is not None:
            ev[3].record(stream)
        return centers

    for _ in range(args.warmup):
        centers = step()
    torch.cuda.synchronize()
    centers_h = centers.cpu().numpy()
    pairs = evaluated_pairs(centers_h, dims, b, w)
    nominal = k * b ** 3 * (2 * w + 1) ** 3

    def host_ms(fn):
        # steps back to back, no timing events (they add markers between the
        # launches); host clock around them, synchronized on both sides
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    ms_step = host_ms(step)
    # the same steps with HIP events around the selection and the search
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(4))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    search_ms = np.array([ev[2].elapsed_time(ev[3]) for ev in evs])
    select_ms = np.array([ev[0].elapsed_time(ev[1]) for ev in evs])
    kern_ms = float(np.mean(search_ms))
    eager = {"ms_per_step": ms_step, "value": pairs / (ms_step * 1e-3)}

    graph, graph_error, graph_step = None, None, None
    if not args.no_graph:
        # the launches before the search (selection on this stream, window
        # statistics on the second) captured once as a HIP graph and replayed
        # each step; the search stays a plain launch between HIP events.  If
        # capture fails, or a replay differs from the eager step, the eager
        # timing above stands and the reason is reported.
        try:
            ref_disp = disp.clone()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                g_centers, _ = nrr.select_and_window_stats(ref, flt, b, stride, frac, w,
                                                           select_workspace=sel_ws,
                                                           match_workspace=mat_ws)
            torch.cuda.synchronize()

            def gstep(ev=None):
                g.replay()
                if ev is not None:
                    ev[2].record(stream)
                nrr.block_match(ref, flt, g_centers, b, w, workspace=mat_ws,
                                out=(disp, ncc, conf), prepared=True)
                if ev is not None:
                    ev[3].record(stream)

            for _ in range(args.warmup):
                gstep()
            torch.cuda.synchronize()
            if not (torch.equal(g_centers.cpu(), centers.cpu()) and torch.equal(disp, ref_disp)):
                raise RuntimeError("a graph replay differs from the eager step")
            g_ms = host_ms(gstep)
            gevs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(4))
                    for _ in range(args.steps)]
            torch.cuda.synchronize()
            for ev in gevs:
                gstep(ev)
            torch.cuda.synchronize()
            g_search = np.array([ev[2].elapsed_time(ev[3]) for ev in gevs])
            graph_step = {"ms_per_step": g_ms, "value": pairs / (g_ms * 1e-3)}
            # the faster of the two launch forms is the step's time
            graph = g_ms < ms_step
            if graph:
                ms_step, search_ms, kern_ms = g_ms, g_search, float(np.mean(g_search))
        except Exception as e:  # noqa: BLE001 - reported in the JSON line
            graph_error = "%s: %s" % (type(e).__name__, e)
            torch.cuda.synchronize()

    lat = []
    for _ in range(args.latency_reps):
        t = time.perf_counter()
        c, _ = nrr.select_and_window_stats(ref, flt, b, stride, frac, w,
                                           select_workspace=sel_ws, match_workspace=mat_ws)
        nrr.block_match(ref, flt, c, b, w, workspace=mat_ws, out=(disp, ncc, conf),
                        prepared=True)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)

    achieved = OPS_PER_PAIR * pairs / (kern_ms * 1e-3) / 1e12
    arith = nrr.match_plan(dt_code, dims, b, w)["form"]
    if arith == "mfma":
        # fp16 matrix-core products of exact 12-bit offsets: measured against
        # the fp16 MFMA peak, with the FP32-vector fraction beside it
        roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_F16_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_F16_TFLOPS,
                    "traffic": measured_traffic(args.workload, arith),
                    "kernel": "k_match_mfma<%d>" % b,
                    "fp32_vector_equivalent": {"peak": PEAK_TOPS, "unit": "TOP/s",
                                               "frac": achieved / PEAK_TOPS}}
        dtype = "f16"
    else:
        roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TOPS, "unit": "TOP/s",
                    "frac": achieved / PEAK_TOPS,
                    "traffic": measured_traffic(args.workload, arith),
                    "kernel": "k_match_u16" if dt_code == nrr.U16 else "k_match_f32"}
        dtype = ("int32" if arith == "dot2" else "f32")
    result = {
        "metric": "NCC voxel-pairs/s (block matching) at 1 GPU; p50/p99 registration latency",
        "value": pairs / (ms_step * 1e-3),
        "unit": "voxel-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "dims_xyz": list(dims), "block": b,
                   "stride": stride, "fraction": frac, "window": w, "blocks": k,
                   "evaluated_pairs": pairs, "nominal_pairs": nominal, "seed": args.seed},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "reps": args.latency_reps,
                       "what": "select_and_window_stats + block_match(prepared), enqueue "
                               "to stream sync"},
        "step_launch": "graph (selection + statistics captured once) + search launch"
                       if graph else "eager (faster than the graph replay here)"
                       if graph_step else "eager",
        "graph_error": graph_error,
        "eager_step": eager,
        "graph_step": graph_step,
        "search_kernel_ms": kern_ms,
        "search_kernel_ms_median": float(np.median(search_ms)),
        "search_pairs_per_s": pairs / (kern_ms * 1e-3),
        "selection_ms": {"mean": float(np.mean(select_ms)), "median": float(np.median(select_ms)),
                         "what": "selection and window statistics, side by side in one "
                                 "call (nrr_select_and_window_stats), eager steps"},
        "search_arith": arith,
        "roofline": roofline,
        "paper_context": PAPER_CONTEXT,
    }
    if args.cpu_budget > 0:
        print("# timing the oracle (%.0f s budget)" % args.cpu_budget, file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(pair, centers_h, b, w, args.cpu_budget)
    print(json.dumps(result), flush=True)
    return 0


def bench_batched(args) -> int:
    """32 parameter sets (block, window, fraction; stride = block) over the
    64^3 float pair: one step = one batch (window statistics per block size,
    one selection launch, one persistent search launch) replayed from a HIP
    graph, against the same 32 sets as 32 sequential plain calls
    (select_blocks + block_match each)."""
    import torch

    import paper_2308_10868_amd as nrr
    from paper_2308_10868_amd import synth

    pair = synth.gen_translation_f32(seed=args.seed)
    sets = synth.gen_param_sets(32, seed=1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ref, flt = to_dev(pair.ref, torch), to_dev(pair.flt, torch)
    dims = pair.dims
    # tile tuner: one trial per distinct (block, window) on that set's blocks
    tuned = {}
    for b, w, stride, frac in sets:
        if (b, w) in tuned:
            continue
        c = nrr.select_blocks(ref, b, stride, frac)
        if c.shape[0] == 0:
            continue
        tuned[(b, w)] = nrr.tune_match(ref, flt, c, b, w, reps=2)
    plan = nrr.BatchPlan(ref, flt, sets, use_graph=True)
    eager = nrr.BatchPlan(ref, flt, sets, use_graph=False)
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    pairs = 0
    blocks = 0
    for (b, w, stride, frac), (c, d, n, cf) in zip(sets, plan.results()):
        ch = c.cpu().numpy()
        pairs += evaluated_pairs(ch, dims, b, w)
        blocks += len(ch)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps

    stream = torch.cuda.current_stream(dev)
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ea.record(stream)
    ms_graph = timed(plan.run, args.steps)
    eb.record(stream)
    torch.cuda.synchronize()
    ms_graph_ev = ea.elapsed_time(eb) / args.steps
    ms_eager = timed(eager.run, args.steps)

    def sequential():
        for b, w, stride, frac in sets:
            c = nrr.select_blocks(ref, b, stride, frac)
            nrr.block_match(ref, flt, c, b, w)

    for _ in range(args.warmup):
        sequential()
    ms_seq = timed(sequential, max(1, args.steps // 4))
    achieved = OPS_PER_PAIR * pairs / (ms_graph_ev * 1e-3) / 1e12
    result = {
        "metric": "NCC voxel-pairs/s (block matching) at 1 GPU; p50/p99 registration latency",
        "value": pairs / (ms_graph * 1e-3),
        "unit": "voxel-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": BATCHED, "dims_xyz": list(dims), "sets": len(sets),
                   "param_sets": sets, "blocks": blocks, "evaluated_pairs": pairs,
                   "seed": args.seed, "graph": True},
        "batched_eager_ms": ms_eager,
        "sequential": {"ms_per_step": ms_seq, "value": pairs / (ms_seq * 1e-3),
                       "what": "32 x (select_blocks + block_match)"},
        "speedup_vs_sequential": ms_seq / ms_graph,
        "tuned_shapes": {"%d,%d" % k: v[0] for k, v in tuned.items()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_TOPS, "traffic": None,
                     "kernel": "whole batch graph (window statistics, selection, search)"},
    }
    if args.cpu_budget > 0:
        # the oracle on a bounded sample: blocks of the most expensive set
        i = max(range(len(sets)), key=lambda j: sets[j][0] ** 3 * (2 * sets[j][1] + 1) ** 3
                * (plan.offsets[j + 1] - plan.offsets[j]))
        b, w = sets[i][0], sets[i][1]
        ch = plan.results()[i][0].cpu().numpy()
        result["cpu_baseline"] = cpu_baseline(pair, ch, b, w, args.cpu_budget)
    plan.close()
    eager.close()
    print(json.dumps(result), flush=True)
    return 0


def bench_aniso(args) -> int:
    """The MRI pair with per-axis sizes: selection, window statistics and the
    general (any block shape) search, one step per pass."""
    import torch

    import paper_2308_10868_amd as nrr

    b, st, frac, w = (ANISO_CFG[k] for k in ("block", "stride", "fraction", "window"))
    pair = make_pair("mri", args.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ref, flt = to_dev(pair.ref, torch), to_dev(pair.flt, torch)
    dims = pair.dims
    sel_b, mat_b = nrr.aniso_workspace_bytes(nrr.U16, dims, b, st)
    sel_ws = torch.empty(sel_b, dtype=torch.uint8, device=dev)
    mat_ws = torch.empty(mat_b, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev_a=None, ev_b=None):
        centers = nrr.select_blocks_aniso(ref, b, st, frac, workspace=sel_ws)
        nrr.window_stats_aniso(flt, b, workspace=mat_ws)
        if ev_a is not None:
            ev_a.record(stream)
        out = nrr.block_match_aniso(ref, flt, centers, b, w, workspace=mat_ws, prepared=True)
        if ev_b is not None:
            ev_b.record(stream)
        return centers, out

    for _ in range(args.warmup):
        centers, _ = step()
    torch.cuda.synchronize()
    centers_h = centers.cpu().numpy()
    pairs = evaluated_pairs(centers_h, dims, b, w)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for ea, eb in evs:
        step(ea, eb)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t) * 1e3 / args.steps
    kern_ms = float(np.mean([ea.elapsed_time(eb) for ea, eb in evs]))
    achieved = OPS_PER_PAIR * pairs / (kern_ms * 1e-3) / 1e12
    result = {
        "metric": "NCC voxel-pairs/s (block matching) at 1 GPU",
        "value": pairs / (ms_step * 1e-3),
        "unit": "voxel-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ANISO, "dims_xyz": list(dims), "block": list(b),
                   "stride": list(st), "fraction": frac, "window": list(w),
                   "blocks": int(len(centers_h)), "evaluated_pairs": pairs, "seed": args.seed},
        "search_kernel_ms": kern_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_TOPS, "traffic": measured_traffic(ANISO, "fma"),
                     "kernel": "k_match_aniso"},
    }
    if args.cpu_budget > 0:
        result["cpu_baseline"] = cpu_baseline(pair, centers_h, b, w, args.cpu_budget)
    print(json.dumps(result), flush=True)
    return 0


def ellipsoid_mask(shape_zyx):
    """A region for the candidates: the ellipsoid inscribed in 84-96% of the
    volume (a stand-in for the intracranial cavity), uint8 [nz][ny][nx]."""
    nz, ny, nx = shape_zyx
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    return (((x - nx / 2) / (0.42 * nx)) ** 2 + ((y - ny / 2) / (0.45 * ny)) ** 2 +
            ((z - nz / 2) / (0.48 * nz)) ** 2 <= 1.0).astype(np.uint8)


def bench_select_ex(args) -> int:
    """The selection variants alone: keys of every candidate block of the
    ref, candidates restricted to a region mask, 6-connectivity greedy in
    rank order, K from F of the masked candidates.  The MRI pair (7^3, stride
    7: 22,032 candidates, one workgroup) or the dense 512x512x256 volume
    (9^3, stride 5: 510,050 candidates, round launches; the call waits on the
    stream between rounds, so the step is timed on the host).  Roofline: HBM
    (one read of ref and of the mask at the candidate centres, keys written
    and read once)."""
    import ctypes

    import torch

    import paper_2308_10868_amd as nrr

    kind, b, st, frac, conn = SELECT_EX_CFG[args.workload]
    pair = make_pair(kind, args.seed)
    mask_h = ellipsoid_mask(pair.ref.shape)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ref = to_dev(pair.ref, torch)
    mask = torch.from_numpy(mask_h).to(dev)
    dims = pair.dims
    lib = nrr.load()
    kmax = nrr.select_count(dims, b, st, frac)
    out = torch.empty((kmax, 3), dtype=torch.int32, device=dev)
    kd = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(nrr.select_workspace_bytes(dims, b, st), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    dims3 = (ctypes.c_int32 * 3)(*dims)

    def call():
        st_ = lib.nrr_select_blocks_ex(ctypes.c_void_p(ref.data_ptr()), nrr.U16, dims3, b, st,
                                      float(frac), ctypes.c_void_p(mask.data_ptr()), conn,
                                      ctypes.c_void_p(out.data_ptr()), kmax,
                                      ctypes.c_void_p(kd.data_ptr()),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      ctypes.c_void_p(stream.cuda_stream))
        if st_ != 0:
            raise RuntimeError("nrr_select_blocks_ex failed: %d" % st_)

    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t = time.perf_counter()
    for a, e in evs:
        a.record(stream)
        call()
        e.record(stream)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t) * 1e3 / args.steps
    kern_ms = float(np.mean([a.elapsed_time(e) for a, e in evs]))
    k = int(kd.item())
    h = b // 2
    grid = [(d - b) // st + 1 for d in dims]
    ncand = grid[0] * grid[1] * grid[2]
    # algorithmic bytes: every candidate block read once from ref (the grid
    # tiles the volume: stride = edge), its mask byte, its key written and read
    nbytes = ncand * (b ** 3 * 2 + 1 + 16) + k * 12
    achieved = nbytes / (kern_ms * 1e-3) / 1e9
    result = {
        "metric": "selected-candidate throughput (block selection with mask and connectivity)",
        "value": ncand / (ms_step * 1e-3),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dims_xyz": list(dims), "block": b, "stride": st,
                   "fraction": frac, "connectivity": conn, "candidates": ncand,
                   "masked_candidates": int(mask_h[(np.arange(grid[2]) * st + h)[:, None, None],
                                                   (np.arange(grid[1]) * st + h)[None, :, None],
                                                   (np.arange(grid[0]) * st + h)[None, None, :]]
                                            .sum()),
                   "taken": k, "seed": args.seed},
        "selection_ms": kern_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0, "traffic": None,
                     "kernel": "k_block_keys_u16 + k_select_ex (one launch each)"
                     if ncand <= 24576 else
                     "k_block_keys_u16, k_ex_init, k_ex_round launches, k_ex_count, radix "
                     "select (the whole selection, host waits between rounds included)"},
    }
    if args.cpu_budget > 0:
        import oracle

        oracle.build()
        t = time.perf_counter()
        want, _ = oracle.select_ex(pair.ref, b, st, frac, mask_h, conn)
        dt = time.perf_counter() - t
        assert np.array_equal(want, out[:k].cpu().numpy()), "selection differs from the oracle"
        result["cpu_baseline"] = {"value": ncand / dt, "unit": "candidates/s",
                                  "cpu_model": cpu_model(),
                                  "cores": oracle.threads(), "kind": "oracle",
                                  "sample": "the whole workload, %.2f s" % dt}
    print(json.dumps(result), flush=True)
    return 0


def bench_serving(args) -> int:
    """Registration requests arrive as a Poisson stream (4 per second) with
    mixed volume sizes and parameters; the server admits them as slots and
    device memory free up.  Reports p50/p99 submit-to-result latency and the
    aggregate voxel-pair rate over the run, then the same requests submitted
    all at once (a saturated server) with 4 slots and with 1 slot."""
    import torch

    import paper_2308_10868_amd as nrr
    from paper_2308_10868_amd import synth

    reqs = synth.gen_serving_requests(args.requests, seed=4, rate_hz=4.0)
    pool = {}
    t0 = time.time()
    for q in reqs:
        key = (q["size"], q["volume_seed"])
        if key not in pool:
            p = synth.gen_blobs_u16(seed=1000 + q["volume_seed"], dims=q["size"], peak=(4.0, 10.0))
            pool[key] = tuple(torch.from_numpy(v.view(np.int16)).view(torch.uint16).pin_memory()
                              for v in (p.ref, p.flt))
    print("# generated %d volume pairs in %.1f s" % (len(pool), time.time() - t0),
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)

    def run(slots, paced, resident=True):
        srv = nrr.Server(device_bytes=16 << 30, slots=slots)
        # resident: every volume pair is added to the server once, before the
        # clock starts, and requests name them (the pre-operative volume of a
        # procedure stays on the device); else each request uploads its pair
        vols = {key: tuple(srv.add_volume(v) for v in pair) for key, pair in pool.items()} \
            if resident else pool
        jobs = []
        start = time.perf_counter()
        for q in reqs:
            if paced:
                delay = start + q["arrival_s"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            ref, flt = vols[(q["size"], q["volume_seed"])]
            jobs.append(srv.submit(ref, flt, q["block"], q["stride"], q["window"], q["fraction"]))
        infos = [j.wait() for j in jobs]
        wall = time.perf_counter() - start
        stats = srv.stats()
        pairs = 0
        for q, j in zip(reqs, jobs):
            pairs += evaluated_pairs(j.centers.numpy(), q["size"], q["block"], q["window"])
        srv.close()
        lat = np.array([i["total_ms"] for i in infos])
        run_ms = np.array([i["run_ms"] for i in infos])
        return {"wall_s": wall, "pairs": pairs, "value": pairs / wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "run_p50_ms": float(np.percentile(run_ms, 50)),
                "busy_frac": stats["busy_ms"] / (wall * 1e3),
                "max_running": stats["max_running"], "peak_device_bytes": stats["peak_bytes"],
                "resident_volumes": resident}

    def sequential():
        """The same requests as plain library calls, one after another on one
        stream, volumes already on the device (no server)."""
        dev = {key: tuple(v.cuda() for v in pair) for key, pair in pool.items()}
        torch.cuda.synchronize()
        start = time.perf_counter()
        for q in reqs:
            ref, flt = dev[(q["size"], q["volume_seed"])]
            c = nrr.select_blocks(ref, q["block"], q["stride"], q["fraction"])
            out = nrr.block_match(ref, flt, c, q["block"], q["window"])
            out[0].cpu()  # results to the host, as a served request's
        torch.cuda.synchronize()
        return time.perf_counter() - start

    run(4, False)  # warm-up: code objects, pinned pools
    paced = run(4, True)
    sat4 = run(4, False)
    sat1 = run(1, False)
    sat4_upload = run(4, False, resident=False)
    seq_s = sequential()
    result = {
        "metric": "NCC voxel-pairs/s (block matching) at 1 GPU; p50/p99 registration latency",
        "value": paced["value"],
        "unit": "voxel-pairs/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 1,
        "ms_per_step": paced["wall_s"] * 1e3 / len(reqs),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": SERVING, "requests": len(reqs), "rate_hz": 4.0,
                   "sizes": [list(s) for s in synth.SERVING_SIZES], "window": "5..15",
                   "block": [5, 7, 9], "fraction": "0.1..0.3", "slots": 4,
                   "device_bytes": 16 << 30, "volume_pairs": len(pool)},
        "latency_ms": {"p50": paced["p50_ms"], "p99": paced["p99_ms"],
                       "what": "submit to results in host memory (selection, kept per resident "
                               "volume and parameters, window statistics, search, download)"},
        "gpu_busy_frac": paced["busy_frac"],
        "paced": paced,
        "saturated_4_slots": sat4,
        "saturated_1_slot": sat1,
        "saturated_4_slots_uploading": sat4_upload,
        "sequential_plain_calls_s": seq_s,
        "overlap_speedup": sat1["wall_s"] / sat4["wall_s"],
        "speedup_vs_sequential_plain_calls": seq_s / sat4["wall_s"],
    }
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
