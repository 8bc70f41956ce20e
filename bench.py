"""Benchmark of the MI355X Erdos-Renyi generator (one GPU).

Default workload: undirected G(n,m), n = 2^26 vertices, m = 2^31 edges from
the strict upper triangle, P = 256 sections (a 256 x 256 chunk grid of 2^16
cells, 32,896 triangle chunks), seeds 1..3 in turn, uint32 (u,v) output.
One step = one kg_gnm call: chunk counts, offsets, tile plan and sampling of
all 2^31 edges into a preallocated 16 GiB buffer resident in HBM.

Prints ONE JSON line: edges/s (value), the sampler's achieved HBM write
bandwidth against the 8 TB/s peak (roofline), and the CPU oracle timed on a
bounded sample of the same workload on this host (cpu_baseline).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_EDGE = 8

WORKLOADS = {
    # name: (description, n, m, p, directed, P, model)
    "gnm_undirected_n26_m31": ("undirected G(n,m) n=2^26 m=2^31 P=256 sections (32896 chunks)",
                               2**26, 2**31, 0.0, False, 256, 0),
    "gnm_directed_n16_m20": ("directed G(n,m) n=2^16 m=2^20 P=64 chunks", 2**16, 2**20, 0.0, True, 64, 0),
    "gnp_directed_n25_d16": ("directed G(n,p) n=2^25 p=16/(n-1) P=2^16 chunks",
                             2**25, 0, 16.0 / (2**25 - 1), True, 2**16, 1),
    "gnp_undirected_n25_d64": ("undirected G(n,p) n=2^25 p=64/(n-1) P=256 sections",
                               2**25, 0, 64.0 / (2**25 - 1), False, 256, 1),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    # the sources of the sampler's code (the host file only launches it)
    for f in ("kg_device.hpp", "kg_kernels.hpp", "kg_tile.hpp"):
        with open(os.path.join(ROOT, "paper_1710_07565_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "tile_kernel_traffic.json")
ROOFLINE_KERNEL = "tile_kernel"


def traffic_for(workload):
    """HBM bytes per tile_kernel launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    path = TRAFFIC_PATH
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload)
    if not ent or ent.get("kernel_source") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def _pmc_per_dispatch(run_dir, counter):
    """{(dispatch id, kernel name): summed counter value} from rocprofv3 CSVs."""
    import csv
    import glob
    out = {}
    for path in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
    return out


def write_traffic(workload, fetch_dir, write_dir, copy_gib, commands):
    """Scale the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of
    tile_kernel by what the same counters read for the calibration copy
    (copy_gib GiB read and written) and record the HBM bytes per launch."""
    res = {}
    for ctr, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = _pmc_per_dispatch(d, ctr)
        copies = [v for (i, nm), v in per.items() if "copyBuffer" in nm or "copy" in nm.lower()]
        tiles = [v for (i, nm), v in per.items() if ROOFLINE_KERNEL in nm]
        if not copies or not tiles:
            raise SystemExit("no %s records for the copy kernel and %s in %s" % (ctr, ROOFLINE_KERNEL, d))
        scale = copy_gib * 2**20 / max(copies)          # KiB expected / KiB counted
        res[ctr] = {"raw_kib_per_launch": sum(tiles) / len(tiles), "launches": len(tiles),
                    "copy_kib": max(copies), "scale": scale}
    total = sum(v["raw_kib_per_launch"] * v["scale"] * 1024 for v in res.values())
    try:
        with open(TRAFFIC_PATH) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec[workload] = {"kernel": ROOFLINE_KERNEL, "kernel_source": kernel_source_hash(), "bytes_per_launch": total,
                     "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"], "calibration_copy_gib": copy_gib,
                     "commands": commands}
    with open(TRAFFIC_PATH, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    log("traffic for %s: %.4g bytes per launch" % (workload, total))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(desc, seconds):
    """The oracle (plain C, OpenMP over chunks) on a bounded sample of the
    same workload: whole chunks in canonical order, blocks of 256, until
    `seconds` have passed; the count pass is charged pro rata."""
    import numpy as np
    from oracle import kgref
    _, n, m, p, directed, P, model = desc
    I = kgref.inst(n, m=m, p=p, directed=directed, seed=1, chunks=P, model=model)
    threads = kgref.max_threads()
    t0 = time.perf_counter()
    counts = kgref.chunk_counts(I)
    t_counts = time.perf_counter() - t0
    C = len(counts)
    buf = np.zeros((int(counts[:256].sum()) * 2 + 1024, 2), dtype=np.uint32)
    edges = 0
    done = 0
    t_gen = 0.0
    # spread the sampled blocks over the chunk grid
    starts = list(range(0, C, 256))
    order = starts[::7] + [s for i, s in enumerate(starts) if i % 7]
    for c0 in order:
        c1 = min(C, c0 + 256)
        need = int(counts[c0:c1].sum())
        if buf.shape[0] < need:
            buf = np.zeros((need, 2), dtype=np.uint32)
        t0 = time.perf_counter()
        r = kgref.generate_chunks(I, counts, c0, c1, out=buf, threads=threads)
        t_gen += time.perf_counter() - t0
        edges += len(r)
        done += c1 - c0
        if t_gen >= seconds:
            break
    t = t_gen + t_counts * done / C
    # one thread, on a short stretch of the same chunk order
    e1, t1 = 0, 0.0
    for c0 in order[:8]:
        c1 = min(C, c0 + 32)
        t0 = time.perf_counter()
        r = kgref.generate_chunks(I, counts, c0, c1, out=buf, threads=1)
        t1 += time.perf_counter() - t0
        e1 += len(r)
        if t1 >= seconds / 5:
            break
    return {"value": edges / t, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d of %d chunks (%d edges, %.1f s), seed 1" % (done, C, edges, t),
            "one_thread": {"value": e1 / t1, "unit": "edges/s", "edges": e1, "seconds": t1}}


def run_plain(args, desc):
    import torch
    import paper_1710_07565_amd as kg
    name, n, m, p, directed, P, model = (args.workload,) + desc[1:]
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    seeds = [1, 2, 3]
    if model == 0:
        cap = m
    else:
        mean = p * (n * (n - 1) // (1 if directed else 2))
        cap = int(mean + 12 * mean ** 0.5 + 1024)
    inst = kg.Instance(n, model, directed, m, p, 1, P)
    ws = torch.empty(kg.workspace_bytes([inst]), dtype=torch.uint8, device=dev)
    out = torch.empty((cap, 2), dtype=torch.uint32, device=dev)
    total = torch.zeros(1, dtype=torch.uint64, device=dev)
    stream = torch.cuda.current_stream()

    def step(i):
        seed = seeds[i % len(seeds)]
        if model == 0:
            kg.gnm(n, m, directed, seed, P, out=out, workspace=ws, stream=stream)
        else:
            kg.gnp(n, p, directed, seed, P, out=out, total=total, workspace=ws, stream=stream)

    log("bench: %s, warmup %d, steps %d" % (desc[0], args.warmup, args.steps))
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    edges_per_step = []
    for i in range(args.steps):
        if model == 0:
            edges_per_step.append(m)
        else:
            edges_per_step.append(kg.gnp_count(n, p, directed, seeds[i % len(seeds)], P, workspace=ws))
    torch.cuda.synchronize()
    # the timed steps: one kg_gnm / kg_gnp call each, nothing else enqueued
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step(i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0].elapsed_time(ev[-1])
    per_step = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    # the same steps again with every kernel launch bracketed by HIP events
    # recorded on the launch stream (the per-kernel split and the sampler's
    # launch time for the roofline)
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 1)
    for k in range(5):
        kg.kernel_time_read(k)
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    for i in range(args.steps):
        step(i)
    f1.record(stream)
    torch.cuda.synchronize()
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 0)
    ms_split = f0.elapsed_time(f1)
    kt = {nm: kg.kernel_time_read(k) for k, nm in ((0, "count"), (1, "scan"), (2, "plan"), (3, "sample"),
                                                   (4, "queue"))}
    if model == 1:
        got = int(total.view(torch.int64).item())
        assert got == edges_per_step[(args.steps - 1) % len(edges_per_step)], "edge total mismatch"
    E = sum(edges_per_step)
    ms_per_step = ms / args.steps
    samp_ms, samp_n = kt["sample"]
    samp_avg = samp_ms / max(samp_n, 1)
    bytes_per_launch = BYTES_PER_EDGE * E / args.steps
    achieved = bytes_per_launch / (samp_avg * 1e-3) / 1e9
    traffic = traffic_for(name)
    res = {
        "metric": "edges/sec and % HBM write BW, 1 GPU; batched vs plain; p50/p99 latency served",
        "value": E / (ms * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": per_step[len(per_step) // 2], "ms_per_step_min": per_step[0],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc[0], "n": n, "m": m, "p": p, "directed": directed, "P": P,
                   "seeds": seeds, "edges_per_step": E // args.steps},
        "pct_hbm_write_bw": 100.0 * BYTES_PER_EDGE * E / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ROOFLINE_KERNEL, "avg_launch_ms": samp_avg,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "kernels_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "kernel_split_pass_ms_per_step": ms_split / args.steps,
        "wall_s_timed": wall,
    }
    return res


def batch_totals(kg, insts, dev):
    """Edges of every instance, from one kg_batch call with an empty arena
    (counts and offsets only; nothing is written)."""
    import torch
    ws = torch.empty(kg.workspace_bytes(insts), dtype=torch.uint8, device=dev)
    offs = torch.empty(len(insts) + 1, dtype=torch.uint64, device=dev)
    empty = torch.empty((0, 2), dtype=torch.uint32, device=dev)
    kg.batch(insts, arena=empty, offsets=offs, workspace=ws)
    o = offs.view(torch.int64).cpu().numpy()
    return [int(o[i + 1] - o[i]) for i in range(len(insts))]


def run_batch(args):
    """4096 uneven instances (n log-uniform in [2^10, 2^22], mean degree
    uniform in [2, 64], half directed, half G(n,m)), per-instance seeds from
    the base seed, generated in waves that fit the arena: one recorded HIP
    graph per wave (kg_batch_upload + kg_batch_launch) replayed, and the same
    waves issued as eager kg_batch calls for comparison."""
    import torch
    import paper_1710_07565_amd as kg
    from paper_1710_07565_amd import workloads
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    specs = workloads.batch_instances(args.instances, base_seed=1, seed_fn=kg.instance_seed)
    insts = [kg.Instance(s.n, s.model, s.directed, s.m, s.p, s.seed, s.chunks) for s in specs]
    tot = batch_totals(kg, insts, dev)
    # two streams, each with its own arena of half the budget: one wave's
    # count / scan / plan kernels overlap the other wave's sampler
    nstreams = 2
    arena_edges = int(args.arena_gib * 2**30) // 8 // nstreams
    waves, cur, acc = [], [], 0
    for i, e in enumerate(tot):
        if cur and acc + e > arena_edges:
            waves.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += e
    if cur:
        waves.append(cur)
    E = sum(tot)
    log("bench: batch of %d instances, %d edges (%.1f GB), %d waves of <= %.0f GiB on %d streams"
        % (len(insts), E, 8 * E / 1e9, len(waves), args.arena_gib / nstreams, nstreams))
    need = min(arena_edges, max(sum(tot[i] for i in w) for w in waves))
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    arenas = [torch.empty((need, 2), dtype=torch.uint32, device=dev) for _ in range(nstreams)]
    arena = arenas[0]
    wsmax = max(kg.workspace_bytes([insts[i] for i in w]) for w in waves)
    wss = [torch.empty(wsmax, dtype=torch.uint8, device=dev) for _ in range(nstreams)]
    ws = wss[0]
    offss = [torch.empty(len(insts) + 1, dtype=torch.uint64, device=dev) for _ in range(nstreams)]
    offs = offss[0]
    torch.cuda.synchronize()

    def eager_pass():
        for j, w in enumerate(waves):
            k = j % nstreams
            kg.batch([insts[i] for i in w], arena=arenas[k], offsets=offss[k], workspace=wss[k], stream=streams[k])

    tuning = None
    if not args.no_tune:
        # launch shapes from the autotuner, timed on a spread of the instances
        # (bit-invariant; recorded graphs keep the shapes in force at capture)
        from paper_1710_07565_amd import tune
        pick = [insts[i] for i in range(0, len(insts), max(1, len(insts) // 64))]
        res = tune.tune(pick, device=dev)
        tuning = {"sample_instances": len(pick), "sample_edges": res["edges"], "best": res["best"],
                  "candidates": len(res["table"])}
        log("bench: tuned launch shape %s" % (res["best"],))
    # one HIP graph per wave, recorded once (descriptor table uploaded into a
    # workspace of its own), replayed on the wave's stream
    graphs = []
    for j, w in enumerate(waves):
        k = j % nstreams
        wl = [insts[i] for i in w]
        wsj = torch.empty(kg.workspace_bytes(wl), dtype=torch.uint8, device=dev)
        offj = torch.empty(len(wl) + 1, dtype=torch.uint64, device=dev)
        graphs.append(kg.BatchGraph(wl, arenas[k], offj, wsj))
    torch.cuda.synchronize()
    log("bench: %d wave graphs recorded" % len(graphs))

    def graph_pass():
        for j, g in enumerate(graphs):
            with torch.cuda.stream(streams[j % nstreams]):
                g.replay()

    def timed(one_pass):
        for _ in range(args.warmup):
            one_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one_pass()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    ms_eager = timed(eager_pass)
    ms = timed(graph_pass)
    # sampler launch times from the eager pass (graph replays carry no events)
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 1)
    kg.kernel_time_read(3)
    eager_pass()
    torch.cuda.synchronize()
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 0)
    samp_ms, samp_n = kg.kernel_time_read(3)
    del graphs
    # the same instances one call at a time (a sample, for the batching gain)
    sample = list(range(0, len(insts), max(1, len(insts) // 256)))
    one = torch.empty((max(tot[i] for i in sample), 2), dtype=torch.uint32, device=dev)
    tot1 = torch.zeros(1, dtype=torch.uint64, device=dev)
    ws1 = torch.empty(max(kg.workspace_bytes([insts[i]]) for i in sample), dtype=torch.uint8, device=dev)

    def singles():
        for i in sample:
            I = insts[i]
            if I.model == kg.GNM:
                kg.gnm(I.n, I.m, I.directed, I.seed, I.chunks, out=one, workspace=ws1)
            else:
                kg.gnp(I.n, I.p, I.directed, I.seed, I.chunks, out=one, total=tot1, workspace=ws1)
    singles()
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    singles()
    f1.record()
    torch.cuda.synchronize()
    ms_single = f0.elapsed_time(f1)
    E_sample = sum(tot[i] for i in sample)
    w_sample = [insts[i] for i in sample]
    kg.batch(w_sample, arena=arena, offsets=offs, workspace=ws)
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    kg.batch(w_sample, arena=arena, offsets=offs, workspace=ws)
    g1.record()
    torch.cuda.synchronize()
    ms_batch_sample = g0.elapsed_time(g1)
    value = E * args.steps / (ms * 1e-3)
    return {
        "metric": "edges/sec and % HBM write BW, 1 GPU; batched vs plain; p50/p99 latency served",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched: %d G(n,m)/G(n,p) instances, n log-uniform [2^10,2^22], mean degree "
                               "uniform [2,64], half directed" % len(insts),
                   "instances": len(insts), "edges_per_step": E, "waves": len(waves), "arena_gib": args.arena_gib},
        "pct_hbm_write_bw": 100.0 * BYTES_PER_EDGE * value / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": BYTES_PER_EDGE * E / (samp_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": BYTES_PER_EDGE * E / (samp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "kernel": ROOFLINE_KERNEL, "avg_launch_ms": samp_ms / max(samp_n, 1)},
        "tuning": tuning,
        "graphs": {"one_graph_replay_per_wave": True, "eager_kg_batch_edges_per_s": E * args.steps / (ms_eager * 1e-3),
                   "eager_ms_per_step": ms_eager / args.steps},
        "batching": {"sample_instances": len(sample), "sample_edges": E_sample,
                     "one_call_each_edges_per_s": E_sample / (ms_single * 1e-3),
                     "one_kg_batch_edges_per_s": E_sample / (ms_batch_sample * 1e-3)},
    }


def run_views(args):
    """The per-PE partition of the headline workload: the views of all P = 256
    sections of undirected G(n,m), n = 2^26, m = 2^31 (each off-diagonal
    chunk belongs to two views, so about twice the graph's edges), generated
    as one kg_batch of 256 view instances per step, seeds 1..3."""
    import torch
    import paper_1710_07565_amd as kg
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, m, P = 2**26, 2**31, 256
    seeds = [1, 2, 3]
    vsets = [[kg.Instance(n, kg.GNM, False, m, 0.0, sd, P, view=r + 1) for r in range(P)] for sd in seeds]
    totals = [sum(batch_totals(kg, vs, dev)) for vs in vsets]
    cap = max(totals)
    log("bench: %d views per step, %.3g view edges per step (%.3f x the graph)" % (P, totals[0], totals[0] / m))
    arena = torch.empty((cap, 2), dtype=torch.uint32, device=dev)
    offs = torch.empty(P + 1, dtype=torch.uint64, device=dev)
    # the three descriptor tables are inputs: uploaded once, each into its own
    # workspace, before the timed region; a step enqueues the kernels only
    wss = [torch.empty(kg.workspace_bytes(vs), dtype=torch.uint8, device=dev) for vs in vsets]
    for vs, w in zip(vsets, wss):
        kg.batch_upload(vs, w)

    def step(i):
        kg.batch_launch(vsets[i % 3], arena, offs, wss[i % 3])

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # kg_batch as one call per step (upload, synchronise, launch): the host's
    # descriptor work and the synchronisation sit between the steps
    e0.record()
    for i in range(args.steps):
        kg.batch(vsets[i % 3], arena=arena, offsets=offs, workspace=wss[i % 3])
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1)
    # the per-kernel split in a separate pass (HIP events around every launch)
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 1)
    for k in range(5):
        kg.kernel_time_read(k)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 0)
    kt = {nm: kg.kernel_time_read(k) for k, nm in ((0, "count"), (1, "scan"), (2, "plan"), (3, "sample"),
                                                   (4, "queue"))}
    samp_ms, samp_n = kt["sample"]
    E = sum(totals[i % 3] for i in range(args.steps))
    value = E / (ms * 1e-3)
    res = {
        "metric": "edges/sec and % HBM write BW, 1 GPU; batched vs plain; p50/p99 latency served",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "per-PE views: all 256 sections of undirected G(n,m) n=2^26 m=2^31 "
                               "(off-diagonal chunks in two views) as one batch launch",
                   "n": n, "m": m, "P": P, "seeds": seeds, "view_edges_per_step": totals[0]},
        "pct_hbm_write_bw": 100.0 * BYTES_PER_EDGE * value / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": BYTES_PER_EDGE * E / (samp_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": BYTES_PER_EDGE * E / (samp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "kernel": ROOFLINE_KERNEL, "avg_launch_ms": samp_ms / max(samp_n, 1)},
        "kernels_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in kt.items()},
        "ms_per_step_kg_batch_with_upload": ms_eager / args.steps,
    }
    if not args.no_cpu_baseline:
        # the oracle's view of a few sections (each PE's work in the paper's run)
        import time as _t
        from oracle import kgref
        I = kgref.inst(n, m=m, directed=False, seed=1, chunks=P)
        t0, done, cnt = _t.perf_counter(), 0, 0
        for r in range(0, P, 37):
            cnt += len(kgref.pe_view(I, r))
            done += 1
            if _t.perf_counter() - t0 > args.cpu_seconds:
                break
        dt = _t.perf_counter() - t0
        res["cpu_baseline"] = {"value": cnt / dt, "unit": "edges/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": "%d of %d views (%d edges, %.1f s), one thread" % (done, P, cnt, dt)}
    else:
        res["cpu_baseline"] = None
    return res


def run_skip(args):
    """The geometric-skip G(n,p) variant on the directed workload (n = 2^25,
    p = 16/(n-1), 2^16 chunks, seeds 1..3) next to the main path's G(n,p) on
    the same parameters: same law, different sampler and bits."""
    import torch
    import paper_1710_07565_amd as kg
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, P = 2**25, 2**16
    p = 16.0 / (n - 1)
    seeds = [1, 2, 3]
    inst = kg.Instance(n, kg.GNP, True, 0, p, 1, P)
    # room for the count pass's event positions (one row per tile); the
    # plain G(n,p) workspace size makes the write pass generate them again
    ws = torch.empty(kg.gnp_skip_workspace_bytes(n, p, True, P), dtype=torch.uint8, device=dev)
    ws_small = ws[:kg.workspace_bytes([inst])]
    tot = torch.zeros(1, dtype=torch.uint64, device=dev)
    E = []
    for sd in seeds:
        kg.gnp_skip(n, p, True, sd, P, out=torch.empty((0, 2), dtype=torch.uint32, device=dev), total=tot,
                    workspace=ws)
        E.append(int(tot.view(torch.int64).cpu()[0]))
    # the main path's totals differ (another sampler): the buffer holds both
    E_main = [kg.gnp_count(n, p, True, sd, P, workspace=ws) for sd in seeds]
    out = torch.empty((max(E + E_main), 2), dtype=torch.uint32, device=dev)

    def timed(fn):
        for i in range(args.warmup):
            fn(seeds[i % 3])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(args.steps):
            fn(seeds[i % 3])
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 1)
    for k in range(5):
        kg.kernel_time_read(k)
    ms = timed(lambda sd: kg.gnp_skip(n, p, True, sd, P, out=out, total=tot, workspace=ws))
    cnt_ms, cnt_n = kg.kernel_time_read(2)
    wr_ms, wr_n = kg.kernel_time_read(3)
    ms_regen = timed(lambda sd: kg.gnp_skip(n, p, True, sd, P, out=out, total=tot, workspace=ws_small))
    rcnt_ms, rcnt_n = kg.kernel_time_read(2)
    rwr_ms, rwr_n = kg.kernel_time_read(3)
    ms_main = timed(lambda sd: kg.gnp(n, p, True, sd, P, out=out, total=tot, workspace=ws))
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 0)
    Etot = sum(E[i % 3] for i in range(args.steps))
    value = Etot / (ms * 1e-3)
    res = {
        "metric": "edges/sec and % HBM write BW, 1 GPU; batched vs plain; p50/p99 latency served",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "directed G(n,p) n=2^25 p=16/(n-1) P=2^16 chunks by geometric skips per tile",
                   "n": n, "p": p, "P": P, "seeds": seeds, "edges_per_step": E[0]},
        "pct_hbm_write_bw": 100.0 * BYTES_PER_EDGE * value / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm",
                     "limited_by": "write pass: the stored positions read (4 B per edge) and the edges written; "
                                   "count pass: FP64 log and divide per gap (VALU)",
                     "kernel": "skip_emit_kernel",
                     "avg_launch_ms": wr_ms / max(wr_n, 1), "count_pass_ms": cnt_ms / max(cnt_n, 1),
                     # per launch: the timers also saw the warm-up launches
                     "achieved": BYTES_PER_EDGE * (sum(E) / 3) / (wr_ms / max(wr_n, 1) * 1e-3) / 1e9,
                     "unit": "GB/s", "peak": HBM_PEAK_GBS,
                     "frac": BYTES_PER_EDGE * (sum(E) / 3) / (wr_ms / max(wr_n, 1) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "positions_generated_again": {"ms_per_step": ms_regen / args.steps,
                                      "count_pass_ms": rcnt_ms / max(rcnt_n, 1),
                                      "write_pass_ms": rwr_ms / max(rwr_n, 1),
                                      "workspace_bytes": ws_small.numel()},
        "workspace_bytes": ws.numel(),
        "main_path_same_parameters": {"ms_per_step": ms_main / args.steps,
                                      "edges_per_s": sum(E_main[i % 3] for i in range(args.steps)) / (ms_main * 1e-3)},
    }
    if not args.no_cpu_baseline:
        import time as _t
        from oracle import kgref
        I = kgref.inst(n, p=p, directed=True, seed=1, chunks=P, model=kgref.GNP)
        t0, c, cnt = _t.perf_counter(), 0, 0
        while _t.perf_counter() - t0 < args.cpu_seconds and c < P:
            cnt += len(kgref.skip_chunk_edges(I, c))
            c += 1
        dt = _t.perf_counter() - t0
        res["cpu_baseline"] = {"value": cnt / dt, "unit": "edges/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": "%d of %d chunks (%d edges, %.1f s), one thread" % (c, P, cnt, dt)}
    else:
        res["cpu_baseline"] = None
    return res


def kg_rgg_level(n, r, dim):
    """Level of the cell grid (the library's rule), for the workload name."""
    L, lmax = 0, 14 if dim == 2 else 10
    while L < lmax and r * 2.0 ** (L + 1) <= 1.0 and 2 ** (dim * (L + 1)) <= n:
        L += 1
    return L


def run_rgg(args, dim=2):
    """Random geometric graph (Sec. 5) in two or three dimensions: n = 2^26
    points, r = 0.55 (ln n / n)^(1/dim) (the radius of the paper's RGG
    experiments), seeds 1..3; points and edges written to HBM every step."""
    import torch
    import paper_1710_07565_amd as kg
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n = 2**26
    r = 0.55 * (math.log(n) / n) ** (1.0 / dim)
    gen = kg.rgg2d if dim == 2 else kg.rgg3d
    wsb = kg.rgg2d_workspace_bytes if dim == 2 else kg.rgg3d_workspace_bytes
    seeds = [1, 2, 3]
    ws = torch.empty(wsb(n, r), dtype=torch.uint8, device=dev)
    pts = torch.empty((n, dim), dtype=torch.float64, device=dev)
    tot = torch.zeros(1, dtype=torch.uint64, device=dev)
    E = []
    for sd in seeds:
        gen(n, r, sd, points=pts, out=torch.empty((0, 2), dtype=torch.uint32, device=dev), total=tot,
            workspace=ws)
        E.append(int(tot.view(torch.int64).cpu()[0]))
    out = torch.empty((max(E), 2), dtype=torch.uint32, device=dev)

    def step(i):
        gen(n, r, seeds[i % 3], points=pts, out=out, total=tot, workspace=ws)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # the per-kernel split in a separate pass (HIP events around every launch)
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 1)
    for k in range(5):
        kg.kernel_time_read(k)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    per = {}
    for k, name in enumerate(["tree", "scans", "edge_count_pass", "edge_write_pass", "points"]):
        t, c = kg.kernel_time_read(k)
        per[name] = t / max(c, 1) if name != "scans" else t / max(args.steps, 1)
    kg.set_option(kg._lib.KG_OPT_TIME_KERNELS, 0)
    Etot = sum(E[i % 3] for i in range(args.steps))
    value = Etot / (ms * 1e-3)
    bytes_step = [BYTES_PER_EDGE * E[i % 3] + 8 * dim * n for i in range(args.steps)]
    wr_ms = per["edge_write_pass"]
    wr_bytes = BYTES_PER_EDGE * Etot / args.steps
    cells = ("4^%d" % kg_rgg_level(n, r, dim)) if dim == 2 else ("8^%d" % kg_rgg_level(n, r, dim))
    res = {
        "metric": "edges/sec and % HBM write BW, 1 GPU; batched vs plain; p50/p99 latency served",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+u32", "data": "synthetic",
        "config": {"workload": "%dD random geometric graph n=2^26 r=0.55 (ln n/n)^(1/%d) (%s cells)" % (dim, dim, cells),
                   "n": n, "r": r, "seeds": seeds, "edges_per_step": E[0]},
        "pct_hbm_write_bw": 100.0 * sum(bytes_step) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "per_launch_ms": per,
        "roofline": {"bound": "hbm",
                     "limited_by": "per-vertex distance tests (FP64, neighbour points from L2), two passes",
                     "kernel": "rgg_edges_kernel<true>" if dim == 2 else "rgg3_edges_kernel<true>",
                     "avg_launch_ms": wr_ms,
                     "achieved": wr_bytes / (wr_ms * 1e-3) / 1e9, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                     "frac": wr_bytes / (wr_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        import time as _t
        from oracle import kgref
        # a bounded sample: the whole oracle on a 2^22-point instance of the
        # same recipe (one thread)
        ns = 2**22
        rs = 0.55 * (math.log(ns) / ns) ** (1.0 / dim)
        t0 = _t.perf_counter()
        _, Es = (kgref.rgg2d if dim == 2 else kgref.rgg3d)(ns, rs, 1)
        dt = _t.perf_counter() - t0
        res["cpu_baseline"] = {"value": len(Es) / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": "n=2^22, r=0.55 (ln n/n)^(1/%d), seed 1: %d edges in %.1f s, one thread"
                               % (dim, len(Es), dt)}
    else:
        res["cpu_baseline"] = None
    return res


def served_summary(args, duration, warmup_s, sat_rate, sat_seconds):
    """The served workload for the default line: Poisson arrivals at
    args.rate for `duration` s with the client's checks on (checksum of every
    request on the device, the length of every G(n,m) list, a 1% sample
    re-generated alone), then one saturation step at `sat_rate` for
    `sat_seconds` s (checks off)."""
    import torch
    import paper_1710_07565_amd as kg
    from paper_1710_07565_amd import serve, workloads
    torch.cuda.set_device(0)
    srv = serve.Server(budget_bytes=int(args.budget_gb * 1e9), streams=args.streams, max_batch=args.max_batch,
                       verify=True, alone_every=100)
    w = workloads.request_stream(rate_per_s=200.0, duration_s=0.5, base_seed=99, seed_fn=kg.instance_seed)
    serve.run_stream(srv, w, warmup_s=0.0)
    stream = workloads.request_stream(rate_per_s=args.rate, duration_s=duration, base_seed=1,
                                      seed_fn=kg.instance_seed)
    log("bench: serving %d requests over %.0f s at %.0f req/s (client checks on)" % (len(stream), duration,
                                                                                     args.rate))
    _, st = serve.run_stream(srv, stream, warmup_s=warmup_s)
    srv.verify = False
    srv.rejected = 0
    sat = workloads.request_stream(rate_per_s=sat_rate, duration_s=sat_seconds, base_seed=2,
                                   seed_fn=kg.instance_seed)
    log("bench: saturation step, %d requests at %.0f req/s" % (len(sat), sat_rate))
    _, s2 = serve.run_stream(srv, sat, warmup_s=min(1.0, sat_seconds / 4))
    del srv
    torch.cuda.empty_cache()
    return {"workload": "Poisson %.0f req/s for %.0f s (first %.0f s excluded), G(n,m)/G(n,p) equal mix, n "
                        "log-uniform [2^12,2^24], mean degree uniform [4,32], %.0f GB budget, %d streams"
                        % (args.rate, duration, warmup_s, args.budget_gb, args.streams),
            "edges_per_s": st["edges_per_s"], "p50_s": st["p50_s"], "p99_s": st["p99_s"],
            "requests": st["requests"], "rejected": st["rejected"], "verified": st["verified"],
            "checked_alone": st["checked_alone"], "verify_failures": st["verify_failures"],
            "saturation": {"rate_per_s": sat_rate, "seconds": sat_seconds, "edges_per_s": s2["edges_per_s"],
                           "p50_s": s2["p50_s"], "p99_s": s2["p99_s"], "requests": s2["requests"]}}


def run_serve(args):
    """Open-loop Poisson requests, continuous batching under an HBM budget."""
    import torch
    import paper_1710_07565_amd as kg
    from paper_1710_07565_amd import serve, workloads
    torch.cuda.set_device(0)
    stream = workloads.request_stream(rate_per_s=args.rate, duration_s=args.duration, base_seed=1,
                                      seed_fn=kg.instance_seed)
    log("bench: serving %d requests over %.0f s at %.0f req/s" % (len(stream), args.duration, args.rate))
    srv = serve.Server(budget_bytes=int(args.budget_gb * 1e9), streams=args.streams, max_batch=args.max_batch,
                       verify=args.verify)
    # warm up the library and allocator
    w = workloads.request_stream(rate_per_s=200.0, duration_s=0.5, base_seed=99, seed_fn=kg.instance_seed)
    serve.run_stream(srv, w, warmup_s=0.0)
    reqs, st = serve.run_stream(srv, stream, warmup_s=args.serve_warmup,
                                progress=lambda t, i, q, f: log("  t=%.0fs arrived=%d queued=%d inflight=%d"
                                                                % (t, i, q, f)))
    sweep = []
    if args.sweep:
        # saturation: double the rate until the p99 latency diverges
        rate = args.rate * 2
        while rate <= args.rate * 64:
            # the same server (one arena of the budget's size), fresh counters
            srv.rejected = 0
            st2 = serve.run_stream(srv, workloads.request_stream(rate_per_s=rate, duration_s=args.sweep_seconds,
                                                                  base_seed=2, seed_fn=kg.instance_seed),
                                   warmup_s=min(2.0, args.sweep_seconds / 4))[1]
            sweep.append({"rate_per_s": rate, "edges_per_s": st2["edges_per_s"], "p50_s": st2["p50_s"],
                          "p99_s": st2["p99_s"], "requests": st2["requests"], "span_s": st2["span_s"]})
            log("  sweep %.0f req/s: %.3g edges/s, p99 %.3f s" % (rate, st2["edges_per_s"], st2["p99_s"] or -1))
            if st2["p99_s"] is None or st2["p99_s"] > 1.0 or st2["span_s"] > 1.5 * args.sweep_seconds:
                break
            rate *= 2
    return {
        "metric": "edges/sec and % HBM write BW, 1 GPU; batched vs plain; p50/p99 latency served",
        "value": st["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": st["span_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "served: Poisson %.0f req/s for %.0f s, G(n,m)/G(n,p) equal mix, n log-uniform "
                               "[2^12,2^24], mean degree uniform [4,32], %.0f GB budget"
                               % (args.rate, args.duration, args.budget_gb)},
        "served": st,
        "saturation_sweep": sweep,
        "peak_served_edges_per_s": max([st["edges_per_s"]] + [x["edges_per_s"] for x in sweep]),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gnm_undirected_n26_m31", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "views", "skip", "rgg", "rgg3"])
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--arena-gib", type=float, default=96.0)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=256)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--no-tune", action="store_true", help="batch mode: keep the default launch shapes")
    ap.add_argument("--sweep", action="store_true", help="serve mode: also sweep the arrival rate up to saturation")
    ap.add_argument("--verify", action="store_true", help="serve mode: client checks on the device")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain mode: leave out the batched and served sub-records of the default line")
    ap.add_argument("--extras-serve-seconds", type=float, default=20.0)
    ap.add_argument("--extras-sat-rate", type=float, default=16000.0)
    ap.add_argument("--extras-sat-seconds", type=float, default=5.0)
    ap.add_argument("--sweep-seconds", type=float, default=10.0)
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first copy this many GiB device-to-device (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no run: read rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output directories of a profiled "
                         "run of this workload (with --calibrate-copy-gib) and record the tile_kernel HBM traffic "
                         "in profiles/tile_kernel_traffic.json")
    ap.add_argument("--count-lanes", type=int, default=0, choices=[0, 1, 2, 4, 8],
                    help="lanes per chunk in the count kernel (0: the library's choice; launch shape only)")
    ap.add_argument("--traffic-command", action="append", default=[],
                    help="the profiling commands, recorded with the traffic figure")
    args = ap.parse_args()
    if args.traffic_from:
        if args.calibrate_copy_gib <= 0:
            raise SystemExit("--traffic-from needs --calibrate-copy-gib (the size of the profiled calibration copy)")
        write_traffic(args.workload, args.traffic_from[0], args.traffic_from[1], args.calibrate_copy_gib,
                      args.traffic_command)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the generator needs no communication and this build "
              "measures a single MI355X (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.count_lanes:
        import paper_1710_07565_amd as kg
        kg.set_option(kg._lib.KG_OPT_COUNT_LANES, args.count_lanes)
    if args.calibrate_copy_gib > 0:
        import torch
        nb = int(args.calibrate_copy_gib * 2**30) // 4
        src = torch.ones(nb, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of %d bytes (read %d + write %d)" % (4 * nb, 4 * nb, 4 * nb))
        del src, dst
    if args.mode == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.mode == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.mode == "views":
        print(json.dumps(run_views(args)), flush=True)
        return
    if args.mode == "skip":
        print(json.dumps(run_skip(args)), flush=True)
        return
    if args.mode in ("rgg", "rgg3"):
        print(json.dumps(run_rgg(args, 2 if args.mode == "rgg" else 3)), flush=True)
        return
    desc = WORKLOADS[args.workload]
    res = run_plain(args, desc)
    if not args.no_extras and args.workload == "gnm_undirected_n26_m31":
        # the other two parts of the metric: batched (4096 instances as one
        # job) and served (continuous batching of a request stream)
        import copy
        import torch
        bargs = copy.copy(args)
        bargs.steps, bargs.warmup = 2, 1
        torch.cuda.empty_cache()
        b = run_batch(bargs)
        torch.cuda.empty_cache()
        res["batched"] = {"workload": b["config"]["workload"], "instances": b["config"]["instances"],
                          "edges_per_step": b["config"]["edges_per_step"], "waves": b["config"]["waves"],
                          "edges_per_s": b["value"], "ms_per_step": b["ms_per_step"],
                          "ratio_plain_to_batched": res["value"] / b["value"],
                          "eager_kg_batch_edges_per_s": b["graphs"]["eager_kg_batch_edges_per_s"],
                          "sampler_frac_of_hbm_peak": b["roofline"]["frac"], "tuning": b["tuning"],
                          "batching_gain": b["batching"]}
        sv = served_summary(args, args.extras_serve_seconds, min(3.0, args.extras_serve_seconds / 4),
                            args.extras_sat_rate, args.extras_sat_seconds)
        sv["ratio_plain_to_saturated"] = res["value"] / sv["saturation"]["edges_per_s"]
        res["served"] = sv
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host (%.0f s budget)" % args.cpu_seconds)
        res["cpu_baseline"] = cpu_baseline(desc, args.cpu_seconds)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
