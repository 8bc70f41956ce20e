"""Launch-shape autotuner.

The generator's launch knobs (resident sampler waves per compute unit,
planner waves per compute unit, the LDS capacity of the general base case)
never change the output bits: every tile is sampled from its own stream and
written at its own offset, whichever wave takes it.  This module times a
sample of the caller's workload under each candidate setting, checks that the
bytes agree with the first candidate's, keeps the fastest, and sets it
process-wide.

What is deliberately not tuned: the chunk count P of an instance and the
tile exponent. Both shape the chunk and tile trees and therefore the bits
(P is part of an instance's definition; the tile exponent follows from n, m
or p), so tuning them would make the output depend on the machine.
"""
import itertools
import json

from . import _lib

# sampler workgroups (one wave each) per compute unit; 0 = as many as are
# resident (16: 4 per SIMD); 20 puts a few past the resident ones
DEFAULT_SAMPLE_WAVES = (0, 8, 12, 20)
DEFAULT_PLAN_WAVES = (0, 4, 8, 16)
DEFAULT_LEAF_CAP = (0, 768)


def _time_batch(kg, torch, insts, arena, offs, ws, reps):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        kg.batch(insts, arena=arena, offsets=offs, workspace=ws)
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return ms[len(ms) // 2]


def tune(instances, sample_waves=DEFAULT_SAMPLE_WAVES, plan_waves=DEFAULT_PLAN_WAVES,
         leaf_cap=DEFAULT_LEAF_CAP, reps=3, apply=True, device="cuda"):
    """Time `instances` (a list of Instance, generated as one batch) under
    every combination of the candidate knob values (0 = the library's
    default) and return {"best": {...}, "table": [...]}; with `apply` the best
    setting stays in force.  Raises if any candidate changes the bytes."""
    import torch
    import paper_1710_07565_amd as kg
    insts = list(instances)
    total = 0
    for I in insts:
        total += int(I.m) if I.model == kg.GNM else kg.gnp_count(I.n, I.p, I.directed, I.seed, I.chunks,
                                                                 device=device)
    arena = torch.empty((max(total, 1), 2), dtype=torch.uint32, device=device)
    ref = torch.empty_like(arena)
    offs = torch.empty(len(insts) + 1, dtype=torch.uint64, device=device)
    ws = torch.empty(max(kg.workspace_bytes(insts), 1), dtype=torch.uint8, device=device)
    opts = (_lib.KG_OPT_SAMPLE_WAVES, _lib.KG_OPT_PLAN_WAVES, _lib.KG_OPT_LEAF_CAP)
    saved = [kg.get_option(o) for o in opts]     # the caller's settings, restored at the end
    table = []
    try:
        for k, cand in enumerate(itertools.product(sample_waves, plan_waves, leaf_cap)):
            for o, v in zip(opts, cand):
                kg.set_option(o, v)
            arena.fill_(0)
            kg.batch(insts, arena=arena, offsets=offs, workspace=ws)     # warm-up, and the bytes
            torch.cuda.synchronize()
            if k == 0:
                ref.copy_(arena)
            elif not torch.equal(arena.view(torch.int32), ref.view(torch.int32)):
                raise RuntimeError("launch setting %s changed the output" % (cand,))
            ms = _time_batch(kg, torch, insts, arena, offs, ws, reps)
            table.append({"sample_waves": cand[0], "plan_waves": cand[1], "leaf_cap": cand[2], "ms": ms})
    finally:
        for o, v in zip(opts, saved):
            kg.set_option(o, v)
    best = min(table, key=lambda r: r["ms"])
    if apply:
        kg.set_option(_lib.KG_OPT_SAMPLE_WAVES, best["sample_waves"])
        kg.set_option(_lib.KG_OPT_PLAN_WAVES, best["plan_waves"])
        kg.set_option(_lib.KG_OPT_LEAF_CAP, best["leaf_cap"])
    return {"best": best, "table": table, "edges": total}


# ---------------------------------------------------------------------------
# The chunk-count table.  P shapes the chunk tree and therefore the bits, so
# it is not tuned per process: this offline run times every candidate on
# seeded probe instances of each table cell and writes the winners to a JSON
# file that is committed with the package (workloads.POLICY_PATH); the
# batched and served workloads then read P from that file.
# ---------------------------------------------------------------------------
P_DIRECTED = (1, 2, 4, 8, 16, 64)
P_UNDIRECTED = (1, 2, 4, 8, 16, 32, 64)


def tune_chunk_policy(out_path, log2n=(10, 24), log2d=(1, 6), probes=4, reps=3, tie=0.03, device="cuda",
                      progress=None):
    """Time every candidate P on `probes` seeded instances of every cell
    (both models and directions, floor(log2 n) in log2n, floor(log2 degree)
    in log2d), generated as one kg_batch; keep the fastest (any candidate
    within `tie` of it: the smallest such P); check that all probes of a cell
    give the same bytes as the same instances generated one call each.
    Writes the table to out_path and returns it."""
    import platform
    import time

    import torch
    import paper_1710_07565_amd as kg
    from . import workloads as W
    table = {}
    detail = {}
    t_start = time.time()
    cells = W.policy_cells(log2n, log2d)
    for ci, (model, directed, ln, ld) in enumerate(cells):
        probes_ = W.policy_probe(model, directed, ln, ld, count=probes, seed_fn=kg.instance_seed)
        cands = [P for P in (P_DIRECTED if directed else P_UNDIRECTED) if P <= 2 ** ln]
        times = {}
        for P in cands:
            insts = [W.make_instance(n, d, directed, model, seed, P=P) for (n, d, seed) in probes_]
            kinsts = [kg.Instance(I.n, I.model, I.directed, I.m, I.p, I.seed, I.chunks) for I in insts]
            total = 0
            for I in kinsts:
                total += int(I.m) if I.model == kg.GNM else kg.gnp_count(I.n, I.p, I.directed, I.seed, I.chunks,
                                                                         device=device)
            arena = torch.empty((max(total, 1), 2), dtype=torch.uint32, device=device)
            offs = torch.empty(len(kinsts) + 1, dtype=torch.uint64, device=device)
            ws = torch.empty(max(kg.workspace_bytes(kinsts), 1), dtype=torch.uint8, device=device)
            kg.batch(kinsts, arena=arena, offsets=offs, workspace=ws)
            torch.cuda.synchronize()
            times[P] = _time_batch(kg, torch, kinsts, arena, offs, ws, reps)
            del arena, offs, ws
        torch.cuda.empty_cache()
        best = min(times.values())
        pick = min(P for P, t in times.items() if t <= best * (1.0 + tie))
        key = W.policy_key(model, directed, ln, ld)
        table[key] = pick
        detail[key] = {str(P): round(t, 4) for P, t in times.items()}
        if progress:
            progress("%d/%d %s -> P=%d %s (%.0f s)" % (ci + 1, len(cells), key, pick, detail[key],
                                                     time.time() - t_start))
    torch.cuda.empty_cache()
    dev = torch.cuda.get_device_properties(0)
    tab = {"version": 1,
           "key": "model/direction/floor(log2 n)/floor(log2 mean degree)",
           "log2n": list(log2n), "log2d": list(log2d),
           "candidates": {"directed": list(P_DIRECTED), "undirected": list(P_UNDIRECTED)},
           "rule": "fastest median of %d kg_batch calls on %d seeded probe instances per cell; ties within %.0f%% "
                   "go to the smaller P" % (reps, probes, 100 * tie),
           "measured_on": "%s (%s), %s" % (dev.name, getattr(dev, "gcnArchName", "?"), platform.node()),
           "P": table, "ms": detail}
    with open(out_path, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    return tab


def main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="offline tuning of the chunk-count table")
    ap.add_argument("--chunk-policy", action="store_true", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--probes", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    tune_chunk_policy(args.out, probes=args.probes, reps=args.reps,
                      progress=lambda msg: print(msg, file=sys.stderr, flush=True))


if __name__ == "__main__":
    main()
