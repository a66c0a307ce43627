"""Benchmark: one step = one resolve call of the linked-tori pair on one MI355X.

Workload: two oriented tori, 128 x 64 segments each (8192 vertices, 16384
triangles), R = 1, r = 0.3, the second rotated 90 degrees about x and
shifted 1.7 along x; float32 storage, float32-filtered predicates, both
meshes oriented (roles alternate), d = 1e-3.  Inputs are resident in HBM
before timing.  A step runs the whole path: ingest, edge sets, Morton
orders, BVH build and refit, traversal with the filtered narrow phase, the
exact tier, hit compaction and sort, stencils, constraints, impact zones,
zone solves and updates, round after round, for a fixed budget of response
rounds (--rounds, default 12).  Without the paper's displacement diffusion
this deep overlap keeps growing new intersections, so the call ends
NOT_CONVERGED with its residual hits reported; the per-call work is the
same every step.

Prints one JSON line.  `value` is narrow-phase E-F tests per second of
whole-step wall time; resolve calls per second and p50/p99 call latency are
reported beside it, plus the roofline of the dominant kernel and the CPU
oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "E-F tests/sec, resolved mesh pairs/sec; p50/p99 resolve latency (1 MI355X)"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20


def traverse_bytes(pair, ne_a: int, ne_b: int, launches_dir: dict, candidates: float) -> float:
    """Compulsory bytes of all traversal launches.

    Per launch in direction E -> F: 16 B per query edge (u, v, id), 12 B per
    edge-mesh vertex (float32 positions), 64 B per internal BVH node (each
    read at least once); plus 8 B per queued candidate (query, leaf) written.
    The leaves' vertex indices and positions are read by the narrow-phase
    kernel, not by the traversal.
    """
    nv_a, nt_a = len(pair.pos_a), len(pair.tri_a)
    nv_b, nt_b = len(pair.pos_b), len(pair.tri_b)
    per = {
        0: 16 * ne_a + 12 * nv_a + 64 * (nt_b - 1),
        1: 16 * ne_b + 12 * nv_b + 64 * (nt_a - 1),
    }
    return sum(per[d] * n for d, n in launches_dir.items()) + 8 * candidates


def measured_traffic():
    """HBM bytes per traversal launch from the committed counter record, or None.

    The record (profiles/k_traverse_hbm_counters.json) holds FETCH_SIZE and
    WRITE_SIZE per dispatch, scaled by what the same counters read for a
    256 MiB device copy, and the SHA-256 of the traversal sources it was
    taken with; a changed kernel makes the figure stale, and then it is None.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_traverse_hbm_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def progress(msg: str) -> None:
    """One line of progress on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def bench_batch(ctx, args) -> dict:
    """Resolved pairs/s of the mixed pair set: batched float32-filtered form vs the plain form.

    Batched: one hfcr_resolve_batch call over every pair (float32 storage,
    float32-filtered predicates, pairs in flight on their own streams).
    Plain: the same pairs resolved one at a time with float64 storage and the
    float64 filter.  Both use the same round budget.
    """
    import dataclasses

    import torch

    import meshgen
    import paper_1409_2081_amd as hf

    progress(f"batch: generating {args.batch_pairs} pairs")
    pairs = meshgen.pair_set(seed=4, n=args.batch_pairs)
    items = [hf.pair_item(p, "cuda:0") for p in pairs]
    plain = [hf.pair_item(dataclasses.replace(p, dtype=meshgen.F64, tier=1).cast(), "cuda:0") for p in pairs]
    kw = dict(max_rounds=args.batch_rounds, want_lists=False)
    # warm-up in chunks (creates the workers and shows where the time goes)
    t = time.perf_counter()
    for c0 in range(0, len(items), 16):
        tc = time.perf_counter()
        w = ctx.resolve_batch(items[c0:c0 + 16], tier=0, timing=True, **kw)
        sm = w["stats"]["stage_ms"]
        progress(f"batch warm-up: pairs {c0}..{c0 + 15}: {time.perf_counter() - tc:.2f} s, "
                 f"max zone {w['stats']['max_zone']}, rounds {w['stats']['rounds']}, "
                 f"solve {sm['solve']:.0f} ms, traverse {sm['traverse']:.0f} ms (summed over pairs)")
    torch.cuda.synchronize()
    progress(f"batch: warm-up took {time.perf_counter() - t:.2f} s")
    call_s = []
    for k in range(args.batch_steps):
        t = time.perf_counter()
        b = ctx.resolve_batch(items, tier=0, **kw)
        torch.cuda.synchronize()
        call_s.append(time.perf_counter() - t)
        progress(f"batch: timed call {k + 1}/{args.batch_steps}: {call_s[-1]:.3f} s")
    tb = sorted(call_s)[len(call_s) // 2]  # median call
    # per-stage GPU time from one more call with HIP events (not timed: the
    # events are extra queue operations)
    b_timed = ctx.resolve_batch(items, tier=0, timing=True, **kw)
    for it in plain[:4]:
        ctx.resolve(it["pos_a"], it["tri_a"], it["pos_b"], it["tri_b"], it["orientation"], it["d"], tier=1, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_status, plain_ms = [], []
    for k, it in enumerate(plain):
        ts = time.perf_counter()
        g = ctx.resolve(it["pos_a"], it["tri_a"], it["pos_b"], it["tri_b"], it["orientation"], it["d"], tier=1,
                        raise_on_error=False, **kw)
        plain_status.append(g["status"])
        plain_ms.append(1e3 * (time.perf_counter() - ts))
        if (k + 1) % 32 == 0:
            progress(f"plain: {k + 1}/{len(plain)} pairs, {time.perf_counter() - t:.1f} s")
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    n = len(pairs)
    st = [p["status"] for p in b["pairs"]]
    return {
        "workload": f"{n} mixed pairs (half sphere-sheet, half linked tori), triangles per mesh log-uniform "
                    f"in [500, 50000], depth U[0.1, 0.4], random rigid motions, seed 4; "
                    f"{sum(len(p.tri_a) + len(p.tri_b) for p in pairs)} triangles in all",
        "max_rounds": args.batch_rounds, "workers": ctx.get_tuning()["batch_workers"],
        "batched_pairs_per_s": n / tb, "batched_ms_per_call": 1e3 * tb,
        "batched_ms_per_call_all": [round(1e3 * x, 2) for x in call_s],
        "plain_f64_pairs_per_s": n / tp, "plain_f64_ms_total": 1e3 * tp,
        "speedup_vs_plain": tp / tb,
        "batched_converged": sum(s == hf.HFCR_OK for s in st),
        "batched_not_converged": sum(s == hf.HFCR_NOT_CONVERGED for s in st),
        "batched_failed": sum(s < 0 for s in st),
        "plain_converged": sum(s == hf.HFCR_OK for s in plain_status),
        "plain_ms_p50": sorted(plain_ms)[len(plain_ms) // 2], "plain_ms_max": max(plain_ms),
        "batched_candidates": b["stats"]["candidates"], "batched_max_zone": b["stats"]["max_zone"],
        "batched_stage_ms_summed_over_pairs": b_timed["stats"]["stage_ms"],
    }


def bench_serving(args) -> dict:
    """Open-loop serving: Poisson arrivals of resolve requests of uneven sizes.

    A pool of 64 pairs (half sphere-sheet, half linked tori, triangles per
    mesh log-uniform in [1k, 200k], seed 5) is made resident; request i
    resolves pool[i % 64] (outputs fresh per request).  The saturated
    closed-loop throughput is measured first (every request submitted at
    once); the open loop then offers 0.7 of it with exponential
    inter-arrival times (seed 5).  Latency = submission to completion.
    """
    import threading

    import numpy as np
    import torch

    import meshgen
    import paper_1409_2081_amd as hf

    progress("serving: generating the request pool")
    pool = meshgen.pair_set(seed=5, n=56, f_lo=1000.0, f_hi=200000.0)
    rng = np.random.default_rng(5)
    for k in range(8):  # body-in-garment pairs, body triangles log-uniform in [2k, 200k]
        fb = float(np.exp(rng.uniform(np.log(2000.0), np.log(200000.0))))
        pool.append(meshgen.body_garment(seed=50 + k, body_tris=int(fb), cloth_tris=int(fb / 2)))
    items = [hf.pair_item(p, "cuda:0") for p in pool]
    torch.cuda.synchronize()
    kw = dict(max_rounds=args.serve_rounds, tier=0, want_lists=False)
    srv = hf.Server(0, slots=args.serve_slots, pool_bytes=args.serve_pool_mib << 20)
    try:
        # warm-up: every pool pair once (workspaces grow to their size)
        for t in [srv.submit(it, **kw) for it in items]:
            srv.wait(t)
        progress("serving: warm-up done")
        n_sat = min(args.serve_requests, 256)
        t0 = time.perf_counter()
        ts = [srv.submit(items[i % len(items)], **kw) for i in range(n_sat)]
        for t in ts:
            srv.wait(t)
        sat = n_sat / (time.perf_counter() - t0)
        rate = 0.7 * sat
        progress(f"serving: saturated {sat:.1f} requests/s; offering {rate:.1f}/s")
        rng = np.random.default_rng(5)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, args.serve_requests))
        tickets, lat, status = [], [], []
        done = threading.Event()

        def collect():
            k = 0
            while k < args.serve_requests:
                if k >= len(tickets):
                    time.sleep(1e-4)
                    continue
                r = srv.wait(tickets[k])
                lat.append(r["latency_ms"])
                status.append(r["status"])
                k += 1
                if k % 100 == 0:
                    progress(f"serving: {k}/{args.serve_requests} requests done")
            done.set()

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i, a in enumerate(arrivals):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            tickets.append(srv.submit(items[i % len(items)], **kw))
        th.join()
        wall = time.perf_counter() - t0
    finally:
        srv.close()
    lat_s = sorted(lat)
    pick = lambda q: lat_s[min(len(lat_s) - 1, int(round(q * (len(lat_s) - 1))))]
    return {
        "workload": f"Poisson arrivals of {args.serve_requests} resolve requests over a pool of 64 pairs "
                    "(56 sphere-sheet / linked tori with triangles per mesh log-uniform in [1k, 200k], seed 5; "
                    "8 body-in-garment pairs with 2k-200k body triangles), "
                    f"max_rounds {args.serve_rounds}, float32-filtered",
        "slots": args.serve_slots, "pool_bytes": args.serve_pool_mib << 20,
        "saturated_requests_per_s": sat, "offered_requests_per_s": rate,
        "completed_requests_per_s": len(lat) / wall, "p50_ms": pick(0.5), "p99_ms": pick(0.99),
        "mean_ms": float(np.mean(lat)), "statuses": {hf.STATUS_NAMES[k]: status.count(k) for k in set(status)},
        "pool_triangles": sum(len(p.tri_a) + len(p.tri_b) for p in pool),
    }


def bench_body(ctx, args) -> dict:
    """The body-in-garment pair (about 200k body and 100k cloth triangles), resolved to convergence."""
    import torch

    import meshgen
    import paper_1409_2081_amd as hf

    progress("body-garment: generating")
    pair = meshgen.body_garment()
    tens = hf.pair_tensors(pair, "cuda:0")
    kw = dict(tier=pair.tier, max_rounds=64, want_lists=False)
    for _ in range(2):
        ctx.resolve(*tens, pair.orientation, pair.d, **kw)
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for _ in range(args.body_steps):
        ts = time.perf_counter()
        g = ctx.resolve(*tens, pair.orientation, pair.d, **kw)
        lat.append(1e3 * (time.perf_counter() - ts))
        stats.append(g["stats"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tstats = [ctx.resolve(*tens, pair.orientation, pair.d, timing=True, **kw)["stats"] for _ in range(2)]
    s = stats[-1]
    return {
        "workload": f"body-in-garment: capsule-union body {len(pair.tri_b)} triangles (oriented), cloth shell "
                    f"{len(pair.tri_a)} triangles, 5% of cloth vertices pushed in by U[0, 0.03]; float32, "
                    "float32-filtered, d=1e-3",
        "converged": s["converged"], "rounds": s["rounds"], "residual_hits": s["residual_hits"],
        "hits0": s["hits0"], "max_zone": s["max_zone"],
        "resolved_pairs_per_s": args.body_steps / wall if s["converged"] else 0.0,
        "ms_per_resolve": 1e3 * wall / args.body_steps, "p50_ms": sorted(lat)[len(lat) // 2],
        "ef_tests_per_s": sum(x["candidates"] for x in stats) / wall,
        "stage_ms_per_resolve": {k: sum(x["stage_ms"][k] for x in tstats) / len(tstats) for k in s["stage_ms"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rounds", type=int, default=12)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU-oracle sample length (whole steps are repeated)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-pairs", type=int, default=256,
                    help="pairs of the mixed pair set in the batched measurement (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--body-steps", type=int, default=5,
                    help="timed resolves of the body-in-garment pair (0: skip it)")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests of the open-loop serving measurement (0: skip it)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-pool-mib", type=int, default=1024)
    ap.add_argument("--serve-rounds", type=int, default=4)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run 3 linked-tori steps and a 256 MiB device copy (for HBM counter passes), then exit")
    ap.add_argument("--batch-rounds", type=int, default=4,
                    help="response-round budget per pair in the batched and plain measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    import paper_1409_2081_amd as hf

    pair = meshgen.linked_tori()
    ctx = hf.Context(0)
    tens = hf.pair_tensors(pair, "cuda:0")
    kw = dict(tier=pair.tier, max_rounds=args.rounds, want_lists=False)
    if args.pmc_probe:
        # the counters of the copy calibrate FETCH_SIZE / WRITE_SIZE against known bytes
        for _ in range(3):
            ctx.resolve(*tens, pair.orientation, pair.d, **kw)
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "copy_bytes": COPY_BYTES}))
        return

    progress("linked tori: warm-up")
    for _ in range(args.warmup):
        ctx.resolve(*tens, pair.orientation, pair.d, **kw)
    torch.cuda.synchronize()

    lat = []
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        g = ctx.resolve(*tens, pair.orientation, pair.d, **kw)
        lat.append(time.perf_counter() - ts)
        stats.append(g["stats"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-stage GPU time (HIP events on the call's stream) from the same
    # number of further steps, kept out of the timed region: the events are
    # extra queue operations
    tstats = [ctx.resolve(*tens, pair.orientation, pair.d, timing=True, **kw)["stats"] for _ in range(args.steps)]
    torch.cuda.synchronize()

    s0 = stats[-1]
    cand = sum(s["candidates"] for s in stats)
    ms_per_step = 1e3 * wall / args.steps
    tests_per_s = cand / wall
    lat_ms = sorted(1e3 * x for x in lat)

    def pct(p):
        return lat_ms[min(len(lat_ms) - 1, int(round(p / 100.0 * (len(lat_ms) - 1))))]

    stage_ms = {k: sum(s["stage_ms"][k] for s in tstats) / args.steps for k in s0["stage_ms"]}
    stage_calls = {k: sum(s["stage_calls"][k] for s in tstats) / args.steps for k in s0["stage_calls"]}
    dominant = max(("traverse", "solve", "refit"), key=lambda k: stage_ms[k])

    # edge counts for the algorithmic byte model
    ne_a = len(np.unique(np.sort(np.concatenate([pair.tri_a[:, [0, 1]], pair.tri_a[:, [1, 2]],
                                                 pair.tri_a[:, [2, 0]]]), axis=1), axis=0))
    ne_b = ne_a
    # directions per step: round r tests direction (r % 2) first; round 0 tests both
    launches = stage_calls["traverse"]
    per_dir = {0: launches / 2.0, 1: launches / 2.0}
    trav_avg_ms = stage_ms["traverse"] / max(stage_calls["traverse"], 1)
    trav_bytes_per_launch = traverse_bytes(pair, ne_a, ne_b, per_dir, cand / args.steps) / max(launches, 1)
    achieved = trav_bytes_per_launch / (trav_avg_ms * 1e-3) / 1e9
    roofline = {
        "kernel": "k_traverse<true,true,64> (BVH traversal; candidates queued for the narrow phase)",
        "bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
        "avg_launch_ms": trav_avg_ms, "algorithmic_bytes_per_launch": trav_bytes_per_launch,
        "launches_per_step": launches,
    }

    out = {
        "metric": METRIC, "value": tests_per_s, "unit": "E-F tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "linked_tori 128x64 (8192 v / 16384 t each), shift 1.7, rot_x 90, "
                               "float32 storage, float32-filtered predicates, both oriented, d=1e-3",
                   "max_rounds": args.rounds, "parallelism": "1 GPU"},
        "resolve_calls_per_s": args.steps / wall,
        "resolved_pairs_per_s": (args.steps / wall) if s0["converged"] else 0.0,
        "p50_ms": pct(50), "p99_ms": pct(99),
        "converged": s0["converged"], "rounds": s0["rounds"], "residual_hits": s0["residual_hits"],
        "hits0": s0["hits0"], "candidates_per_step": cand / args.steps,
        "node_visits_per_step": sum(s.get("node_visits", 0) for s in stats) / args.steps,
        "exact_tests_per_step": s0["exact_tests"], "f32_unsure_per_step": s0["f32_ambiguous"],
        "max_zone": s0["max_zone"], "stage_ms_per_step": stage_ms, "stage_launches_per_step": stage_calls,
        "dominant_stage": dominant,
        "roofline": roofline,
    }

    progress(f"linked tori: {args.steps} steps in {wall:.2f} s")
    if args.body_steps > 0:
        out["body_garment"] = bench_body(ctx, args)
    if args.batch_pairs > 0:
        out["batch"] = bench_batch(ctx, args)
    if args.serve_requests > 0:
        out["serving"] = bench_serving(args)

    if not args.no_cpu:
        import oracle
        nthreads = min(os.cpu_count() or 1, 16)
        oracle.lib()
        progress("cpu oracle sample")
        t = time.perf_counter()
        n_steps, cand_cpu = 0, 0
        while True:
            o = oracle.resolve_pair(pair, nthreads=nthreads, max_rounds=args.rounds)
            n_steps += 1
            cand_cpu += o["candidates"]
            dt = time.perf_counter() - t
            if dt >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {
            "value": cand_cpu / dt, "unit": "E-F tests/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n_steps} oracle resolves of the same pair and round budget "
                      f"({o['rounds']} responses each, {cand_cpu} candidate tests, {dt:.1f} s; "
                      "brute-force E-F DCD with box rejection and OpenMP over edges, numpy zone solves)",
            "seconds": dt, "ms_per_step": 1e3 * dt / n_steps,
        }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
