"""Benchmark: bitruss decomposition throughput on one MI355X.

One step = one full bt_decompose (validation, priority order, rank-space
CSR, wedge counting, BE-Index construction, peel) of the 5M-edge Chung-Lu
graph, with the input CSR already resident in HBM.  Prints one JSON line:
the timed steps (value, ms_per_step, p50/p99 step times), the peel kernel
against the HBM roofline and its measured HBM traffic, its atomic
throughput, and, outside the timed steps: launch parameters picked by the
autotuner (--tune), the same peel without batch bloom processing
(--ablation), batched against plain graphs/s on 256 pool graphs (--batch)
and on the whole 4,096-graph pool (--batch-all), served against plain FIFO
latency on a burst of requests (--serve), and the CPU oracle on a sample
(cpu_baseline).

  python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s
# Random device-scope int32 atomics per second on one MI355X, measured with a
# microbenchmark (many waves, one atomic per lane over a 20-160 MB array).
ATOMIC_PEAK_PER_S = 2.7e10


def phi_digest(phi) -> str:
    return hashlib.sha256(phi.astype("<i8").tobytes()).hexdigest()


def cpu_baseline(g, frac: float, seed: int = 2027):
    """The oracle, untuned, on a vertex-sampled induced subgraph (host cores)."""
    import oracle
    from paper_2001_06111_amd import synth
    sub = synth.vertex_sample(g, frac, seed)
    t0 = time.perf_counter()
    sup, _, _ = oracle.support(sub.n_upper, sub.n_lower, sub.row_ptr, sub.col)
    oracle.bitruss(sub.n_upper, sub.n_lower, sub.row_ptr, sub.col, sup=sup)
    dt = time.perf_counter() - t0
    return {"value": sub.m / dt, "unit": "edges/s", "cores": oracle.max_threads(),
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"{frac:g} vertex-sampled induced subgraph of the workload "
                      f"(seed {seed}): {sub.n_upper}x{sub.n_lower}, m={sub.m}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-frac", type=float, default=0.5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="chunglu5m", choices=["chunglu5m", "uniform10k", "hub20m"])
    ap.add_argument("--batch", type=int, default=256,
                    help="graphs of the many-small-graphs pool for the batched-vs-plain line (0: skip)")
    ap.add_argument("--batch-all", type=int, default=4096,
                    help="graphs of the pool decomposed as one batch (0: skip)")
    ap.add_argument("--serve", type=float, default=1.0,
                    help="seconds of Poisson arrivals for the served-vs-plain-FIFO line (0: skip)")
    ap.add_argument("--serve-pool", type=int, default=512,
                    help="small graphs in the request pool (of the 4096)")
    ap.add_argument("--serve-big", type=int, default=4, help="2M-edge graphs in the request pool")
    ap.add_argument("--tune", type=int, default=1,
                    help="autotune launch parameters (untimed) before measuring; 0 = defaults")
    ap.add_argument("--ablation", type=int, default=1,
                    help="also peel once without batch bloom processing (BiT-BU+); 0 = skip")
    ap.add_argument("--calib", action="store_true",
                    help="also run a 256 MiB device copy (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library decomposes on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2001_06111_amd import binding, synth

    gen = {"chunglu5m": synth.plain_chunglu_5m, "uniform10k": synth.plain_uniform_10k,
           "hub20m": synth.plain_hub_20m}[args.workload]
    g = gen()
    print(f"[bench] workload {g.name}: {g.n_upper}x{g.n_lower}, m={g.m}", file=sys.stderr,
          flush=True)
    dg = binding.DeviceGraph.upload(g, "cuda:0")
    phi = torch.empty(g.m, dtype=torch.int64, device="cuda:0")
    sup = torch.empty(g.m, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream()

    if args.calib:
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    tuning = {}
    if args.tune:
        t0 = time.perf_counter()
        tuning["single"] = binding.bt_tune(dg)
        tuning["single_seconds"] = round(time.perf_counter() - t0, 2)
        print(f"[bench] tuned {tuning['single']}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        binding.bt_decompose(dg, stats=True, out_phi=phi, out_sup=sup)
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    step_ms = []
    stats = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        _, _, st = binding.bt_decompose(dg, stats=True, out_phi=phi, out_sup=sup)
        ev[i + 1].record(stream)
        stats.append(st)
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for i in range(args.steps):
        step_ms.append(ev[i].elapsed_time(ev[i + 1]))
    ms = wall * 1000.0 / args.steps

    phi_h = phi.cpu().numpy()
    digest = phi_digest(phi_h)
    golden = {}
    gp = os.path.join(ROOT, "tests", "golden", "digests.json")
    if os.path.exists(gp):
        golden = json.load(open(gp))
    want = golden.get(g.name, {}).get("phi_sha256")
    check = "no-oracle-digest" if want is None else ("match" if want == digest else "MISMATCH")

    st = stats[-1]
    # Dominant kernel: the peel (over 95% of a step).  Its device time is
    # taken by the library with HIP events around each launch on this stream.
    peel_s = st["ms_peel_kernel"] / 1e3
    alg_bytes = peel_bytes(st, g.m)
    achieved = alg_bytes / peel_s / 1e9 if peel_s > 0 else 0.0
    launches = max(1, st["peel_launches"])
    traffic = measured_traffic(launches)
    out = {
        "metric": "edges decomposed/s (bit-exact phi_e), batched vs plain; p50/p99 latency",
        "value": g.m / (ms / 1000.0),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": g.name, "n_upper": g.n_upper, "n_lower": g.n_lower, "m": g.m,
                   "generator": "Chung-Lu edge sampling, exponents 2.1/2.5, cap 50k, seed 1"
                   if args.workload == "chunglu5m" else args.workload},
        "phi_check": check,
        "wedges_per_s": st["wedges_po"] / (ms / 1000.0),
        "phases_ms": {k: round(st[k], 3) for k in ("ms_prepare", "ms_count", "ms_link", "ms_peel")},
        "counters": {k: st[k] for k in ("butterflies", "wedges_po", "blooms", "bloom_wedges",
                                        "levels", "rounds", "max_phi", "support_updates",
                                        "bloom_visits", "index_bytes",
                                        "support_updates_unbatched")},
        "roofline": {"kernel": "k_peel_persistent (bloom peel, all rounds)", "bound": "hbm",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes / launches,
                     "avg_launch_ms": st["ms_peel_kernel"] / launches, "launches": launches},
        # The peel's other ceiling: its support decrements are device-scope atomics.
        "atomic_throughput": {"decrements_per_s": st["support_updates"] / peel_s if peel_s else 0.0,
                              "measured_peak_per_s": ATOMIC_PEAK_PER_S,
                              "frac": (st["support_updates"] / peel_s / ATOMIC_PEAK_PER_S)
                              if peel_s else 0.0},
    }
    if args.ablation:
        out["ablation"] = ablation(dg, phi_h, st)
    if args.batch > 0:
        out["batched"] = batch_compare(args.batch, tuning if args.tune else None)
    if args.batch_all > 0:
        out["batched_all"] = batch_all(args.batch_all,
                                       out.get("batched", {}).get("plain_graphs_per_s"))
    if args.serve > 0:
        out["served"] = serve_compare(args.serve, args.serve_pool, args.serve_big)
    if tuning:
        out["tuning"] = tuning
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_frac)
    print(json.dumps(out), flush=True)


def ablation(dg, phi_ref, st_bloom):
    """One decompose of the same graph by BiT-BU+ (batch edge processing
    only): its peel time and support updates against BiT-BU++'s."""
    from paper_2001_06111_amd import binding
    print("[bench] ablation: peel without batch bloom processing", file=sys.stderr, flush=True)
    _, phi_e, st_e = binding.bt_decompose_variant(dg, binding.BT_PEEL_BATCH_EDGE, want_sup=False,
                                                  stats=True)
    same = bool((phi_e.cpu().numpy() == phi_ref).all())
    return {"variant": "BiT-BU+ (batch edge processing only)",
            "same_phi": same,
            "peel_ms": round(st_e["ms_peel_kernel"], 3),
            "peel_ms_batched": round(st_bloom["ms_peel_kernel"], 3),
            "support_updates": st_e["support_updates"],
            "support_updates_batched": st_bloom["support_updates"],
            "time_ratio": st_e["ms_peel_kernel"] / st_bloom["ms_peel_kernel"]
            if st_bloom["ms_peel_kernel"] else None}


def batch_compare(n, tuning=None):
    """Graphs/s of the batched form against the plain per-graph loop (same
    graphs).  With `tuning`, batch launch parameters are tuned on these
    graphs first (untimed) and recorded there."""
    import torch
    from paper_2001_06111_amd import binding, synth
    gs = [synth.batch_graph(i) for i in range(n)]
    dgs = [binding.DeviceGraph.upload(g, "cuda:0") for g in gs]
    m = sum(g.m for g in gs)
    binding.bt_decompose_batch(dgs[:8])
    binding.bt_decompose(dgs[0])
    if tuning is not None:
        t0 = time.perf_counter()
        tuning["batch"] = binding.bt_tune(dgs)
        tuning["batch_seconds"] = round(time.perf_counter() - t0, 2)
        print(f"[bench] tuned batch {tuning['batch']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [binding.bt_decompose(d)[1] for d in dgs]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, phis, st = binding.bt_decompose_batch(dgs, stats=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(plain, phis))
    print(f"[bench] batch of {n}: plain {t_plain:.3f}s batched {t_batch:.3f}s same={same}",
          file=sys.stderr, flush=True)
    return {"workload": f"first {n} graphs of the 4096-graph pool", "graphs": n, "edges": m,
            "plain_graphs_per_s": n / t_plain, "batched_graphs_per_s": n / t_batch,
            "plain_edges_per_s": m / t_plain, "batched_edges_per_s": m / t_batch,
            "speedup": t_plain / t_batch, "batched_equals_plain": same,
            "batched_rounds": st["rounds"]}


def _pool_graph(i):
    from paper_2001_06111_amd import synth
    return synth.batch_graph(i)


def batch_all(n, plain_graphs_per_s):
    """The whole pool batched (graphs generated on host cores in parallel).

    The plain per-graph rate is the one measured on the pool's first graphs
    (same distribution); the whole pool would take minutes in the plain loop.
    """
    import concurrent.futures as cf
    import torch
    from paper_2001_06111_amd import binding
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        gs = list(ex.map(_pool_graph, range(n), chunksize=16))
    dgs = [binding.DeviceGraph.upload(g, "cuda:0") for g in gs]
    m = sum(g.m for g in gs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st = binding.bt_decompose_batch(dgs, want_sup=False, stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] whole pool of {n}: batched {dt:.3f}s", file=sys.stderr, flush=True)
    out = {"workload": f"all {n} graphs of the pool", "graphs": n, "edges": m,
           "batched_graphs_per_s": n / dt, "batched_edges_per_s": m / dt, "seconds": dt,
           "peel_launches": st["peel_launches"], "rounds_max": st["rounds"]}
    if plain_graphs_per_s:
        out["speedup_vs_plain_rate"] = (n / dt) / plain_graphs_per_s
    return out


def serve_compare(seconds, n_small, n_big, rate=200.0):
    """p50/p99 latency and graphs/s: the serving engine vs a plain FIFO loop.

    Poisson arrivals at `rate`/s for `seconds`; 95% of requests are graphs of
    the small-graph pool, 5% are 2M-edge graphs (indices drawn from pools of
    n_small and n_big graphs).  Latency = completion - arrival.
    """
    import threading
    import numpy as np
    import torch
    from paper_2001_06111_amd import binding, synth
    reqs = synth.serving_arrivals(rate=rate, duration=seconds, n_small=n_small, n_big=n_big)
    small = {i: binding.DeviceGraph.upload(synth.batch_graph(i), "cuda:0")
             for i in sorted({k for _, kind, k in reqs if kind == "small"})}
    big = {j: binding.DeviceGraph.upload(synth.big_serving_graph(j), "cuda:0")
           for j in sorted({k for _, kind, k in reqs if kind == "big"})}
    graph = [small[k] if kind == "small" else big[k] for _, kind, k in reqs]
    arrive = np.array([t for t, _, _ in reqs])
    # warm both paths
    binding.bt_decompose(graph[0])
    torch.cuda.synchronize()

    # plain FIFO: one request at a time, in arrival order
    done_plain = np.zeros(len(reqs))
    t0 = time.perf_counter()
    for i, g in enumerate(graph):
        now = time.perf_counter() - t0
        if now < arrive[i]:
            time.sleep(arrive[i] - now)
        binding.bt_decompose(g, want_sup=False)
        torch.cuda.synchronize()
        done_plain[i] = time.perf_counter() - t0
    span_plain = done_plain.max()
    lat_plain = done_plain - arrive

    # served: submit at arrival times, poll completions
    eng = binding.BtEngine()
    done_srv = np.zeros(len(reqs))
    t0 = time.perf_counter()
    finished = threading.Event()

    def poller():
        got = 0
        while got < len(reqs):
            for rid, st in eng.bt_engine_poll():
                done_srv[rid] = time.perf_counter() - t0
                got += 1
            time.sleep(0.0005)
        finished.set()

    th = threading.Thread(target=poller, daemon=True)
    th.start()
    for i, g in enumerate(graph):
        now = time.perf_counter() - t0
        if now < arrive[i]:
            time.sleep(arrive[i] - now)
        eng.bt_engine_submit(g, i)
    finished.wait()
    est = eng.bt_engine_stats()
    eng.bt_engine_destroy()
    span_srv = done_srv.max()
    lat_srv = done_srv - arrive
    same = True
    for i in range(0, len(reqs), max(1, len(reqs) // 32)):
        _, phi, _ = binding.bt_decompose(graph[i], want_sup=False)
        same &= bool(torch.equal(phi, eng.results[i][2]))
    print(f"[bench] serve {len(reqs)} reqs: plain p99 {np.percentile(lat_plain, 99):.3f}s "
          f"served p99 {np.percentile(lat_srv, 99):.3f}s", file=sys.stderr, flush=True)
    return {"workload": f"Poisson {rate:g}/s for {seconds:g}s: 95% small-pool graphs (of {n_small}), "
                        f"5% 2M-edge graphs (of {n_big})",
            "requests": len(reqs), "big_requests": sum(1 for _, k, _ in reqs if k == "big"),
            "served_p50_s": float(np.percentile(lat_srv, 50)),
            "served_p99_s": float(np.percentile(lat_srv, 99)),
            "plain_p50_s": float(np.percentile(lat_plain, 50)),
            "plain_p99_s": float(np.percentile(lat_plain, 99)),
            "served_graphs_per_s": len(reqs) / span_srv, "plain_graphs_per_s": len(reqs) / span_plain,
            "served_batches": est["batches"], "served_equals_plain": same}


def peel_bytes(st, m):
    """Algorithmic HBM bytes of the peel (what the method must move).

    Per support decrement: a 4-byte read-modify-write (8 B).  Per link (each
    of the 2 n_W edge-wedge links is walked once, when its edge is removed):
    the 12-byte link (wedge, bloom, twin edge), the wedge's alive word (RMW,
    8 B) and the bloom's k and wedge range (12 B).  Per touched-bloom visit:
    its C and k (8 B) and the 16-byte work item (written, read).  Per edge:
    one frontier item (16 B written and read) and its phi (4 B).
    """
    return (8 * st["support_updates"] + 32 * 2 * st["bloom_wedges"]
            + 40 * st["bloom_visits"] + 36 * m)


def measured_traffic(launches):
    """HBM bytes per peel launch from the committed rocprofv3 counter summary.

    profiles/peel_chunglu5m_traffic.md records FETCH_SIZE and WRITE_SIZE of
    the peel kernel, scaled by what the counters read for a copy of known
    size, together with the SHA-256 of the peel source they were taken on
    (peel.hip followed by peel_common.h).  Returns None when the source has
    changed since (or no summary exists).
    """
    path = os.path.join(ROOT, "profiles", "peel_chunglu5m_traffic.md")
    csrc = os.path.join(ROOT, "paper_2001_06111_amd", "csrc")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ("peel.hip", "peel_common.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    want = h.hexdigest()
    if fields.get("peel_source_sha256") != want or "hbm_bytes_total" not in fields:
        return None
    return float(fields["hbm_bytes_total"]) / launches


if __name__ == "__main__":
    main()
