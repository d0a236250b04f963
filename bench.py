"""Benchmark: bitruss decomposition on one MI355X (one JSON line).

Headline: the batched form on the pool of 4,096 Chung-Lu graphs (|U|, |L|
log-uniform in [50, 20k], m log-uniform in [200, 200k], exponent 2.2).  One
step = one bt_decompose_batch over all 4,096 graphs (validation, priority
order, rank-space CSR, wedge counting, BE-Index, peel, per-graph outputs),
with every graph already resident in HBM; `value` = pool edges / step time.
In the same run, untimed by the step contract but measured: the plain
per-graph loop over the same 4,096 graphs (bt_decompose one at a time), so
batched and plain graphs/s come from identical inputs, and every plain
result is compared with the batched one.

Also reported, each only if the wall-time budget (--budget) still allows
it: the dominant kernel (k_peel_multi) against the HBM roofline with the
algorithmic bytes of the method; single graphs (10k-edge uniform, 5M-edge
Chung-Lu, 20M-edge hub graph by the plain peel and by BiT-PC) with their
own rooflines; served against plain FIFO latency on a window of Poisson
arrivals; and the CPU oracle on a bounded sample of the pool.

Every input is generated on host cores before the first GPU call.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget SECONDS]
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

T_START = time.perf_counter()
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s
POOL = 4096


def log(msg):
    print(f"[bench {time.perf_counter() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def left(budget):
    return budget - (time.perf_counter() - T_START)


def sha_i64(arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(a.astype("<i8").tobytes())
    return h.hexdigest()


# --- algorithmic bytes of the peel -----------------------------------------

def peel_bytes(st):
    """Algorithmic HBM bytes of a peel (what the method must move).

    Each of the 2 n_W edge-to-wedge links is walked once, when its edge is
    removed: the link, the wedge record, the exchange of the wedge's alive
    flag, the read-modify-write of the twin's support and of the bloom's
    removed-wedge count C (40 B with int64 supports).  Each live wedge of a
    touched bloom visited in a round (L_touch, counted on the device): its
    record, its alive flag and the read-modify-writes of its two supports
    (41 B).  The second figure restates both at the 32-bit supports and
    counts this library uses: 29 B per link, 25 B per visit.
    """
    links = 2 * st["bloom_wedges"]
    visits = st["wedge_visits"]
    return 40 * links + 41 * visits, 29 * links + 25 * visits


def roofline(kernel, st, traffic_total):
    launches = max(1, st["peel_launches"])
    secs = st["ms_peel_kernel"] / 1e3
    alg, alg32 = peel_bytes(st)
    ach = alg / secs / 1e9 if secs > 0 else 0.0
    out = {"kernel": kernel, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
           "traffic": traffic_total / launches if traffic_total else None,
           "algorithmic_bytes_per_launch": alg / launches,
           "algorithmic_bytes_int32_per_launch": alg32 / launches,
           "frac_int32": (alg32 / secs / 1e9) / PEAK_HBM_GBS if secs > 0 else 0.0,
           "avg_launch_ms": st["ms_peel_kernel"] / launches, "launches": launches,
           "bytes_formula": "40 B x 2 n_W links + 41 B x L_touch (int32: 29 B, 25 B)",
           "n_w": st["bloom_wedges"], "l_touch": st["wedge_visits"]}
    if traffic_total and secs > 0:
        out["traffic_gbs"] = traffic_total / secs / 1e9
        out["traffic_frac"] = out["traffic_gbs"] / PEAK_HBM_GBS
    out["decrements_per_s"] = st["support_updates"] / secs if secs > 0 else 0.0
    return out


def measured_traffic(profile, sources):
    """HBM bytes of a kernel from a committed rocprofv3 counter summary.

    The summary records FETCH_SIZE plus WRITE_SIZE of the kernel over one
    run, each scaled by what the counter reads for a device copy of known
    size, with the SHA-256 of the kernel's sources at the time.  Returns
    None when those sources have changed since (or no summary exists).
    """
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2001_06111_amd", "csrc", f), "rb").read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "hbm_bytes_total" not in fields:
        return None
    return float(fields["hbm_bytes_total"])


# --- inputs (host cores, before any GPU call) -------------------------------

def _gen(task):
    from paper_2001_06111_amd import synth
    kind, i = task
    if kind == "pool":
        return [synth.batch_graph(j) for j in range(i, min(i + 32, POOL))]
    if kind == "big":
        return [synth.big_serving_graph(i)]
    return [{"c0": synth.plain_uniform_10k, "c1": synth.plain_chunglu_5m,
             "c2": synth.plain_hub_20m}[kind]()]


def generate(args, arrivals):
    import concurrent.futures as cf
    tasks = []
    if args.single:
        tasks += [(k, 0) for k in ("c2", "c1", "c0") if k in args.single]
    bigs = sorted({k for _, kind, k in arrivals if kind == "big"})
    tasks += [("big", j) for j in bigs]
    tasks += [("pool", i) for i in range(0, POOL, 32)]
    out = {"pool": [], "big": {}}
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for t, gs in zip(tasks, ex.map(_gen, tasks)):
            if t[0] == "pool":
                out["pool"].extend(gs)
            elif t[0] == "big":
                out["big"][t[1]] = gs[0]
            else:
                out[t[0]] = gs[0]
    return out


# --- measurements ------------------------------------------------------------

def headline(dgs, steps, warmup):
    import torch
    from paper_2001_06111_amd import binding
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        binding.bt_decompose_batch(dgs, want_sup=False)
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    stats, phis = [], None
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        _, phis, st = binding.bt_decompose_batch(dgs, want_sup=False, stats=True)
        ev[i + 1].record(stream)
        stats.append(st)
        log(f"step {i} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return wall, step_ms, stats[-1], phis


def plain_loop(dgs, ref_phis, budget_s):
    """bt_decompose on each graph in turn; every result compared with the
    batched one.  Stops early only if the budget runs out (then says so)."""
    import torch
    from paper_2001_06111_amd import binding
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same, done = True, 0
    for i, d in enumerate(dgs):
        _, phi, _ = binding.bt_decompose(d, want_sup=False)
        same &= bool(torch.equal(phi, ref_phis[i]))
        done += 1
        if i % 512 == 511:
            torch.cuda.synchronize()
            log(f"plain loop {i + 1}/{len(dgs)}")
            if time.perf_counter() - t0 > budget_s and i + 1 < len(dgs):
                break
    torch.cuda.synchronize()
    return time.perf_counter() - t0, done, same


def single(name, g, reps, warmup, golden, variant=None, tau=None, traffic=None):
    import torch
    from paper_2001_06111_amd import binding
    dg = binding.DeviceGraph.upload(g, "cuda:0")
    phi = torch.empty(g.m, dtype=torch.int64, device="cuda:0")

    def run():
        if tau is not None:
            return binding.bt_decompose_pc(dg, tau=tau, want_sup=False, stats=True, out_phi=phi)[2]
        if variant is not None:
            r = binding.bt_decompose_variant(dg, variant, want_sup=False, stats=True)
            phi.copy_(r[1])
            return r[2]
        return binding.bt_decompose(dg, want_sup=False, stats=True, out_phi=phi)[2]

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ts, st = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        st = run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    t = ts[len(ts) // 2]
    d = sha_i64([phi.cpu().numpy()])
    want = golden.get(g.name, {}).get("phi_sha256")
    out = {"workload": g.name, "m": g.m, "seconds": t, "edges_per_s": g.m / t,
           "wedges_per_s": st["wedges_po"] / t, "reps": reps, "warmup": warmup,
           "p50_s": t, "p99_s": ts[min(len(ts) - 1, int(0.99 * len(ts)))],
           "phi_check": "no-oracle-digest" if want is None else
           ("match" if want == d else "MISMATCH"),
           "phases_ms": {k: round(st[k], 3) for k in ("ms_prepare", "ms_count", "ms_link",
                                                      "ms_peel")},
           "counters": {k: st[k] for k in ("butterflies", "wedges_po", "blooms", "bloom_wedges",
                                           "levels", "rounds", "max_phi", "support_updates",
                                           "wedge_visits", "passes")}}
    out["roofline"] = roofline("k_peel_persistent", st,
                               traffic * max(1, st["peel_launches"]) if traffic else None)
    del dg, phi
    torch.cuda.empty_cache()
    return out


def serve_compare(seconds, graphs, big, arrivals, slots):
    """p50/p99 latency and graphs/s: the serving engine vs a plain FIFO loop.

    Requests arrive as a Poisson stream (200/s; 95% pool graphs, 5% 2M-edge
    graphs); latency = completion - arrival.  Every served result is compared
    with the plain result of the same request, and every status is checked.
    """
    import threading
    import numpy as np
    import torch
    from paper_2001_06111_amd import binding
    graph = [graphs[k] if kind == "small" else big[k] for _, kind, k in arrivals]
    arrive = np.array([t for t, _, _ in arrivals])
    binding.bt_decompose(graph[0])
    torch.cuda.synchronize()
    done_plain = np.zeros(len(graph))
    plain_phi = []
    t0 = time.perf_counter()
    for i, g in enumerate(graph):
        now = time.perf_counter() - t0
        if now < arrive[i]:
            time.sleep(arrive[i] - now)
        _, phi, _ = binding.bt_decompose(g, want_sup=False)
        torch.cuda.synchronize()
        done_plain[i] = time.perf_counter() - t0
        plain_phi.append(phi)
    log(f"serve: plain FIFO done ({len(graph)} requests)")
    eng = binding.BtEngine(slots=slots)
    done_srv = np.zeros(len(graph))
    status = {}
    t0 = time.perf_counter()
    finished = threading.Event()

    def poller():
        got = 0
        while got < len(graph):
            for rid, st in eng.bt_engine_poll():
                done_srv[rid] = time.perf_counter() - t0
                status[rid] = st
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
    ok = all(status.get(i) == binding.BT_OK for i in range(len(graph)))
    same = ok and all(torch.equal(plain_phi[i], eng.results[i][2]) for i in range(len(graph)))
    lat_p, lat_s = done_plain - arrive, done_srv - arrive
    log(f"serve: plain p99 {np.percentile(lat_p, 99):.3f}s served p99 "
        f"{np.percentile(lat_s, 99):.3f}s")
    # The engine's size classes: below 2^14 edges, below 2^19, larger.
    m = np.array([g.m for g in graph])
    by_class = {}
    for name, sel in (("small", m < (1 << 14)), ("medium", (m >= (1 << 14)) & (m < (1 << 19))),
                      ("large", m >= (1 << 19))):
        if sel.any():
            by_class[name] = {"requests": int(sel.sum()),
                              "served_p50_s": float(np.percentile(lat_s[sel], 50)),
                              "served_p99_s": float(np.percentile(lat_s[sel], 99)),
                              "plain_p50_s": float(np.percentile(lat_p[sel], 50)),
                              "plain_p99_s": float(np.percentile(lat_p[sel], 99))}
    return {"workload": f"Poisson 200/s for {seconds:g} s: 95% graphs of the 4,096-graph pool, "
                        f"5% 2M-edge graphs of a pool of 32 (50k x 200k, exponent 2.0)",
            "requests": len(graph), "big_requests": sum(1 for _, k, _ in arrivals if k == "big"),
            "slots": slots,
            "served_p50_s": float(np.percentile(lat_s, 50)),
            "served_p99_s": float(np.percentile(lat_s, 99)),
            "plain_p50_s": float(np.percentile(lat_p, 50)),
            "plain_p99_s": float(np.percentile(lat_p, 99)),
            "served_graphs_per_s": len(graph) / done_srv.max(),
            "plain_graphs_per_s": len(graph) / done_plain.max(),
            "served_batches": est["batches"], "peel_yields": est["peel_yields"],
            "by_class": by_class, "all_status_ok": ok,
            "every_result_equals_plain": bool(same)}


def cpu_baseline(pool, budget_s, golden):
    """The oracle, as it stands, on the first pool graphs in pool order until
    about budget_s seconds of CPU work (host cores)."""
    import oracle
    t_all, m_all, n = 0.0, 0, 0
    for g in pool:
        t0 = time.perf_counter()
        sup, _, _ = oracle.support(g.n_upper, g.n_lower, g.row_ptr, g.col)
        oracle.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col, sup=sup)
        t_all += time.perf_counter() - t0
        m_all += g.m
        n += 1
        if t_all >= budget_s:
            break
    out = {"value": m_all / t_all, "unit": "edges/s", "cores": oracle.max_threads(),
           "kind": "oracle", "seconds": round(t_all, 3),
           "sample": f"the first {n} graphs of the 4,096-graph pool in pool order "
                     f"({m_all} edges), one after another, each on all host threads"}
    full = golden.get(f"pool:{POOL}", {})
    if full.get("oracle_seconds"):
        out["whole_pool_recorded"] = {
            "seconds": full["oracle_seconds"], "threads": full.get("oracle_threads"),
            "edges_per_s": full["m"] / full["oracle_seconds"],
            "note": "the oracle over all 4,096 graphs when their digests were written "
                    "(another host, not this run)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget", type=float, default=500.0,
                    help="wall seconds for the whole run; extras that would not fit are skipped")
    ap.add_argument("--single", default="c0,c1,c2",
                    help="single-graph lines: any of c0,c1,c2 (empty: none)")
    ap.add_argument("--c2-plain", type=int, default=1,
                    help="also time the 20M-edge hub graph by the plain peel (besides BiT-PC)")
    ap.add_argument("--serve", type=float, default=1.0,
                    help="seconds of Poisson arrivals for served vs plain FIFO (0: skip)")
    ap.add_argument("--slots", type=int, default=2, help="serving engine slots")
    ap.add_argument("--plain", type=int, default=1, help="plain per-graph loop (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib", action="store_true",
                    help="also copy 256 MiB device-to-device first (calibrates rocprofv3 byte "
                         "counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build decomposes on one GPU; run with --gpus 1"}))
        sys.exit(2)
    args.single = [s for s in args.single.split(",") if s]

    from paper_2001_06111_amd import synth
    arrivals = synth.serving_arrivals(duration=args.serve) if args.serve > 0 else []
    inputs = generate(args, arrivals)
    pool = inputs["pool"]
    m_pool = sum(g.m for g in pool)
    log(f"inputs generated: pool of {len(pool)} graphs, {m_pool} edges")

    import numpy as np
    import torch
    from paper_2001_06111_amd import binding
    golden = {}
    gp = os.path.join(ROOT, "tests", "golden", "digests.json")
    if os.path.exists(gp):
        golden = json.load(open(gp))

    if args.calib:
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    dgs = [binding.DeviceGraph.upload(g, "cuda:0") for g in pool]
    torch.cuda.synchronize()
    log("pool uploaded")

    wall, step_ms, st, phis = headline(dgs, args.steps, args.warmup)
    ms = wall * 1000.0 / args.steps
    digest = sha_i64([p.cpu().numpy() for p in phis])
    want = golden.get(f"pool:{POOL}", {}).get("phi_sha256")
    check = "no-oracle-digest" if want is None else ("match" if want == digest else "MISMATCH")
    # api.hip sets the union's edge order, which the traffic depends on.
    traffic = measured_traffic("peel_multi_pool4096_traffic.md",
                               ("peel_multi.hip", "peel_common.h", "api.hip"))
    out = {
        "metric": "edges decomposed/s (bit-exact phi_e), batched vs plain; p50/p99 latency",
        "value": m_pool / (ms / 1000.0),
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
        "config": {"workload": "chunglu-pool4096-batched", "graphs": POOL, "m": m_pool,
                   "generator": "Chung-Lu edge sampling; |U|, |L| log-uniform in [50, 20000], "
                                "m log-uniform in [200, 200000] clamped to |U||L|/4, "
                                "exponent 2.2; graph i seeded 3,000,000 + i",
                   "form": "one bt_decompose_batch call over all graphs per step"},
        "phi_check": check,
        "graphs_per_s": POOL / (ms / 1000.0),
        "wedges_per_s": st["wedges_po"] / (ms / 1000.0),
        "phases_ms": {k: round(st[k], 3) for k in ("ms_prepare", "ms_count", "ms_link",
                                                   "ms_peel")},
        "counters": {k: st[k] for k in ("butterflies", "wedges_po", "blooms", "bloom_wedges",
                                        "levels", "rounds", "support_updates", "bloom_visits",
                                        "wedge_visits", "peel_launches", "index_bytes")},
        "roofline": roofline("k_peel_multi", st, traffic),
    }
    skipped = {}

    if args.plain:
        est = ms / 1000.0 * 17.5 + 10
        if left(args.budget) > est:
            t_plain, n_done, same = plain_loop(dgs, phis, left(args.budget) - 60)
            m_done = sum(g.m for g in pool[:n_done])
            out["plain"] = {"workload": f"the same {n_done} pool graphs, one bt_decompose each",
                            "graphs": n_done, "seconds": t_plain,
                            "plain_graphs_per_s": n_done / t_plain,
                            "plain_edges_per_s": m_done / t_plain,
                            "batched_graphs_per_s": POOL / (ms / 1000.0),
                            "speedup": (POOL / (ms / 1000.0)) / (n_done / t_plain),
                            "every_result_equals_batched": same}
        else:
            skipped["plain"] = f"budget: {left(args.budget):.0f} s left, needs about {est:.0f} s"
    del dgs
    torch.cuda.empty_cache()

    if not args.no_cpu:
        if left(args.budget) > args.cpu_seconds + 15:
            log("cpu baseline (oracle)")
            out["cpu_baseline"] = cpu_baseline(pool, args.cpu_seconds, golden)
        else:
            skipped["cpu_baseline"] = "budget"

    singles = {}
    costs = {"c0": ("c0", 2, None, None), "c1": ("c1", 8, None, None)}
    for key in ("c0", "c1"):
        if key in args.single and key in inputs:
            if left(args.budget) > costs[key][1] + 10:
                log(f"single {key}")
                tr = measured_traffic("peel_chunglu5m_traffic.md",
                                      ("peel.hip", "peel_common.h", "api.hip")) \
                    if key == "c1" else None
                singles[key] = single(key, inputs[key], 5 if key == "c1" else 20, 1, golden,
                                      traffic=tr)
                if key == "c1":
                    _, _, st_e = binding.bt_decompose_variant(
                        binding.DeviceGraph.upload(inputs["c1"], "cuda:0"),
                        binding.BT_PEEL_BATCH_EDGE, want_sup=False, stats=True)
                    singles[key]["ablation_batch_edge_only"] = {
                        "variant": "BiT-BU+ (batch edge processing only)",
                        "peel_ms": round(st_e["ms_peel_kernel"], 3),
                        "support_updates": st_e["support_updates"],
                        "peel_ms_batched": singles[key]["roofline"]["avg_launch_ms"],
                        "support_updates_batched": singles[key]["counters"]["support_updates"]}
            else:
                skipped[key] = "budget"
    if args.serve > 0:
        n_big = sum(1 for _, k, _ in arrivals if k == "big")
        est = 2.5 * n_big + 0.05 * len(arrivals) + 20
        if left(args.budget) > est + 10:
            log("serve")
            dsm = {k: binding.DeviceGraph.upload(pool[k], "cuda:0")
                   for k in sorted({k for _, kind, k in arrivals if kind == "small"})}
            dbg = {k: binding.DeviceGraph.upload(g, "cuda:0") for k, g in inputs["big"].items()}
            out["served"] = serve_compare(args.serve, dsm, dbg, arrivals, args.slots)
            del dsm, dbg
            torch.cuda.empty_cache()
        else:
            skipped["served"] = f"budget: needs about {est:.0f} s"
    if "c2" in args.single and "c2" in inputs:
        if left(args.budget) > 60:
            log("single c2 (BiT-PC)")
            singles["c2_pc"] = single("c2", inputs["c2"], 1, 0, golden, tau=0.05)
        else:
            skipped["c2_pc"] = "budget"
        if args.c2_plain:
            if left(args.budget) > 60:
                log("single c2 (plain peel)")
                singles["c2_plain"] = single("c2", inputs["c2"], 1, 0, golden)
            else:
                skipped["c2_plain"] = "budget"
    if singles:
        out["single"] = singles
    if skipped:
        out["skipped"] = skipped
    out["wall_s"] = round(time.perf_counter() - T_START, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
