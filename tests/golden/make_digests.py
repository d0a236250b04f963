"""Write tests/golden/digests.json (and digests_requests.json) from the CPU oracle.

For each seeded workload: SHA-256 of the oracle's int64 supports and int64
bitruss numbers (little-endian, edge order = CSR position), the butterfly
total and the generator version.  For the many-small-graphs pool the
digest covers the concatenation of the per-graph arrays in pool order.
Calls only `oracle` and the seeded generators.

  python tests/golden/make_digests.py [uniform10k] [chunglu5m] [hub20m] [hub20m:sup]
                                      [hub20m:vsF] [pool:N] [big:N] [bigs:A-B]

hub20m:vsF is the induced subgraph of the 20M-edge hub graph on a random
fraction F of each layer's vertices (sampling seed 2027), the protocol of
the paper's scalability experiments.  bigs:A-B adds request graphs A..B-1
one at a time to tests/golden/digests_requests.json (per-graph digests, a
file of their own so that long runs of other workloads, which rewrite
digests.json when they end, leave them alone); a run can be stopped and
resumed.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2001_06111_amd import synth  # noqa: E402

VS_SEED = 2027
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")
OUT_REQ = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests_requests.json")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def run(g):
    t0 = time.time()
    sup, bf, pairs = oracle.support(g.n_upper, g.n_lower, g.row_ptr, g.col)
    assert bf == pairs
    phi, st = oracle.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col, sup=sup)
    return sup, bf, phi, st, time.time() - t0


def main(args):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for a in args:
        if a in ("uniform10k", "chunglu5m", "hub20m"):
            g = {"uniform10k": synth.plain_uniform_10k, "chunglu5m": synth.plain_chunglu_5m,
                 "hub20m": synth.plain_hub_20m}[a]()
            sup, bf, phi, st, dt = run(g)
            data[g.name] = {"m": g.m, "butterflies": bf, "sup_sha256": sha(sup),
                            "phi_sha256": sha(phi), "max_phi": int(phi.max()) if g.m else 0,
                            "levels": st["levels"], "rounds": st["rounds"],
                            "oracle_seconds": round(dt, 1), "oracle_threads": oracle.max_threads(),
                            "generator_version": synth.GENERATOR_VERSION}
        elif a.startswith("hub20m:vs"):
            frac = float(a.split(":vs")[1])
            g = synth.vertex_sample(synth.plain_hub_20m(), frac, VS_SEED)
            sup, bf, phi, st, dt = run(g)
            data[g.name] = {"m": g.m, "n_upper": g.n_upper, "n_lower": g.n_lower,
                            "butterflies": bf, "sup_sha256": sha(sup),
                            "phi_sha256": sha(phi), "max_phi": int(phi.max()) if g.m else 0,
                            "levels": st["levels"], "rounds": st["rounds"],
                            "sample": {"of": "chunglu-100kx2M-m20M-hub", "fraction": frac,
                                       "seed": VS_SEED},
                            "oracle_seconds": round(dt, 1), "oracle_threads": oracle.max_threads(),
                            "generator_version": synth.GENERATOR_VERSION}
        elif a.startswith("bigs:"):
            lo, hi = (int(x) for x in a.split(":")[1].split("-"))
            req = json.load(open(OUT_REQ)) if os.path.exists(OUT_REQ) else {}
            ent = req.setdefault("per_graph", {})
            for j in range(lo, hi):
                if str(j) in ent:
                    continue
                g = synth.big_serving_graph(j)
                sup, bf, phi, st, dt = run(g)
                ent[str(j)] = {"m": g.m, "butterflies": bf, "sup_sha256": sha(sup),
                               "phi_sha256": sha(phi), "max_phi": int(phi.max()),
                               "oracle_seconds": round(dt, 1),
                               "oracle_threads": oracle.max_threads(),
                               "generator_version": synth.GENERATOR_VERSION}
                json.dump(req, open(OUT_REQ, "w"), indent=1, sort_keys=True)
                print(f"big {j}: m={g.m} bf={bf} {dt:.0f}s", flush=True)
            print("wrote", a, flush=True)
            continue
        elif a == "hub20m:sup":
            # Support counting only: the oracle's peel would take hours here.
            g = synth.plain_hub_20m()
            t0 = time.time()
            sup, bf, pairs = oracle.support(g.n_upper, g.n_lower, g.row_ptr, g.col)
            assert bf == pairs
            data[g.name] = {"m": g.m, "butterflies": bf, "sup_sha256": sha(sup),
                            "max_sup": int(sup.max()) if g.m else 0,
                            "oracle_support_seconds": round(time.time() - t0, 1),
                            "oracle_threads": oracle.max_threads(),
                            "generator_version": synth.GENERATOR_VERSION}
        elif a.startswith("pool:") or a.startswith("big:"):
            kind, n = a.split(":")
            n = int(n)
            hs, hp = hashlib.sha256(), hashlib.sha256()
            m_tot = bf_tot = 0
            t0 = time.time()
            per = []
            for i in range(n):
                g = synth.batch_graph(i) if kind == "pool" else synth.big_serving_graph(i)
                sup, bf, phi, _, _ = run(g)
                hs.update(np.ascontiguousarray(sup, dtype="<i8").tobytes())
                hp.update(np.ascontiguousarray(phi, dtype="<i8").tobytes())
                m_tot += g.m
                bf_tot += bf
                per.append({"m": g.m, "butterflies": bf, "phi_sha256": sha(phi)})
                print(f"{kind} {i}: m={g.m} bf={bf}", flush=True)
            data[f"{kind}:{n}"] = {"graphs": n, "m": m_tot, "butterflies": bf_tot,
                                   "sup_sha256": hs.hexdigest(), "phi_sha256": hp.hexdigest(),
                                   "per_graph": per[:64],
                                   "oracle_seconds": round(time.time() - t0, 1),
                                   "oracle_threads": oracle.max_threads(),
                                   "generator_version": synth.GENERATOR_VERSION}
        else:
            raise SystemExit(f"unknown workload {a}")
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print("wrote", a, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform10k"])
