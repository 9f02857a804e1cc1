"""Write the stored expected values for the full-size parity cases.

Calls only the CPU oracle and the seeded generators; nothing here touches the
HIP library.  Run from the repository root:

    python tests/golden/make_goldens.py [config2|config3|config3lit|config4|all]

Each record holds the verdict (found, witness, K), the accepting count at
exit, the per-iteration |Del_k| list and the per-iteration map digests
(SHA-256 over their little-endian uint64 values, plus the first and last
few values in hex).
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
import synth  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "full_size.json")


def record(g, label):
    t = time.time()
    d = oracle.map_detect(g, mode="desc")
    dt = time.time() - t
    digests = d.trace[:, 2].astype(np.uint64)
    return {
        "label": label, "graph": g.name, "n": g.n, "m": g.m, "accepting": g.n_acc,
        "found": d.found, "witness": d.witness, "iterations": d.iterations,
        "accepting_left": d.accepting_left,
        "dels": [int(x) for x in d.trace[:, 0]],
        "digest_sha256": hashlib.sha256(digests.astype("<u8").tobytes()).hexdigest(),
        "digest_head": [f"{int(x):016x}" for x in digests[:8]],
        "digest_tail": [f"{int(x):016x}" for x in digests[-8:]],
        "oracle_seconds": round(dt, 1),
    }


def batch_record(count=4096, seed=4):
    """Verdicts of every graph of the config-4 batch: [found, witness, K, |A| at exit]."""
    t = time.time()
    rows, ns, ms = [], [], []
    for i in range(count):
        g = synth.config4(i, seed=seed)
        d = oracle.map_detect(g, mode="desc")
        rows.append([d.found, d.witness, d.iterations, d.accepting_left])
        ns.append(g.n)
        ms.append(g.m)
    return {"label": f"config 4 batch ({count} graphs, seed {seed})", "count": count, "seed": seed,
            "total_n": int(sum(ns)), "total_m": int(sum(ms)), "verdicts": rows,
            "oracle_seconds": round(time.time() - t, 1)}


def main(which):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if which in ("config2", "all"):
        data["c2B"] = record(synth.config2(), "config 2 variant B (no accepting cycle)")
        data["c2A"] = record(synth.config2(planted=True), "config 2 variant A (planted accepting 64-cycle)")
    if which in ("config3", "all"):
        data["c3"] = record(synth.config3(), "config 3 (2^25-vertex DAG, 0.1% accepting)")
    if which in ("config3lit", "all"):
        data["c3lit"] = record(synth.config1(seed=3, n=1 << 25, dag=True),
                               "config 3, literal reading (the config-1 generator at 2^25 vertices, edges "
                               "with s > d: a DAG of about 1.25 edges per vertex, 5% accepting)")
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    if which in ("config4", "all"):
        rec = batch_record()
        with open(os.path.join(ROOT, "tests", "golden", "batch_c4.json"), "w") as f:
            json.dump(rec, f, separators=(",", ":"))
        print("c4", rec["count"], rec["total_n"], rec["oracle_seconds"])
    for k, v in data.items():
        print(k, v["found"], v["witness"], v["iterations"], v["accepting_left"], v["oracle_seconds"])


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
