"""Writes the stored expected values under tests/golden/.

Every value here is computed by the CPU oracle (``oracle/``) from inputs made
by ``workloads/``; nothing comes from the GPU path.  Run from the repository
root:

    python tests/golden/make_golden.py [c0 c1 c2 c3 ...]

Files written (JSON):
  c0_equivalence_k6.json   DNF words (hex) and models of the k=6 theory
  c1_3cnf_n32.json         per seed: count and ascending model indices
  c2_theories.json         equivalence k=9, 5x5 permutations, triangle-free
                           k=8: counts, model lists (or a SHA-256 of the
                           little-endian uint64 model array when large)
  c3_dag_batch.json        per formula of the 4096-DAG batch: n and count
  c4_requests.json         the serving stream (seed 0, any arrival rate > 0):
                           the count of every random 3-CNF request with
                           n <= 20 among the first 20,000
"""

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402
from workloads.formulas import random_dag_batch  # noqa: E402

C1_SEEDS = list(range(16))
C3_SEED = 0
C3_COUNT = 4096
C4_REQUESTS = 20000


def models_sha256(arr):
    return hashlib.sha256(np.ascontiguousarray(arr, dtype="<u8").tobytes()).hexdigest()


def write(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    print("wrote", path, flush=True)


def c0():
    text, n = workloads.equivalence_relations(6)
    d = oracle.dnf(text, n)
    m, total = oracle.models(text, n)
    write("c0_equivalence_k6.json", {
        "workload": "equivalence relations k=6 (60 transitivity clauses)",
        "n": n, "count": int(total),
        "dnf_words_hex": ["%016x" % int(w) for w in d],
        "models": [int(v) for v in m],
    })


def c1():
    out = {"workload": "random 3-CNF n=32 m=136", "n": 32, "m": 136, "seeds": {}}
    for s in C1_SEEDS:
        t0 = time.time()
        text, n = workloads.random_3cnf(32, 136, s)
        m, total = oracle.models(text, n)
        out["seeds"][str(s)] = {"count": int(total), "models": [int(v) for v in m]}
        print("c1 seed", s, "count", total, "%.1fs" % (time.time() - t0), flush=True)
        write("c1_3cnf_n32.json", out)


def c2():
    out = {}
    for key, (text, n) in (("permutations_k5", workloads.permutation_matrices(5)),
                           ("triangle_free_k8", workloads.triangle_free(8)),
                           ("equivalence_k9", workloads.equivalence_relations(9))):
        t0 = time.time()
        m, total = oracle.models(text, n)
        rec = {"n": n, "count": int(total), "models_sha256": models_sha256(m)}
        if total <= 50000:
            rec["models"] = [int(v) for v in m]
        out[key] = rec
        print("c2", key, total, "%.1fs" % (time.time() - t0), flush=True)
        write("c2_theories.json", out)


def c3():
    batch = random_dag_batch(C3_COUNT, C3_SEED)
    out = {"workload": "4096 random DAGs, n in [10,30], size in [50,2000], seed 0",
           "count_method": "blocked evaluation (orc_bitpar_count); per-valuation "
                           "oracle also run where 2^n * size <= 2^30",
           "formulas": []}
    t0 = time.time()
    for i, (text, n) in enumerate(batch):
        c = oracle.bitpar_count(text, n)
        size = text.count("\n") - 1
        rec = {"n": n, "count": int(c)}
        if (1 << n) * size <= (1 << 30):
            c2 = oracle.count(text, n)
            if c2 != c:
                raise SystemExit("per-valuation and blocked oracle disagree on formula %d" % i)
            rec["checked_per_valuation"] = True
        out["formulas"].append(rec)
        if i % 256 == 255:
            print("c3", i + 1, "%.1fs" % (time.time() - t0), flush=True)
    write("c3_dag_batch.json", out)


def c4():
    from workloads.serving import request_stream
    reqs = request_stream(C4_REQUESTS, 1.0, seed=0)  # the texts do not depend on the rate
    out = {"workload": "serving stream, seed 0, first %d requests: 3-CNF requests with n <= 20" % C4_REQUESTS,
           "requests": C4_REQUESTS, "counts": {}}
    t0 = time.time()
    for r in reqs:
        if r["kind"] == "3cnf" and r["n"] <= 20:
            out["counts"][str(r["id"])] = {"n": r["n"], "count": int(oracle.count(r["text"], r["n"]))}
    print("c4", len(out["counts"]), "requests %.1fs" % (time.time() - t0), flush=True)
    write("c4_requests.json", out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c0", "c2", "c3", "c1"]
    for w in which:
        globals()[w]()
