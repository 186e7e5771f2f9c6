"""GPU parity at the two full configurations that have no closed form per
case: the batch of 4096 random DAG formulas and the serving mix.

Counts are integers, so the bar is equality.  Expected values come from the
CPU oracle only: the stored per-formula counts of the DAG batch
(tests/golden/c3_dag_batch.json, written by make_golden.py from oracle/), the
stored theory counts (tests/golden/c2_theories.json), and oracle.count /
oracle.bitpar_count called here on the requests of the serving mix.
"""

import json
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads.formulas import random_3cnf, cnf_clause_count, random_dag_batch
from workloads.serving import request_stream, theory

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1310_6978_amd import fbg
    return fbg


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64).tolist()


@pytest.fixture(scope="module")
def dag_batch(F):
    """The 4096 formulas of the batched workload (seed 0), compiled once."""
    forms = random_dag_batch(4096, 0)
    progs = [F.Program(t, n) for t, n in forms]
    want = [r["count"] for r in golden("c3_dag_batch.json")["formulas"]]
    assert [r["n"] for r in golden("c3_dag_batch.json")["formulas"]] == [n for _, n in forms]
    return forms, progs, want


def test_dag_batch_counts_equal_the_oracle(F, dag_batch):
    """One batched count of all 4096 programs at the library's tiling."""
    _, progs, want = dag_batch
    print("dag batch: default tiling", flush=True)
    b = F.Batch(progs)
    got = host(b.count())
    b.free()
    bad = [i for i, (g, w) in enumerate(zip(got, want)) if g != w]
    assert not bad, "formulas %s differ (first: got %d want %d)" % (bad[:8], got[bad[0]], want[bad[0]])


@pytest.mark.parametrize("wpl", [8, 16, 32])
def test_dag_batch_at_fixed_tilings(F, dag_batch, wpl):
    _, progs, want = dag_batch
    print("dag batch: %d words per lane" % wpl, flush=True)
    b = F.Batch(progs, words_per_lane=wpl)
    assert host(b.count()) == want
    b.free()


def test_dag_batch_graph_replays(F, dag_batch):
    """The captured graph, replayed several times with eager work and
    synchronisations in between: every replay equals the oracle."""
    import torch
    _, progs, want = dag_batch
    print("dag batch: graph replays", flush=True)
    b = F.Batch(progs)
    out = torch.empty(len(progs), dtype=torch.int64, device="cuda")
    for rep in range(3):
        out.fill_(-1)                              # eager work between replays
        b.count(out=out, graph=True)
        assert host(out) == want, "replay %d" % rep
        eager = host(b.count())                    # the eager launch in between
        assert eager == want
    b.free()


def test_dag_batch_cofactor(F, dag_batch):
    _, progs, want = dag_batch
    print("dag batch: uniform cofactor", flush=True)
    b = F.Batch(progs, cofactor=True)
    assert host(b.count()) == want
    b.free()


def test_dag_batch_sample_alone(F, dag_batch):
    """A sample of single-program launches equals the batched counts."""
    _, progs, want = dag_batch
    for i in range(0, 4096, 97):
        assert host(F.count(progs[i]))[0] == want[i], i


def _serving_mix():
    """A seeded slice of the serving stream with its real shape (n in
    [12, 36], 10 % theories), plus forced requests of every heavy kind: the
    k=9 equivalence theory (36 letters), the 5x5 permutations, the k=8
    triangle-free graphs and a 36-variable 3-CNF."""
    reqs = request_stream(96, 3000.0, seed=0)
    extra = [theory("equivalence_k9") + ("equivalence_k9",), theory("permutations_k5") + ("permutations_k5",),
             theory("triangle_free_k8") + ("triangle_free_k8",),
             random_3cnf(36, cnf_clause_count(36), 7) + ("3cnf",)]
    last = reqs[-1]["arrival"]
    for k, (text, n, kind) in enumerate(extra):
        reqs.append({"id": len(reqs), "arrival": last * (k + 1) / (len(extra) + 1), "kind": kind, "text": text,
                     "n": n})
    return reqs


def test_serving_mix_alone_equals_mixed_and_oracle(F):
    import torch
    from paper_1310_6978_amd.serve import ServeLoop
    reqs = _serving_mix()
    kinds = {r["kind"] for r in reqs}
    assert {"equivalence_k9", "permutations_k5", "triangle_free_k8", "3cnf"} <= kinds
    assert max(r["n"] for r in reqs) == 36
    print("serving mix: %d requests" % len(reqs), flush=True)
    loop = ServeLoop(words_per_lane=16, slice_words=4e9, max_active=64)
    res = loop.run(reqs, realtime=True)
    loop.close()
    assert res["requests"] == len(reqs)
    mixed = res["counts"]
    th = golden("c2_theories.json")
    checked_oracle = 0
    for r in reqs:
        if r["kind"] != "3cnf":
            assert mixed[r["id"]] == th[r["kind"]]["count"], r["kind"]
        elif r["n"] <= 26:
            assert mixed[r["id"]] == oracle.count(r["text"], r["n"]), (r["id"], r["n"])
            checked_oracle += 1
        elif r["n"] <= 30:
            assert mixed[r["id"]] == oracle.bitpar_count(r["text"], r["n"]), (r["id"], r["n"])
            checked_oracle += 1
    assert checked_oracle >= 40
    print("serving mix: theories and %d 3-CNF requests equal the oracle; alone runs next" % checked_oracle,
          flush=True)
    # every request alone: one program, one launch
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    for r in reqs:
        p = F.Program(r["text"], r["n"])
        assert host(F.count(p, out=out))[0] == mixed[r["id"]], (r["id"], r["kind"], r["n"])
        p.free()
    assert res["latency_p99_ms"] >= res["latency_p50_ms"] > 0
