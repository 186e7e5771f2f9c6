"""Input generators: determinism, sizes, and the SplitMix64 definition."""

import os

import workloads
from workloads import SplitMix64
from workloads.formulas import cnf_clause_count, random_dag_batch


def test_splitmix64_seed0():
    # first output of SplitMix64 from state 0 (published generator)
    assert SplitMix64(0).next() == 0xE220A8397B1DCDAF


def test_deterministic():
    assert workloads.random_3cnf(32, 136, 7) == workloads.random_3cnf(32, 136, 7)
    assert workloads.random_3cnf(32, 136, 7) != workloads.random_3cnf(32, 136, 8)
    assert workloads.random_dag(20, 300, 1) == workloads.random_dag(20, 300, 1)


def test_clause_counts():
    def lines(t):
        return len(t.strip().split("\n"))
    assert lines(workloads.equivalence_relations(6)[0]) == 60
    assert lines(workloads.equivalence_relations(6, deduplicate=False)[0]) == 120
    assert lines(workloads.equivalence_relations(9)[0]) == 252
    assert workloads.equivalence_relations(9)[1] == 36
    assert lines(workloads.permutation_matrices(5)[0]) == 110
    assert lines(workloads.triangle_free(8)[0]) == 56
    assert workloads.triangle_free(8)[1] == 28
    assert cnf_clause_count(32) == 136
    t, n = workloads.random_3cnf(32, 136, 0)
    assert lines(t) == 136 and n == 32


def test_3cnf_clauses_have_distinct_vars():
    t, n = workloads.random_3cnf(12, 51, 0)
    for line in t.strip().split("\n"):
        vs = [int(l.strip().lstrip("~x")) for l in line.split("|")]
        assert len(set(vs)) == 3 and all(0 <= v < n for v in vs)


def test_dag_batch_ranges():
    batch = random_dag_batch(64, 0)
    for text, n in batch:
        assert 10 <= n <= 30
        size = len(text.strip().split("\n")) - 1
        assert 50 <= size <= 2000


def test_serving_golden_matches_the_stream():
    """tests/golden/c4_requests.json (written by make_golden.py from the
    oracle) still describes the stream: a sample of its entries regenerated
    here has the same n and the oracle's count."""
    import json
    import os
    import random
    import oracle
    from workloads.serving import request_stream
    with open(os.path.join(os.path.dirname(__file__), "golden", "c4_requests.json")) as f:
        g = json.load(f)
    reqs = request_stream(g["requests"], 1.0, seed=0)
    ids = sorted(g["counts"], key=int)
    assert len(ids) > 6000
    assert {str(r["id"]) for r in reqs if r["kind"] == "3cnf" and r["n"] <= 20} == set(ids)
    for i in random.Random(4).sample(ids, 12):
        r = reqs[int(i)]
        assert r["n"] == g["counts"][i]["n"]
        assert oracle.count(r["text"], r["n"]) == g["counts"][i]["count"]


def test_traffic_digest_ignores_comments_only():
    """roofline.traffic is tied to the digest of the kernel sources' code: an
    edit of comments keeps it, an edit of code does not."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    code = 'x = 1; // one\n/* two\n three */ asm("s_nop 0\\n");  \n'
    assert b.code_of(code) == b.code_of('x = 1;\n asm("s_nop 0\\n"); // other words\n')
    assert b.code_of(code) != b.code_of('x = 2; asm("s_nop 0\\n");')
    assert len(b.kernel_sources_sha1()) == 40
