"""GPU parity of the uniform-cofactor variant (FBG_TUNE_COFACTOR): on every
tile the tile variables are constants, so clauses that they satisfy are
skipped and a clause that they falsify ends the tile.  The variant must give
the same DNF words, counts and models as the oracle, bit for bit."""

import json
import os
import random

import numpy as np
import pytest

import oracle
import workloads
from tests.formula_gen import random_cnf, random_program

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WPL = [1, 2, 4, 8, 16, 32]


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1310_6978_amd import fbg
    return fbg


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def cof_check(F, text, n, wpls=WPL):
    want = oracle.dnf(text, n)
    total = int(np.unpackbits(want.view(np.uint8)).sum())
    p = F.Program(text, n)
    for w in wpls:
        got = host(F.eval_dnf(p, words_per_lane=w, cofactor=True))
        assert np.array_equal(got, want), ("dnf", w, n)
        assert int(host(F.count(p, words_per_lane=w, cofactor=True))[0]) == total, ("count", w, n)
    return p, total


@pytest.mark.parametrize("seed", range(8))
def test_random_cnf(F, seed):
    rng = random.Random(7100 + seed)
    n = rng.choice([18, 20, 22, 23])
    cof_check(F, random_cnf(rng, n, rng.randrange(4, 60)), n)


@pytest.mark.parametrize("seed", range(6))
def test_random_formulas_general_code(F, seed):
    rng = random.Random(7300 + seed)
    n = rng.choice([12, 16, 18, 20])
    _, text = random_program(rng, n)
    cof_check(F, text, n)


def test_dead_tiles_and_unit_clauses(F):
    # tile-only clauses (high variables only) that kill most tiles, mixed
    # with clauses over in-word, lane and word variables
    for text, n in (("x22 & ~x21 & (x0 | x7 | x12)", 23),
                    ("(x20 | x21) & (~x20 | ~x22) & (x1 | ~x15) & ~x19", 23),
                    ("x19 & ~x19", 20),                      # unsatisfiable
                    ("(x23 | ~x23) & (x3 | x4)", 24),        # tautological clause
                    ("~x0 & (x17 | x18 | x19 | x20)", 21)):
        cof_check(F, text, n)


def test_c1_instances_count_and_models(F):
    path = os.path.join(GOLDEN, "c1_3cnf_n32.json")
    if not os.path.exists(path):
        pytest.skip("c1 golden not generated")
    with open(path) as f:
        g = json.load(f)
    for s, rec in sorted(g["seeds"].items(), key=lambda kv: int(kv[0]))[:4]:
        text, n = workloads.random_3cnf(32, 136, int(s))
        p = F.Program(text, n)
        for w in (8, 16, 32):
            assert int(host(F.count(p, words_per_lane=w, cofactor=True))[0]) == rec["count"], (s, w)
        p.set_tuning(16, cofactor=True)        # enumeration takes the program's default
        idx, tot = F.enumerate_models(p, 4096)
        t = int(host(tot)[0])
        assert t == rec["count"]
        assert host(idx)[:t].tolist() == rec["models"]


def test_enumeration_with_default_cofactor(F):
    text, n = workloads.random_3cnf(22, 93, 5)
    want, total = oracle.models(text, n)
    p = F.Program(text, n)
    p.set_tuning(4, cofactor=True)
    idx, tot = F.enumerate_models(p, total + 3)
    assert int(host(tot)[0]) == total
    assert np.array_equal(host(idx)[:total], want)


def test_batch_and_server(F):
    import torch
    rng = random.Random(11)
    texts = [workloads.random_3cnf(rng.choice([14, 18, 22]), 60, s) for s in range(8)]
    texts += [workloads.random_dag(18, 300, 4), workloads.triangle_free(6)]
    progs = [F.Program(t, n) for t, n in texts]
    want = [oracle.count(t, n) for t, n in texts]
    for wpl in (1, 16):
        assert host(F.count_batch(progs, words_per_lane=wpl, cofactor=True)).tolist() == want, wpl
    b = F.Batch(progs, words_per_lane=8, cofactor=True)
    assert host(b.count()).tolist() == want
    assert host(b.count(graph=True)).tolist() == want
    sv = F.Server(len(progs), 64, 8, nbuf=2, cofactor=True)
    counts = torch.zeros(len(progs), dtype=torch.int64, device="cuda")
    items = [(i, i, 0, F.program_tiles(p, 8)) for i, p in enumerate(progs)]
    sv.launch(progs, items, counts)
    assert host(counts).tolist() == want
    sv.free()


def many_tile_clauses(n, lo, count, seed):
    """count distinct 3-clauses over the tile variables lo .. n-1, each true
    under one planted assignment (so some tiles live), then clauses that
    reach the in-word, lane and word variables."""
    rng = random.Random(seed)
    plant = {v: rng.random() < 0.5 for v in range(lo, n)}
    parts = set()
    while len(parts) < count:
        vs = sorted(rng.sample(range(lo, n), 3))
        keep = rng.choice(vs)                   # this literal holds under the plant
        lits = []
        for v in vs:
            neg = (not plant[v]) if v == keep else rng.random() < 0.5
            lits.append(("~x%d" if neg else "x%d") % v)
        parts.add(" | ".join(lits))
    parts = sorted(parts) + ["x0 | ~x%d | x3" % (lo + 1), "~x5 | x%d" % (n - 1), "x9 | x12 | ~x14"]
    return " & ".join("(%s)" % c for c in parts)


def test_more_tile_clauses_than_a_chunk(F):
    # 48 tile-only clauses at 32 words per lane (tile variables 16 .. 24),
    # more at smaller tilings: the test reads all of them from the block's
    # table; tiles visited in hashed order (single-program launches) and
    # interleaved pieces (batch, server) must still cover every tile once
    import torch
    n = 25
    text = many_tile_clauses(n, 16, 48, 9)
    p, total = cof_check(F, text, n)
    assert 0 < total < (1 << n) // 20           # most valuations are not models
    want, _ = oracle.models(text, n)
    for w in (1, 16, 32):
        p.set_tuning(w, cofactor=True)
        idx, tot = F.enumerate_models(p, total + 5)
        assert int(host(tot)[0]) == total
        assert np.array_equal(host(idx)[:total], want), w
    other = F.Program(workloads.random_3cnf(20, 85, 3)[0], 20)
    progs = [p, other, p]
    cnts = [total, oracle.count(*workloads.random_3cnf(20, 85, 3)), total]
    for wpl in (1, 8, 32):
        b = F.Batch(progs, words_per_lane=wpl, cofactor=True)
        assert host(b.count()).tolist() == cnts, wpl
    for wpl in (1, 16):
        sv = F.Server(len(progs), 256, wpl, nbuf=2, cofactor=True)
        counts = torch.zeros(len(progs), dtype=torch.int64, device="cuda")
        nt = F.program_tiles(p, wpl)
        # one request split over two launches, the second from an odd tile
        items = [(0, 0, 0, nt // 3), (1, 1, 0, F.program_tiles(other, wpl)), (2, 2, 0, nt)]
        sv.launch(progs, items, counts)
        sv.launch(progs[:1], [(0, 0, nt // 3, nt)], counts)
        assert host(counts).tolist() == cnts, wpl
        sv.free()


def test_c2a_equivalence_k9_with_cofactor(F):
    # 90 tile-only clauses at 32 words per lane, 105 at 16; most tiles dead
    path = os.path.join(GOLDEN, "c2_theories.json")
    with open(path) as f:
        g = json.load(f)["equivalence_k9"]
    text, n = workloads.equivalence_relations(9)
    p = F.Program(text, n)
    for w in (8, 16, 32):
        assert int(host(F.count(p, words_per_lane=w, cofactor=True))[0]) == 21147 == g["count"], w
    for w in (16, 32):
        p.set_tuning(w, cofactor=True)
        idx, tot = F.enumerate_models(p, 30000)
        assert int(host(tot)[0]) == 21147
        assert host(idx)[:21147].tolist() == g["models"], w


def test_c2c_triangle_free_with_cofactor(F):
    import hashlib
    with open(os.path.join(GOLDEN, "c2_theories.json")) as f:
        g = json.load(f)["triangle_free_k8"]
    text, n = workloads.triangle_free(8)
    p = F.Program(text, n)
    p.set_tuning(16, cofactor=True)
    idx, tot = F.enumerate_models(p, g["count"])
    assert int(host(tot)[0]) == g["count"]
    assert hashlib.sha256(host(idx)[:g["count"]].astype("<u8").tobytes()).hexdigest() == g["models_sha256"]
