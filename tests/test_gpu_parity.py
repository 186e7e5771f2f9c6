"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact throughout: DNF words, counts and model lists are integers.  Small
cases compare every element with the oracle; full-size cases compare against
stored oracle results (tests/golden, written by make_golden.py) and check
sampled DNF words and every enumerated model with the oracle one valuation
at a time.
"""

import hashlib
import json
import os
import random

import numpy as np
import pytest

import oracle
import workloads
from tests.formula_gen import many_registers, random_cnf, random_program

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


def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("golden file %s not generated" % name)
    with open(path) as f:
        return json.load(f)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def gpu_dnf(F, p, wpl=0):
    return host(F.eval_dnf(p, words_per_lane=wpl))


def gpu_count(F, p, wpl=0):
    return int(host(F.count(p, words_per_lane=wpl))[0])


def gpu_models(F, p, cap):
    idx, tot = F.enumerate_models(p, cap)
    return host(idx)[:cap].copy(), int(host(tot)[0])


def full_check(F, text, n, wpls=WPL):
    """DNF, count and models for every tiling against the oracle."""
    want = oracle.dnf(text, n)
    want_models, total = oracle.models(text, n)
    p = F.Program(text, n)
    for w in wpls:
        got = gpu_dnf(F, p, w)
        assert np.array_equal(got, want), ("dnf", w, n)
        assert gpu_count(F, p, w) == total, ("count", w, n)
    m, t = gpu_models(F, p, max(total, 1))
    assert t == total
    assert np.array_equal(m[:total], want_models)
    return p


def test_generators_are_the_rows_of_M(F):
    # Section 2.2: bit mu of generator k is bit k of mu
    for n in range(0, 13):
        for k in range(n):
            p = F.Program("x%d" % k, n)
            assert np.array_equal(gpu_dnf(F, p), oracle.dnf("x%d" % k, n)), (n, k)


def test_small_n_tails(F):
    for n in range(0, 8):
        for text in ("1", "0", "x0" if n else "1", "~x%d" % (n - 1) if n else "0"):
            full_check(F, text, n)


@pytest.mark.parametrize("seed", range(24))
def test_random_formulas(F, seed):
    rng = random.Random(500 + seed)
    n = rng.choice([3, 6, 9, 12, 14, 16, 17, 18, 20])
    _, text = random_program(rng, n)
    full_check(F, text, n)


def multi_literal_cnf(rng, n, nmulti):
    """CNF whose clauses mostly carry two or more literals on the word-index
    variables x11..x15, plus a few ordinary 3-clauses."""
    clauses = []
    for _ in range(nmulti):
        k = rng.choice([2, 3, 3, 4])
        vs = rng.sample(range(11, 16), min(k, 5) - 1) + [rng.randrange(n)]
        clauses.append("(" + " | ".join(("~" if rng.random() < 0.5 else "") + "x%d" % v for v in vs) + ")")
    for _ in range(8):
        vs = rng.sample(range(n), 3)
        clauses.append("(" + " | ".join(("~" if rng.random() < 0.5 else "") + "x%d" % v for v in vs) + ")")
    return " & ".join(clauses)


@pytest.mark.parametrize("seed", range(6))
def test_multi_literal_keys_inside_and_after_the_tree(F, seed):
    # the first 32 multi-literal clauses act inside the product tree at their
    # level and half, the rest after it: every tiling, both variants, batched
    rng = random.Random(4900 + seed)
    n = rng.choice([17, 19, 22])
    text = multi_literal_cnf(rng, n, rng.choice([12, 40, 75]))
    p = full_check(F, text, n, wpls=[4, 8, 16, 32])
    want = oracle.dnf(text, n)
    for w in (8, 32):
        assert np.array_equal(host(F.eval_dnf(p, words_per_lane=w, cofactor=True)), want), w
    q = F.Program(multi_literal_cnf(random.Random(seed), n, 20), n)
    got = host(F.count_batch([p, q], words_per_lane=32)).tolist()
    assert got == [gpu_count(F, p, 32), gpu_count(F, q, 32)]


@pytest.mark.parametrize("seed", range(8))
def test_random_cnf_several_tiles(F, seed):
    rng = random.Random(700 + seed)
    n = rng.choice([18, 19, 20, 21])
    full_check(F, random_cnf(rng, n, rng.randrange(4, 30)), n)


@pytest.mark.parametrize("seed", range(6))
def test_random_dags(F, seed):
    rng = random.Random(900 + seed)
    n = rng.choice([10, 14, 18, 20])
    text, n = workloads.random_dag(n, rng.randrange(50, 2000), seed)
    full_check(F, text, n)


def test_baequ4(F):
    text, n = workloads.baequ4()
    p = full_check(F, text, n)
    m, t = gpu_models(F, p, 8)
    assert t == 3 and m[:t].tolist() == [0, 9, 15]


def test_c0_equivalence_k6(F):
    g = golden("c0_equivalence_k6.json")
    text, n = workloads.equivalence_relations(6)
    p = F.Program(text, n)
    want = np.array([int(h, 16) for h in g["dnf_words_hex"]], dtype=np.uint64)
    for w in WPL:
        assert np.array_equal(gpu_dnf(F, p, w), want)
        assert gpu_count(F, p, w) == 203
    m, t = gpu_models(F, p, 1000)
    assert t == 203 and m[:203].tolist() == g["models"]


def test_c2b_permutations(F):
    g = golden("c2_theories.json")["permutations_k5"]
    text, n = workloads.permutation_matrices(5)
    p = F.Program(text, n)
    assert gpu_count(F, p) == 120 == g["count"]
    m, t = gpu_models(F, p, 200)
    assert t == 120 and m[:120].tolist() == g["models"]


def test_c2c_triangle_free(F):
    g = golden("c2_theories.json")["triangle_free_k8"]
    text, n = workloads.triangle_free(8)
    p = F.Program(text, n)
    assert gpu_count(F, p) == 4682270 == g["count"]
    m, t = gpu_models(F, p, 4682270)
    assert t == 4682270
    assert hashlib.sha256(m.astype("<u8").tobytes()).hexdigest() == g["models_sha256"]
    d = gpu_dnf(F, p)
    assert int(np.unpackbits(d.view(np.uint8)).sum()) == 4682270
    # every set bit of the DNF is a model and vice versa
    bits = np.flatnonzero(np.unpackbits(d.view(np.uint8), bitorder="little"))
    assert np.array_equal(bits.astype(np.uint64), m)


def test_c2a_equivalence_k9(F):
    text, n = workloads.equivalence_relations(9)
    p = F.Program(text, n)
    assert gpu_count(F, p) == 21147  # Bell number B_9
    m, t = gpu_models(F, p, 30000)
    assert t == 21147
    m = m[:t]
    assert np.all(np.diff(m.astype(np.int64)) > 0)
    assert np.all(oracle.eval_at(text, n, m) == 1)
    g = golden("c2_theories.json").get("equivalence_k9")
    if g:
        assert m.tolist() == g["models"]


def test_c1_random_3cnf_counts_and_models(F):
    g = golden("c1_3cnf_n32.json")
    for s, rec in sorted(g["seeds"].items(), key=lambda kv: int(kv[0])):
        text, n = workloads.random_3cnf(32, 136, int(s))
        p = F.Program(text, n)
        assert gpu_count(F, p) == rec["count"], s
        m, t = gpu_models(F, p, 4096)
        assert t == rec["count"]
        assert m[:t].tolist() == rec["models"]


def test_c1_dnf_sampled_words(F):
    import torch
    text, n = workloads.random_3cnf(32, 136, 0)
    p = F.Program(text, n)
    d = F.eval_dnf(p)
    rng = np.random.default_rng(1)
    words = np.sort(rng.choice(d.numel(), 256, replace=False))
    sample = d[torch.from_numpy(words.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
    idx = (words[:, None].astype(np.uint64) * 64 + np.arange(64, dtype=np.uint64)[None, :]).ravel()
    bits = oracle.eval_at(text, n, idx).reshape(-1, 64)
    want = (bits.astype(np.uint64) << np.arange(64, dtype=np.uint64)[None, :]).sum(axis=1).astype(np.uint64)
    assert np.array_equal(sample, want)
    assert gpu_count(F, p) == oracle_count_golden(0)


def oracle_count_golden(seed):
    path = os.path.join(GOLDEN, "c1_3cnf_n32.json")
    if not os.path.exists(path):
        pytest.skip("c1 golden not generated")
    with open(path) as f:
        return json.load(f)["seeds"][str(seed)]["count"]


def test_enumerate_truncation(F):
    text, n = workloads.triangle_free(6)
    want, total = oracle.models(text, n)
    p = F.Program(text, n)
    for cap in (0, 1, 7, 100, total - 1, total, total + 5):
        m, t = gpu_models(F, p, cap)
        assert t == total
        assert np.array_equal(m[:min(cap, total)], want[:min(cap, total)])


def test_determinism(F):
    text, n = workloads.random_3cnf(24, 102, 3)
    p = F.Program(text, n)
    a, b = gpu_dnf(F, p), gpu_dnf(F, p)
    assert np.array_equal(a, b)
    assert gpu_count(F, p) == gpu_count(F, p) == oracle.count(text, n)


def test_batch_equals_solo_and_oracle(F):
    rng = random.Random(42)
    progs, want = [], []
    for i in range(40):
        n = rng.choice([4, 9, 12, 15, 18, 20, 22])
        if i % 3 == 0:
            text, n = workloads.random_dag(n, rng.randrange(50, 800), i)
        else:
            text = random_cnf(rng, n, rng.randrange(1, 30))
        progs.append(F.Program(text, n))
        want.append(oracle.count(text, n))
    for wpl in (0, 1, 4, 16):
        got = host(F.count_batch(progs, words_per_lane=wpl))
        assert got.tolist() == want, wpl
    b = F.Batch(progs)
    for _ in range(3):
        assert host(b.count()).tolist() == want
    solo = [gpu_count(F, p) for p in progs]
    assert solo == want


def test_argument_errors(F):
    import torch
    p = F.Program("x0 | x9", 12)
    small = torch.empty(3, dtype=torch.int64, device="cuda")
    with pytest.raises(F.FbgError) as ei:
        F.eval_dnf(p, out=small)
    assert ei.value.status == F.FBG_E_INVAL
    with pytest.raises(F.FbgError):
        F.count(p, words_per_lane=3)
    big = F.Program("x40", 41)
    with pytest.raises(F.FbgError) as ei:
        F.eval_dnf(big, out=small)
    assert ei.value.status == F.FBG_E_RANGE


def test_enumerate_from_stored_dnf(F):
    for text, n in (workloads.triangle_free(6), workloads.baequ4(), workloads.random_3cnf(22, 93, 5),
                    ("x0 | ~x0", 3), ("0", 9)):
        want, total = oracle.models(text, n)
        p = F.Program(text, n)
        d = F.eval_dnf(p)
        for cap in (0, 3, total + 1):
            idx, tot = F.enumerate_dnf(d, n, cap)
            got = host(idx)[:min(cap, total)]
            assert int(host(tot)[0]) == total
            assert np.array_equal(got, want[:min(cap, total)])


def test_server_items_add_up(F):
    import torch
    rng = random.Random(7)
    texts = [workloads.random_3cnf(rng.choice([12, 16, 20, 23]), 40, s) for s in range(6)]
    texts.append(workloads.triangle_free(6))
    texts.append(workloads.random_dag(18, 300, 4))
    progs = [F.Program(t, n) for t, n in texts]
    want = [oracle.count(t, n) for t, n in texts]
    for wpl in (1, 8, 32):
        sv = F.Server(len(progs), 64, wpl, nbuf=2)
        counts = torch.zeros(len(progs) + 3, dtype=torch.int64, device="cuda")
        # every program's tiles cut into random ranges, spread over launches
        pending = []
        for i, p in enumerate(progs):
            nt = F.program_tiles(p, wpl)
            cuts = sorted(set([0, nt] + [rng.randrange(0, nt + 1) for _ in range(3)]))
            pending += [(i, i + 3, a, b) for a, b in zip(cuts, cuts[1:])]
        rng.shuffle(pending)
        while pending:
            take, pending = pending[:5], pending[5:]
            used = sorted(set(it[0] for it in take))
            local = {g: k for k, g in enumerate(used)}
            sv.launch([progs[g] for g in used], [(local[a], b, c, d) for a, b, c, d in take], counts)
        got = host(counts).tolist()
        assert got[:3] == [0, 0, 0]
        assert got[3:] == want, wpl
        sv.free()


def test_server_rejects_bad_items(F):
    import torch
    p = F.Program("x1 | x7", 12)
    sv = F.Server(4, 8, 4)
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    nt = F.program_tiles(p, 4)
    for bad in ([(1, 0, 0, nt)], [(0, 2, 0, nt)], [(0, 0, 0, nt + 1)], [(0, 0, 2, 1)]):
        with pytest.raises(F.FbgError) as ei:
            sv.launch([p], bad, counts)
        assert ei.value.status == F.FBG_E_INVAL
    sv.free()


def test_programs_compiled_for_some_tilings(F):
    """Programs encoded only for the tilings asked for (FBG_COMPILE_WPL)
    count as full compiles at those tilings, alone, batched and served; the
    host refuses every other tiling before anything is launched."""
    import torch
    texts = [workloads.random_3cnf(16, 40, 1), workloads.random_dag(18, 300, 4), workloads.triangle_free(6)]
    want = [oracle.count(t, n) for t, n in texts]
    progs = [F.Program(t, n, F.compile_wpl(16)) for t, n in texts]
    assert [gpu_count(F, p) for p in progs] == want
    assert [gpu_count(F, p, 16) for p in progs] == want
    assert host(F.Batch(progs, words_per_lane=16).count()).tolist() == want
    sv = F.Server(len(progs), 8, 16, nbuf=2)
    counts = torch.zeros(len(progs), dtype=torch.int64, device="cuda")
    sv.launch(progs, [(i, i, 0, F.program_tiles(p, 16)) for i, p in enumerate(progs)], counts)
    assert host(counts).tolist() == want
    sv.free()
    for call in (lambda: F.count(progs[0], words_per_lane=8),
                 lambda: F.eval_dnf(progs[1], words_per_lane=32),
                 lambda: F.Batch(progs, words_per_lane=4)):
        with pytest.raises(F.FbgError) as ei:
            call()
        assert ei.value.status == F.FBG_E_INVAL
    sv = F.Server(len(progs), 8, 8, nbuf=2)
    with pytest.raises(F.FbgError) as ei:
        sv.launch(progs[:1], [(0, 0, 0, F.program_tiles(progs[0], 8))], counts)
    assert ei.value.status == F.FBG_E_INVAL
    sv.free()
    # clause-only programs at 32 words per lane keep the XCD-local write-out
    t, n = workloads.random_3cnf(22, 60, 3)
    full, part = F.Program(t, n), F.Program(t, n, F.compile_wpl(32))
    assert np.array_equal(gpu_dnf(F, part, 32), gpu_dnf(F, full, 32))


def test_batch_graph_replays_match_eager(F):
    import torch
    rng = random.Random(3)
    texts = [workloads.random_dag(rng.choice([12, 16, 20]), rng.randrange(50, 600), i) for i in range(30)]
    texts += [workloads.random_3cnf(22, 93, s) for s in range(6)]
    progs = [F.Program(t, n) for t, n in texts]
    want = [oracle.count(t, n) for t, n in texts]
    b = F.Batch(progs)
    eager = host(b.count()).tolist()
    assert eager == want
    out = torch.zeros(len(progs), dtype=torch.int64, device="cuda")
    for rep in range(4):
        # eager work and synchronisation between replays
        junk = torch.arange(1000, device="cuda").sum()
        torch.cuda.synchronize()
        out.fill_(-1)
        b.count(out=out, graph=True)
        assert host(out).tolist() == want, rep
        del junk


def test_autotuner_choice_is_exact(F, tmp_path):
    from paper_1310_6978_amd import autotune
    text, n = workloads.random_3cnf(24, 102, 9)
    p = F.Program(text, n)
    t = autotune.Tuner(path=str(tmp_path / "tune.json"), reps=2)
    w = t.apply(p)
    assert w in autotune.CANDIDATES and p.info["words_per_lane"] == w
    assert gpu_count(F, p) == oracle.count(text, n)
    entry = t.table[autotune.key_of(p)]
    assert len(entry["ms"]) == 2 * len(autotune.CANDIDATES)      # with and without the cofactor test
    m, tot = gpu_models(F, p, 1 << 16)                           # the enumeration takes the choice too
    want, total = oracle.models(text, n)
    assert tot == total and np.array_equal(m[:total], want)
    # the theory whose tile-only clauses kill most tiles: the cofactor wins
    eq, ne = workloads.equivalence_relations(9)
    q = F.Program(eq, ne)
    t.apply(q)
    assert t.table[autotune.key_of(q)]["cofactor"] is True
    assert gpu_count(F, q) == 21147                              # Bell number B_9


def test_batch_eval_dnf_writes_every_vector(F):
    import torch
    rng = random.Random(77)
    texts = [("x0", 1), ("~x2 | x1", 3), ("0", 7)]
    texts += [workloads.random_3cnf(rng.choice([12, 17, 21, 23]), 50, s) for s in range(5)]
    texts += [workloads.random_dag(rng.choice([14, 19]), rng.randrange(50, 400), s) for s in range(4)]
    texts.append(workloads.triangle_free(6))
    progs = [F.Program(t, n) for t, n in texts]
    outs = [torch.full((F.dnf_words(n) + 3,), -1, dtype=torch.int64, device="cuda") for _, n in texts]
    for wpl, cof in ((0, False), (1, False), (16, True), (32, False)):
        b = F.Batch(progs, words_per_lane=wpl, cofactor=cof)
        b.set_dnf_outputs(outs)
        for rep in range(2):
            for o in outs:
                o.fill_(-1)
            counts = host(b.eval_dnf())
            for (t, n), o, c in zip(texts, outs, counts):
                want = oracle.dnf(t, n)
                got = host(o)
                assert np.array_equal(got[:len(want)], want), (wpl, n, t[:60])
                assert np.all(got[len(want):] == np.uint64(2**64 - 1))   # nothing past the vector
                assert int(c) == int(np.unpackbits(want.view(np.uint8)).sum())
        b.free()


def test_dnf_on_any_grid(F):
    """The single-program DNF write-out runs one wave per tile by default;
    an explicit grid (a single block, a few blocks, more than the tiles)
    strides over the tiles instead, with the same words."""
    texts = [workloads.random_3cnf(19, 80, 2), workloads.random_dag(17, 250, 9), ("x2 | x15", 21)]
    for t, n in texts:
        p = F.Program(t, n)
        want = oracle.dnf(t, n)
        for w in (1, 4, 32):
            for grid in (0, 1, 7, 1 << 20):
                got = host(F.eval_dnf(p, words_per_lane=w, grid_blocks=grid))
                assert np.array_equal(got, want), (n, w, grid)


def test_dnf_into_offset_views(F):
    """An output that starts 8 bytes past an aligned address (a view into a
    larger buffer) receives the same words, solo and batched, and nothing
    around it is written."""
    import torch
    texts = [workloads.random_3cnf(21, 90, 3), workloads.random_dag(19, 300, 5), ("x4 & ~x17", 24)]
    progs = [F.Program(t, n) for t, n in texts]
    for (t, n), p in zip(texts, progs):
        want = oracle.dnf(t, n)
        for w in (0, 4, 8, 16, 32):
            for off in (0, 1):
                buf = torch.full((F.dnf_words(n) + 2,), -1, dtype=torch.int64, device="cuda")
                got = host(F.eval_dnf(p, out=buf[off:off + F.dnf_words(n)], words_per_lane=w))
                assert np.array_equal(got, want), (n, w, off)
                assert np.all(host(buf)[:off] == np.uint64(2**64 - 1))
    for off in (0, 1):
        bufs = [torch.full((F.dnf_words(n) + 2,), -1, dtype=torch.int64, device="cuda") for _, n in texts]
        b = F.Batch(progs, words_per_lane=32)
        b.set_dnf_outputs([o[off:] for o in bufs])
        counts = host(b.eval_dnf())
        for (t, n), o, c in zip(texts, bufs, counts):
            want = oracle.dnf(t, n)
            got = host(o)
            assert np.array_equal(got[off:off + len(want)], want), (n, off)
            assert np.all(got[:off] == np.uint64(2**64 - 1)) and np.all(got[off + len(want):] == np.uint64(2**64 - 1))
            assert int(c) == int(np.unpackbits(want.view(np.uint8)).sum())
        b.free()


def test_batch_eval_dnf_argument_errors(F):
    import torch
    p = F.Program("x3 | x9", 12)
    b = F.Batch([p])
    with pytest.raises(F.FbgError) as ei:
        b.eval_dnf()                               # no outputs set
    assert ei.value.status == F.FBG_E_INVAL
    with pytest.raises(F.FbgError) as ei:
        b.set_dnf_outputs([torch.empty(10, dtype=torch.int64, device="cuda")])
    assert ei.value.status == F.FBG_E_INVAL
    with pytest.raises(ValueError):
        b.set_dnf_outputs([])
    b.free()


@pytest.mark.parametrize("k", [3, 5, 9, 17])
def test_registers_beyond_the_vgpr_set(F, k):
    rng = random.Random(4400 + k)
    for n in (12, 19):
        text = many_registers(rng, n, k)
        p = full_check(F, text, n, wpls=[1, 2, 4, 8, 16])
        assert p.info["n_regs"] >= min(k, 5) - 1
        # and inside a batch next to clause-only programs (two plans)
        cnf = workloads.random_3cnf(n, 40, k)
        progs = [p, F.Program(*cnf)]
        want = [oracle.count(text, n), oracle.count(*cnf)]
        assert host(F.count_batch(progs)).tolist() == want


@pytest.mark.parametrize("k", [9, 17])
def test_batch_registers_in_global_scratch(F, k):
    # at 16 words per lane a batch keeps two registers of a wave in LDS and
    # the rest in a global scratch block: programs with many registers, next
    # to clause-only ones and small ones, in one launch, vs the oracle
    rng = random.Random(5100 + k)
    texts = [(many_registers(rng, n, k), n) for n in (12, 17, 19)]
    texts += [workloads.random_3cnf(19, 40, k), ("x0 & ~x3 | x5", 8)]
    progs = [F.Program(t, n) for t, n in texts]
    assert max(p.info["n_regs"] for p in progs) >= 6
    want = [oracle.count(t, n) for t, n in texts]
    b = F.Batch(progs, words_per_lane=16)
    assert host(b.count()).tolist() == want
    assert host(b.count(graph=True)).tolist() == want
    b.free()


def test_jump_table_copy_for_any_load_address(F, monkeypatch):
    """The interpreter at 16 words per lane keeps a second copy of its jump
    table for code loaded off a 64 KiB boundary; FBG_J16_TABLE=any makes every
    launch use it.  Its results are the oracle's: random DAGs (every case of
    the table), registers in LDS and in global scratch, alone and batched."""
    import torch
    monkeypatch.setenv("FBG_J16_TABLE", "any")
    rng = random.Random(6100)
    texts = [workloads.random_dag(n, rng.randrange(300, 2000), 61 + n) for n in (12, 16, 19)]
    texts += [(many_registers(rng, n, 17), n) for n in (12, 17)]
    for text, n in texts:
        full_check(F, text, n, wpls=[16])
    progs = [F.Program(t, n) for t, n in texts]
    want = [oracle.count(t, n) for t, n in texts]
    b = F.Batch(progs, words_per_lane=16)
    assert host(b.count()).tolist() == want
    assert host(b.count(graph=True)).tolist() == want
    b.free()
    monkeypatch.delenv("FBG_J16_TABLE")
    # and back on the aligned copy
    assert host(F.count_batch(progs, words_per_lane=16)).tolist() == want
    torch.cuda.synchronize()


def test_batch_enumerate_lists_every_program(F):
    import torch
    rng = random.Random(91)
    texts = [("x0", 1), ("0", 9), ("x1 | ~x1", 4)]
    texts += [workloads.random_3cnf(rng.choice([16, 19, 22]), 60, s) for s in range(5)]
    texts += [workloads.random_dag(rng.choice([12, 17]), rng.randrange(50, 300), s) for s in range(3)]
    texts += [workloads.triangle_free(6), workloads.baequ4()]
    progs = [F.Program(t, n) for t, n in texts]
    wants = [oracle.models(t, n) for t, n in texts]
    caps = [w[1] + 2 if i % 3 == 0 else (max(0, w[1] // 2) if i % 3 == 1 else 0) for i, w in enumerate(wants)]
    for wpl in (0, 2, 16):
        b = F.Batch(progs, words_per_lane=wpl)
        dnfs = [torch.empty(F.dnf_words(n), dtype=torch.int64, device="cuda") for _, n in texts]
        b.set_dnf_outputs(dnfs)
        outs = [torch.full((c,), -1, dtype=torch.int64, device="cuda") if c else None for c in caps]
        b.set_enum_outputs(outs)
        for rep in range(2):
            counts = host(b.eval_dnf())
            b.enumerate()
            for (m, total), c, o, got_c in zip(wants, caps, outs, counts):
                assert int(got_c) == total
                if c:
                    got = host(o)
                    k = min(c, total)
                    assert np.array_equal(got[:k], m[:k]), (wpl, rep)
                    assert np.all(got[k:] == np.uint64(2**64 - 1))
        b.free()


def test_batch_dnf_with_tile_counts(F):
    """Once the tile counts exist (enumeration outputs set), the DNF write-out
    of clause-only programs without the cofactor runs one wave per tile and
    takes its counts from the tile counts: vectors and counts still equal the
    oracle's, at every tiling, next to general programs, on repeated calls;
    the cofactor and an explicit grid keep the queued launch."""
    import torch
    texts = [("x0", 1), ("0", 9), ("x3 & ~x11", 14)]
    texts += [workloads.random_3cnf(n, 4 * n, s) for s, n in enumerate((12, 17, 21, 23))]
    texts += [workloads.random_dag(n, 200, s) for s, n in enumerate((13, 18))]
    texts.append(workloads.triangle_free(6))
    progs = [F.Program(t, n) for t, n in texts]
    wants = [oracle.dnf(t, n) for t, n in texts]
    for wpl, grid, cof in ((0, 0, False), (1, 0, False), (4, 0, False), (16, 0, False), (32, 0, False),
                           (32, 0, True), (8, 64, False)):
        b = F.Batch(progs, words_per_lane=wpl, grid_blocks=grid, cofactor=cof)
        dnfs = [torch.full((F.dnf_words(n) + 1,), -1, dtype=torch.int64, device="cuda") for _, n in texts]
        b.set_dnf_outputs(dnfs)
        b.set_enum_outputs([None] * len(progs))
        for rep in range(2):
            for o in dnfs:
                o.fill_(-1)
            counts = host(b.eval_dnf())
            for (t, n), w, o, c in zip(texts, wants, dnfs, counts):
                got = host(o)
                assert np.array_equal(got[:len(w)], w), (wpl, grid, cof, n, rep)
                assert got[len(w)] == np.uint64(2**64 - 1)
                assert int(c) == int(np.unpackbits(w.view(np.uint8)).sum()), (wpl, grid, cof, n, rep)
        b.free()


@pytest.mark.parametrize("run", [0, 1, 4])
def test_batch_dnf_xcd_local_layout(F, run):
    """Programs of clauses alone with n >= 21 are written out by the batched
    write-out in the XCD-local layout (an encoding with variables 15..17 and
    18..20 exchanged; piece counts summed into tile counts): DNF vectors,
    counts and the batched enumeration equal the oracle, next to smaller
    programs in the same plan (whose tiles pad the XCD-aligned starts), at the
    default one tile per wave and at explicit runs of tiles."""
    import torch
    texts = [workloads.random_3cnf(12, 51, 1), workloads.random_3cnf(21, 89, 2), ("x3 & ~x11", 14),
             workloads.random_3cnf(22, 94, 3), workloads.random_3cnf(19, 81, 4), ("~x20 | x16 & x17", 21),
             workloads.random_3cnf(24, 102, 5), ("x15 & x18 & ~x19", 22)]
    progs = [F.Program(t, n) for t, n in texts]
    wants = [oracle.dnf(t, n) for t, n in texts]
    cap = 3000
    models = [oracle.models(t, n, cap=cap) for t, n in texts]   # (first cap models, total)
    b = F.Batch(progs, words_per_lane=32, direct_run=run)
    dnfs = [torch.full((F.dnf_words(n) + 1,), -1, dtype=torch.int64, device="cuda") for _, n in texts]
    idx = [torch.full((cap,), -1, dtype=torch.int64, device="cuda") for _ in texts]
    b.set_dnf_outputs(dnfs)
    b.set_enum_outputs(idx)
    for rep in range(2):
        for o in dnfs:
            o.fill_(-1)
        print("xcd layout: run %d, repeat %d" % (run, rep), flush=True)
        counts = host(b.eval_dnf())
        b.enumerate()
        for (t, n), w, (m, total), o, ii, c in zip(texts, wants, models, dnfs, idx, counts):
            got = host(o)
            assert np.array_equal(got[:len(w)], w), (run, n, rep)
            assert got[len(w)] == np.uint64(2**64 - 1)
            assert int(c) == total, (run, n, rep)
            assert np.array_equal(host(ii)[:len(m)], m), (run, n, rep)
    b.free()


@pytest.mark.parametrize("grid", [0, 96])
def test_single_dnf_xcd_local_layout(F, grid):
    """fbg_eval_dnf of a program of clauses alone with n >= 21 at 32 words
    per lane writes through the XCD-local encoding: the vector equals the
    oracle's, on the default grid of one tile per wave and on an explicit
    smaller grid whose waves stride over the tiles; the word after the
    vector is untouched."""
    import torch
    for t, n in (workloads.random_3cnf(21, 89, 7), ("x15 & ~x18 | x20", 22), workloads.random_3cnf(23, 98, 8),
                 ("~x16 & (x19 | x2)", 21)):
        p = F.Program(t, n)
        out = torch.full((F.dnf_words(n) + 1,), -1, dtype=torch.int64, device="cuda")
        print("single xcd: n %d grid %d" % (n, grid), flush=True)
        F.eval_dnf(p, out=out, words_per_lane=32, grid_blocks=grid)
        got = host(out)
        want = oracle.dnf(t, n)
        assert np.array_equal(got[:len(want)], want), (n, grid)
        assert got[len(want)] == np.uint64(2**64 - 1)
        p.free()


@pytest.mark.parametrize("skip", [1, 2])
def test_batch_dnf_xcd_local_layout_unaligned_outputs(F, skip):
    """The write-out into output views that start 8 bytes (plain layout: the
    XCD-local one stores 16-byte groups) or 16 bytes (XCD-local layout) past a
    32 KiB boundary, with guard words on both sides left untouched."""
    import torch
    texts = [workloads.random_3cnf(21, 89, 11), workloads.random_3cnf(22, 94, 12), workloads.random_3cnf(13, 55, 13)]
    progs = [F.Program(t, n) for t, n in texts]
    wants = [oracle.dnf(t, n) for t, n in texts]
    bufs = [torch.full((F.dnf_words(n) + 2 * skip,), -1, dtype=torch.int64, device="cuda") for _, n in texts]
    views = [b[skip:skip + F.dnf_words(n)] for b, (_, n) in zip(bufs, texts)]
    b = F.Batch(progs, words_per_lane=32)
    b.set_dnf_outputs(views)
    b.set_enum_outputs([None] * len(progs))
    print("xcd layout: outputs %d words past a boundary" % skip, flush=True)
    counts = host(b.eval_dnf())
    for w, buf, c in zip(wants, bufs, counts):
        got = host(buf)
        assert (got[:skip] == np.uint64(2**64 - 1)).all() and (got[skip + len(w):] == np.uint64(2**64 - 1)).all()
        assert np.array_equal(got[skip:skip + len(w)], w)
        assert int(c) == int(np.unpackbits(w.view(np.uint8)).sum())
    for (t, n), w in zip(texts, wants):
        out = torch.full((F.dnf_words(n) + 2 * skip,), -1, dtype=torch.int64, device="cuda")
        F.eval_dnf(F.Program(t, n), out=out[skip:skip + F.dnf_words(n)], words_per_lane=32)
        got = host(out)
        assert (got[:skip] == np.uint64(2**64 - 1)).all() and (got[skip + len(w):] == np.uint64(2**64 - 1)).all()
        assert np.array_equal(got[skip:skip + len(w)], w)
    b.free()


def test_batch_enumerate_needs_outputs(F):
    import torch
    p = F.Program("x1 & x5", 9)
    b = F.Batch([p])
    with pytest.raises(F.FbgError):
        b.enumerate()
    with pytest.raises(F.FbgError):      # DNF outputs first
        b.set_enum_outputs([torch.empty(4, dtype=torch.int64, device="cuda")])
    b.free()


def test_c1_batched_step_at_full_size(F):
    """The benchmark step itself (16 instances, n = 32, one batched DNF launch
    and one batched enumeration, default tiling): counts and model lists
    against the oracle goldens, and sampled DNF words of every instance
    against the oracle one valuation at a time."""
    import torch
    g = golden("c1_3cnf_n32.json")["seeds"]
    seeds = list(range(16))
    if not all(str(s) in g for s in seeds):
        pytest.skip("c1 golden incomplete")
    texts = [workloads.random_3cnf(32, 136, s) for s in seeds]
    progs = [F.Program(t, n) for t, n in texts]
    b = F.Batch(progs)
    dnfs = [torch.empty(1 << 26, dtype=torch.int64, device="cuda") for _ in seeds]
    idx = [torch.full((4096,), -1, dtype=torch.int64, device="cuda") for _ in seeds]
    b.set_dnf_outputs(dnfs)
    b.set_enum_outputs(idx)
    counts = host(b.eval_dnf())
    b.enumerate()
    rng = np.random.default_rng(5)
    for s, (text, n), d, ii, c in zip(seeds, texts, dnfs, idx, counts):
        rec = g[str(s)]
        assert int(c) == rec["count"], s
        assert host(ii)[:rec["count"]].tolist() == rec["models"], s
        words = np.sort(rng.choice(1 << 26, 64, replace=False))
        sample = d[torch.from_numpy(words.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
        vals = (words[:, None].astype(np.uint64) * 64 + np.arange(64, dtype=np.uint64)[None, :]).ravel()
        bits = oracle.eval_at(text, n, vals).reshape(-1, 64)
        want = (bits.astype(np.uint64) << np.arange(64, dtype=np.uint64)[None, :]).sum(axis=1).astype(np.uint64)
        assert np.array_equal(sample, want), s
    b.free()
    del dnfs


def test_batch_autotuner_choice_is_exact(F, tmp_path):
    from paper_1310_6978_amd import autotune
    rng = random.Random(17)
    texts = [workloads.random_dag(rng.choice([12, 16, 20]), rng.randrange(50, 400), i) for i in range(20)]
    texts += [workloads.random_3cnf(21, 89, s) for s in range(4)]
    progs = [F.Program(t, n) for t, n in texts]
    t = autotune.Tuner(path=str(tmp_path / "tune.json"), reps=1)
    w = t.tune_batch(progs, candidates=(0, 4, 16))
    assert w in (0, 4, 16) and set(t.table[t.last_key]["ms"]) <= {0, 4, 16}
    assert autotune.Tuner(path=str(tmp_path / "tune.json")).tune_batch(progs) == w   # cached
    want = [oracle.count(tx, n) for tx, n in texts]
    assert host(F.count_batch(progs, words_per_lane=w)).tolist() == want


@pytest.mark.parametrize("n", [36, 40])
def test_large_counts_per_wave(F, n):
    # waves that count more than 2^31 models each: the 64-bit wave sums must
    # carry exactly (7/8 of 2^n models, single-program and batched paths)
    p = F.Program("x0 | x1 | x2", n)
    want = 7 << (n - 3)
    for w in (1, 8, 32):
        assert int(host(F.count(p, words_per_lane=w))[0]) == want
    q = F.Program("x5 | ~x39" if n == 40 else "x5 | ~x35", n)
    assert host(F.count_batch([p, q])).tolist() == [want, 3 << (n - 2)]


def test_maximum_sizes(F):
    # n = 48, the largest valuation space (2^48 valuations, two clauses)
    n = 48
    p = F.Program("x0 & ~x47", n)
    assert gpu_count(F, p) == 1 << 46
    none = F.Program("x5 & 0 | 0 & x47", n)                            # folds to 0
    assert gpu_count(F, none) == 0 and none.info["const_value"] == 0
    assert host(F.count_batch([p, none])).tolist() == [1 << 46, 0]
    assert p.info["code_bytes"] >= 4096
    # n = 40: a single model at the last index, found by the enumeration
    full = F.Program(" & ".join("x%d" % k for k in range(40)), 40)
    assert gpu_count(F, full) == 1
    m, t = gpu_models(F, full, 4)
    assert t == 1 and int(m[0]) == (1 << 40) - 1


def test_dnf_at_36_variables(F):
    # an 8 GiB DNF vector: sampled words against the oracle, total = count
    import torch
    text, n = workloads.equivalence_relations(9)
    p = F.Program(text, n)
    d = F.eval_dnf(p)
    assert d.numel() == 1 << 30
    rng = np.random.default_rng(3)
    words = np.sort(rng.choice(1 << 30, 128, replace=False))
    sample = d[torch.from_numpy(words.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
    vals = (words[:, None].astype(np.uint64) * 64 + np.arange(64, dtype=np.uint64)[None, :]).ravel()
    bits = oracle.eval_at(text, n, vals).reshape(-1, 64)
    want = (bits.astype(np.uint64) << np.arange(64, dtype=np.uint64)[None, :]).sum(axis=1).astype(np.uint64)
    assert np.array_equal(sample, want)
    idx, tot = F.enumerate_dnf(d, n, 30000)
    assert int(host(tot)[0]) == 21147
    g = golden("c2_theories.json").get("equivalence_k9")
    if g:
        assert host(idx)[:21147].tolist() == g["models"]
    del d
