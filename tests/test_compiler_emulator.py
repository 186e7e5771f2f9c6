"""The compiler and the device-program encoding, checked on the CPU: the
library's host interpretation of the encoded program (fbg_program_emulate,
slice by slice exactly as the kernels read it) must reproduce the oracle's
DNF vector bit for bit, for every words-per-lane setting, so that every
class of index bit (in-word, lane, word-in-lane, tile) is exercised."""

import random

import numpy as np
import pytest

import oracle
import workloads
from paper_1310_6978_amd import fbg
from tests.formula_gen import many_registers, random_cnf, random_program

WPL = [1, 2, 4, 8, 16, 32]


def check(text, n, wpl=WPL):
    want = oracle.dnf(text, n)
    want_count = int(sum(bin(int(w)).count("1") for w in want))
    p = fbg.Program(text, n)
    for cof in (False, True):
        for w in wpl:
            p.set_tuning(w, cofactor=cof)
            got, c = p.emulate(w)
            assert np.array_equal(got, want), (w, cof, text[:200])
            assert c == want_count
    p.set_tuning(0)
    for w in wpl:
        assert_clause_block(p, w)
    return p


MERGED = ("XYS", "LIS", "ORS", "ACM")   # jump-table instructions that hold a store or an ACC as well


def instructions(listing):
    """(pc, opcode) of the instruction lines of a listing."""
    out = []
    for line in listing.splitlines():
        f = line.split()
        if f and f[0].isdigit():
            out.append((int(f[0]), f[1]))
    return out


def assert_clause_block(p, w):
    """The leading clauses form the clause block: no clause is left in the
    instruction stream, and the block holds at most n_clause_instr clauses
    (always-true ones are dropped), each chunk at most 32."""
    lst = p.disasm(w)
    assert all(op != "CL" for _, op in instructions(lst))
    head = [l for l in lst.splitlines() if l.startswith("; clause block:")][0]
    ncl = int(head.split()[3])
    assert ncl <= p.info["n_clause_instr"]
    chunks = [int(l.split()[3].split("=")[1]) for l in lst.splitlines() if l.startswith("chunk ")]
    assert sum(chunks) == ncl and all(1 <= c <= 32 for c in chunks)
    # a merged store (XYS, LIS, ORS at 16 words per lane) is two instructions
    ops = [op for _, op in instructions(lst)]
    assert p.info["n_instr"] == p.info["n_clause_instr"] + len(ops) + sum(op in MERGED for op in ops)


@pytest.mark.parametrize("seed", range(60))
def test_random_formulas(seed):
    rng = random.Random(1000 + seed)
    n = rng.choice([0, 1, 3, 5, 6, 7, 11, 12, 13, 14, 15, 16, 17])
    if n == 0:
        stmts, text = random_program(rng, 1)
        text = text.replace("x0", "1")
    else:
        stmts, text = random_program(rng, n)
    check(text, n)


@pytest.mark.parametrize("seed", range(20))
def test_random_cnf_all_classes(seed):
    rng = random.Random(2000 + seed)
    n = rng.choice([12, 14, 16, 18])
    check(random_cnf(rng, n, rng.randrange(1, 40)), n)


@pytest.mark.parametrize("seed", range(12))
def test_random_dags(seed):
    rng = random.Random(3000 + seed)
    n = rng.choice([6, 10, 12, 14, 16])
    text, n = workloads.random_dag(n, rng.randrange(20, 400), seed)
    check(text, n)


def test_wide_xor_and_and_sets():
    n = 16
    check(" ^ ".join("x%d" % k for k in range(n)), n)
    check("~(" + " ^ ".join("x%d" % k for k in range(0, n, 3)) + ")", n)
    check(" & ".join("x%d" % k for k in range(4, n)), n)
    check("~(" + " & ".join("~x%d" % k for k in range(n)) + ")", n)
    # x and ~x of every class in one clause: a tautology clause
    for k in (0, 7, 11, 15):
        check("x%d | ~x%d | x3" % (k, k), n)
        check("x%d ^ ~x%d ^ x3" % (k, k), n)
        check("(x%d & ~x%d) | x3 & x12" % (k, k), n)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_equivalence(k):
    check(*workloads.equivalence_relations(k))


@pytest.mark.parametrize("k", [3, 4])
def test_permutations(k):
    check(*workloads.permutation_matrices(k))


@pytest.mark.parametrize("k", [4, 5, 6])
def test_triangle_free(k):
    check(*workloads.triangle_free(k))


@pytest.mark.parametrize("m", [2, 3, 4])
def test_special_element_posets(m):
    check(*workloads.special_element_posets(m))


@pytest.mark.parametrize("m", [4, 5, 6])
def test_bounded_posets(m):
    check(*workloads.bounded_posets(m))


def test_baequ4():
    p = check(*workloads.baequ4())
    assert p.info["l2in"] > 0


def test_constants_and_info():
    for n in (0, 3, 9, 17):
        p = check("1", n)
        assert p.info["const_value"] == 1
        p = check("0", n)
        assert p.info["const_value"] == 0
        p = check("x0 & ~x0 | 0", max(n, 1))
        assert p.info["const_value"] == 0


def test_l2in_counts_cnf_ops():
    # a 3-literal clause is 2 ORs, and the conjunction of m clauses m-1 ANDs
    text, n = workloads.random_3cnf(20, 30, 1)
    p = fbg.Program(text, n)
    assert p.info["l2in"] == 3 * 30 - 1
    assert p.info["n_clause_instr"] == 30
    assert p.info["n_regs"] == 0


def test_shared_subterms_use_registers():
    text = "t = (x1 ^ x12) & (x3 | x14)\nu = t ^ x5\n(t | x7) & (u ^ x13)\n"
    p = check(text, 16)
    assert p.info["n_regs"] >= 1


@pytest.mark.parametrize("bad,status", [
    ("x0 &", fbg.FBG_E_PARSE), ("x0 & (x1", fbg.FBG_E_PARSE), ("2", fbg.FBG_E_PARSE),
    ("y0", fbg.FBG_E_PARSE), ("t = x0\nt = x1\nt", fbg.FBG_E_PARSE), ("x0 = x1", fbg.FBG_E_PARSE),
    ("", fbg.FBG_E_PARSE), ("x3", fbg.FBG_E_RANGE), ("x0 $ x1", fbg.FBG_E_PARSE)])
def test_errors(bad, status):
    with pytest.raises(fbg.FbgError) as ei:
        fbg.Program(bad, 3)
    assert ei.value.status == status


def test_parse_error_offset():
    with pytest.raises(fbg.FbgError) as ei:
        fbg.Program("x0 & x1\nx1 | | x2\n", 3)
    assert ei.value.offset == 13


def test_n_range():
    with pytest.raises(fbg.FbgError) as ei:
        fbg.Program("x0", 49)
    assert ei.value.status == fbg.FBG_E_RANGE
    with pytest.raises(fbg.FbgError):
        fbg.Program("x0", -1)


def test_deep_nesting_compiles():
    n = 12
    text = "x0"
    for i in range(3000):
        text = "(%s %s x%d)" % (text, "&|^"[i % 3], (i * 7) % n)
    check(text, n, wpl=[1, 16])


def test_deep_text_compiles_from_several_threads():
    """The compiler recurses on a large stack of its own per calling thread:
    deep text from several Python threads at once, each result as on the
    main thread, and later compiles on the same threads still work."""
    import threading
    n = 9
    texts = ["(" * 20000 + "x%d | ~x%d" % (k, k + 1) + ")" * 20000 for k in range(4)]
    texts += [" ^ ".join("x%d" % ((i * 5 + k) % n) for i in range(30000)) for k in range(4)]
    want = [fbg.Program(t, n).emulate(4)[1] for t in texts]
    got = [None] * len(texts)
    errors = []

    def work(k):
        try:
            for _ in range(2):
                got[k] = fbg.Program(texts[k], n).emulate(4)[1]
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(texts))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors and got == want


def test_set_tuning_changes_the_default():
    p = fbg.Program(*workloads.random_3cnf(20, 85, 0))
    for w in (1, 4, 32):
        p.set_tuning(w)
        assert p.info["words_per_lane"] == w
    with pytest.raises(fbg.FbgError) as ei:
        p.set_tuning(3)
    assert ei.value.status == fbg.FBG_E_INVAL


def test_autotune_cache_keys(tmp_path):
    from paper_1310_6978_amd import autotune
    p = fbg.Program(*workloads.random_3cnf(20, 85, 0))
    k = autotune.key_of(p)
    assert "n=20" in k and "gen=0" in k
    t = autotune.Tuner(path=str(tmp_path / "t.json"))
    t.table[k] = {"words_per_lane": 8}
    assert t.apply(p, save=False) == 8          # a cached choice needs no device
    assert p.info["words_per_lane"] == 8
    t.save()
    assert autotune.Tuner(path=str(tmp_path / "t.json")).table[k]["words_per_lane"] == 8


def test_tile_only_clauses_fill_the_cofactor_table():
    """At every tiling the uniform-cofactor table at the end of the clause
    block lists every clause made only of tile variables, once (the
    uniform-cofactor kernels drop a tile on which one of them is false before
    any other work), and the emulated cofactor reading equals the oracle."""
    text, n = workloads.random_3cnf(32, 136, 4)
    clauses = set()
    for part in text.splitlines():
        lits = frozenset(tok.strip() for tok in part.split("|"))
        clauses.add(lits)
    p = fbg.Program(text, n)
    for w in WPL:
        tile_bit = 11 + w.bit_length() - 1
        want = sum(all(int(l.lstrip("~")[1:]) >= tile_bit for l in c) for c in clauses)
        first = [l for l in p.disasm(w).splitlines() if l.startswith("chunk 0 ")][0]
        k = int(first.split("cofactor=")[1].split()[0])
        assert k == want > 32 if w == 1 else k == want, (w, want, k)
    check("(x0|x1) & (x22|~x23) & (x2|x12) & ~x21 & (x18|x20)", 24, wpl=[1, 32])
    # more tile-only clauses than one chunk holds (40 on variables 11..19),
    # read by the emulated uniform-cofactor kernels
    rng = random.Random(5)
    parts = set()
    while len(parts) < 40:
        vs = sorted(rng.sample(range(11, 20), 2))
        parts.add(" | ".join(("~x%d" if rng.random() < 0.5 else "x%d") % v for v in vs))
    parts = sorted(parts) + ["x0 | ~x12 | x3", "~x5 | x15", "x9 | x10"]
    text = " & ".join("(%s)" % c for c in parts)
    p = fbg.Program(text, 20)
    assert int([l for l in p.disasm(1).splitlines() if l.startswith("chunk 0 ")][0]
               .split("cofactor=")[1].split()[0]) == 40
    want = oracle.count(text, 20)
    for w in (1, 2, 8):
        p.set_tuning(w, cofactor=True)
        dnf, cnt = p.emulate(w)
        assert cnt == want, (w, cnt, want)
        assert np.array_equal(dnf, oracle.dnf(text, 20)), w


def test_clause_groups_by_word_literals():
    """Keys of the static chunks fall in groups 0 .. 2 log2 W by their word
    literals; clauses with two word literals go to multi chunks."""
    # W = 4: word bits are x11 (j = 0) and x12 (j = 1)
    text = "(x0 | x1) & (x11 | x2) & (~x11 | x3) & (x12 | x5) & (~x12 | x6) & (x11 | x12 | x7) & (x40 | ~x41)"
    p = fbg.Program(text, 42)
    lst = p.disasm(4)
    groups = sorted(int(l.split("group=")[1].split()[0]) for l in lst.splitlines() if "key group=" in l)
    assert groups == [0, 0, 1, 2, 3, 4]
    assert sum(1 for l in lst.splitlines() if "key multi" in l) == 1
    small = text.replace("x40", "x9").replace("x41", "x10")
    check(small, 14, wpl=[1, 2, 4, 8])


@pytest.mark.parametrize("seed", range(6))
def test_multi_keys_inside_and_after_the_tree(seed):
    """Clauses with two or more word-index literals (x11..x15 at 32 words per
    lane): the first 32 act inside the product tree at their level and half,
    the rest after it on the words.  Every level, half and pattern shape."""
    rng = random.Random(4700 + seed)
    n = 17
    clauses = []
    for _ in range(rng.choice([12, 40, 75])):
        k = rng.choice([2, 3, 3, 4])
        vs = rng.sample(range(11, 16), min(k, 5) - 1) + [rng.randrange(n)]
        clauses.append("(" + " | ".join(("~" if rng.random() < 0.5 else "") + "x%d" % v for v in vs) + ")")
    # a few static clauses as well
    for _ in range(10):
        vs = rng.sample(range(n), 3)
        clauses.append("(" + " | ".join(("~" if rng.random() < 0.5 else "") + "x%d" % v for v in vs) + ")")
    p = check(" & ".join(clauses), n, wpl=[4, 8, 16, 32])
    lst = p.disasm(32)
    assert "multi-tree" in lst


@pytest.mark.parametrize("k", [3, 5, 9, 17])
def test_registers_beyond_the_vgpr_set(k):
    # registers 0..3 live in VGPRs, the rest in LDS: programs on both sides
    rng = random.Random(4400 + k)
    text = many_registers(rng, 14, k)
    p = check(text, 14, wpl=[1, 4, 8])
    assert p.info["n_regs"] >= min(k, 5) - 1


@pytest.mark.parametrize("seed", range(8))
def test_chains_of_literal_sets(seed):
    """At 16 words per lane, two or more literal sets in a row without
    word-index literals (x11..x14) run as a chain: XYF, XYM ..., XYL, and the
    emulated chain (X and Y per lane, then one pass over the words) equals
    the oracle.  Runs of every length from 1 to 6, OR- and XOR-sets, with lane,
    in-word and tile literals (x15..)."""
    rng = random.Random(5100 + seed)
    n = 19
    pool = [v for v in range(n) if not 11 <= v <= 14]
    parts = []
    for _ in range(4):
        e = "x%d" % rng.choice(pool)
        for _ in range(rng.randrange(1, 7)):
            lit = ("~" if rng.random() < 0.3 else "") + "x%d" % rng.choice(pool)
            e = "(%s %s %s)" % (e, rng.choice("&|^"), lit)
        parts.append(e)
    text = "(%s ^ %s) | (%s & ~%s)" % tuple(parts)
    p = check(text, n, wpl=[16, 1, 32])
    ops = [op for _, op in instructions(p.disasm(16))]
    # every chain opens with XYF, continues with XYM and closes with XYL (or
    # XYS, its result stored into a register)
    i = 0
    while i < len(ops):
        if ops[i] == "XYF":
            j = i + 1
            while ops[j] == "XYM":
                j += 1
            assert ops[j] in ("XYL", "XYS"), ops
            i = j + 1
        else:
            assert ops[i] not in ("XYM", "XYL", "XYS"), ops
            i += 1
    assert "XYF" not in [op for _, op in instructions(p.disasm(8))]
    # the plain form and the jump-table form hold the same instructions (a
    # merged store counts twice)
    assert len(ops) + sum(op in MERGED for op in ops) == len(instructions(p.disasm(8)))


def test_merged_stores():
    """At 16 words per lane a store into a VGPR register after which cur is
    dead merges into the instruction before it: the last set of a chain
    (XYS), a literal set (LIS) or an operation on the same register (ORS).  Where cur is still
    read after the store (here by ACC), the store stays.  The emulator runs
    the merged forms as the kernel does (cur left stale), so a merge where cur
    is live would show as a wrong vector."""
    # (a ^ b) & (c | d) with chained literal sets on both sides
    text = "t1 = ((x0 ^ x6) & x7 | x16) ^ x2\nt2 = ((x1 | x9) ^ x17) & x4\nt1 & t2 | (t1 ^ x3) & ~t2"
    p = check(text, 18, wpl=[16, 8])
    ops = [op for _, op in instructions(p.disasm(16))]
    assert any(op in MERGED for op in ops), ops
    rng = random.Random(5300)
    for _ in range(12):
        t = many_registers(rng, 17, rng.choice([3, 5, 8]))
        check(t, 17, wpl=[16])


@pytest.mark.parametrize("text", ["t = x0 ^ x7 | x16\nt & (t | x3 & x9) & (t ^ x17)",
                                  "t = (x0 ^ x7) & x16\nu = t | x4\nt & u & (u ^ x2)",
                                  "t = x1 & ~x12\nu = t ^ x5\n(u | x17) & ~(t & x3) & (u | t)"])
def test_merged_acc(text):
    """An ACC after which cur is dead merges into the register operation or
    literal set before it (ACM: acc = f(acc, cur, operand), ACC's inversion
    folded in); where cur is read after the ACC, or the instruction before
    it is a store, the ACC stays.  Emulated with cur left stale."""
    p = check(text, 18, wpl=[16, 8, 32])
    ops = [op for _, op in instructions(p.disasm(16))]
    assert "ACM" in ops, ops


def test_run_of_four_literal_sets_is_one_chain():
    """Four literal sets in a row (lane, in-word and tile literals) become
    XYF, XYM, XYM, XYL; the clause x9 stays in the clause block."""
    text = "((((x0 ^ x6) & x7) | x16) ^ x2) & x9"
    p = fbg.Program(text, 18)
    assert [op for _, op in instructions(p.disasm(16))][:4] == ["XYF", "XYM", "XYM", "XYL"]
    check(text, 18, wpl=[16])
