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
    for w in wpl:
        got, c = p.emulate(w)
        assert np.array_equal(got, want), (w, text[:200])
        assert c == want_count
    assert_clause_prefix(p)
    return p


def assert_clause_prefix(p):
    """The kernels run the CL instructions as a prefix loop: no CL may follow
    another instruction, and the prefix length is n_clause_instr."""
    ops = [line.split()[1] for line in p.disasm(1).splitlines()[1:]]
    k = 0
    while k < len(ops) and ops[k] == "CL":
        k += 1
    assert "CL" not in ops[k:], ops
    assert k == p.info["n_clause_instr"]


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


def test_tile_only_clauses_lead_the_prefix():
    """At every tiling the clauses made only of tile variables come first (the
    uniform-cofactor kernel can then drop a dead tile early); the emulated
    result is unchanged."""
    text, n = workloads.random_3cnf(32, 136, 4)
    p = fbg.Program(text, n)
    for w in WPL:
        rows = p.disasm(w).splitlines()[1:]
        kinds = []
        for r in rows:
            f = dict(x.split("=") for x in r.split()[2:] if "=" in x)
            kinds.append(int(f["mconst"], 16) == 0 and int(f["lane"], 16) == 0 and int(f["pat"], 16) == 0)
        k = kinds.index(False) if False in kinds else len(kinds)
        assert k > 0 and not any(kinds[k:]), w
    check("(x0|x1) & (x22|~x23) & (x2|x12) & ~x21 & (x18|x20)", 24, wpl=[1, 32])


@pytest.mark.parametrize("k", [3, 5, 9, 17])
def test_registers_beyond_the_vgpr_set(k):
    # registers 0..3 live in VGPRs, the rest in LDS: programs on both sides
    rng = random.Random(4400 + k)
    text = many_registers(rng, 14, k)
    p = check(text, 14, wpl=[1, 4, 8])
    assert p.info["n_regs"] >= min(k, 5) - 1
