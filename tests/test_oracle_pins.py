"""Pins for the CPU oracle: it is checked against facts the paper and the
mathematics fix, never against itself or the GPU path.

* the paper's worked example of the free generators for n = 3 (Section 2.2);
* the minterm property of free generators (each full conjunction of
  literals has exactly one model, Section 2.2) and Proposition 2.2 through an
  independent route: Python's own parser and big-integer bitwise arithmetic
  on the rows of M;
* closed forms: 2^n, 1, 2^n - 1, 2^(n-1), Bell numbers, k!, and brute force
  over structures (set partitions, permutations, graphs, relations) written
  here from their definitions;
* the worked system BAequ4 of Section 5.1 (solutions derived by hand in the
  fixture).
"""

import os
import random
import re
from itertools import combinations, permutations, product

import numpy as np
import pytest

import oracle
import workloads
from workloads.formulas import equivalence_var

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def models_of(src, n):
    m, total = oracle.models(src, n)
    assert len(m) == total
    return [int(v) for v in m]


def rows_of_M(n):
    """Rows of the matrix M of Section 2.2 as Python integers: bit i of row k
    (variable xk) is bit k of the column index i."""
    rows = []
    for k in range(n):
        r = 0
        for i in range(1 << n):
            if (i >> k) & 1:
                r |= 1 << i
        rows.append(r)
    return rows


def python_dnf(stmts, n):
    """Proposition 2.2 evaluated by Python itself: the statements are executed
    with the variables bound to the rows of M as big integers; the result is
    the AND of the assertions masked to 2^n bits."""
    full = (1 << (1 << n)) - 1
    env = {"x%d" % k: r for k, r in enumerate(rows_of_M(n))}
    env["ONE"] = full
    env["ZERO"] = 0
    acc = full
    for kind, name, text in stmts:
        py = re.sub(r"\b1\b", "ONE", re.sub(r"\b0\b", "ZERO", text))
        val = eval(py, {}, env) & full
        if kind == "def":
            env[name] = val
        else:
            acc &= val
    return acc & full


def words_to_int(words):
    v = 0
    for i, w in enumerate(words):
        v |= int(w) << (64 * i)
    return v


def random_expr(rng, n, names, depth):
    """Random expression text over ~ & ^ |, sometimes without parentheses so
    that precedence decides."""
    if depth == 0 or rng.random() < 0.25:
        r = rng.random()
        if r < 0.06:
            return rng.choice(["0", "1"])
        if names and r < 0.3:
            return rng.choice(names)
        return "x%d" % rng.randrange(n)
    r = rng.random()
    if r < 0.2:
        return "~" + random_expr(rng, n, names, depth - 1)
    op = rng.choice(["&", "|", "^"])
    a = random_expr(rng, n, names, depth - 1)
    b = random_expr(rng, n, names, depth - 1)
    if rng.random() < 0.5:
        return "(%s %s %s)" % (a, op, b)
    return "%s %s %s" % (a, op, b)


def random_program(rng, n):
    stmts = []
    names = []
    for t in range(rng.randrange(0, 6)):
        name = "t%d" % t
        stmts.append(("def", name, random_expr(rng, n, names, 4)))
        names.append(name)
    for _ in range(rng.randrange(1, 4)):
        stmts.append(("assert", None, random_expr(rng, n, names, 4)))
    text = "\n".join(("%s = %s" % (nm, tx)) if k == "def" else tx for k, nm, tx in stmts) + "\n"
    return stmts, text


# ---------------------------------------------------------- paper examples

def test_paper_generators_n3():
    rows = {}
    with open(os.path.join(GOLDEN, "paper_generators_n3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, bits = line.split()
            rows[name] = bits
    # the paper's b1 (top row, most significant bit) is our x2
    for paper_name, var in (("b1", 2), ("b2", 1), ("b3", 0)):
        w = int(oracle.dnf("x%d" % var, 3)[0])
        printed = "".join(str((w >> i) & 1) for i in range(8))
        assert printed == rows[paper_name]
        assert oracle.bitpar_dnf("x%d" % var, 3)[0] == w


def test_baequ4_fixture():
    want = {}
    with open(os.path.join(GOLDEN, "baequ4.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            want[k] = v
    text, n = workloads.baequ4()
    assert models_of(text, n) == [int(v) for v in want["models"]]
    assert int(oracle.dnf(text, n)[0]) == int(want["dnf_word0"][0], 16)
    assert oracle.count(text, n) == 3


# ------------------------------------------------- free generator property

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_minterms_have_one_model(n):
    for alpha in range(1 << n):
        lits = [("x%d" % k) if (alpha >> k) & 1 else ("~x%d" % k) for k in range(n)]
        assert models_of(" & ".join(lits), n) == [alpha]


def test_minterms_n10_sample():
    rng = random.Random(5)
    n = 10
    for alpha in rng.sample(range(1 << n), 40):
        lits = [("x%d" % k) if (alpha >> k) & 1 else ("~x%d" % k) for k in range(n)]
        assert models_of(" & ".join(lits), n) == [alpha]


# --------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [0, 1, 3, 5, 6, 7, 12])
def test_closed_forms(n):
    assert oracle.count("1", n) == 1 << n
    assert oracle.count("0", n) == 0
    if n == 0:
        return
    allv = ["x%d" % k for k in range(n)]
    assert models_of(" & ".join(allv), n) == [(1 << n) - 1]
    assert oracle.count(" | ".join(allv), n) == (1 << n) - 1
    assert oracle.count(" ^ ".join(allv), n) == 1 << (n - 1)
    assert oracle.count("x%d" % (n - 1), n) == 1 << (n - 1)
    assert oracle.count("~x0", n) == 1 << (n - 1)
    assert oracle.count("x0 ^ x0", n) == 0
    assert oracle.count("x0 | ~x0", n) == 1 << n


def test_unused_variables_double_the_count():
    # a letter that does not occur still indexes valuations (all of 2^P)
    for n in range(2, 9):
        assert oracle.count("x0 & x1", n) == 1 << (n - 2)


def test_dnf_tail_bits_zero_small_n():
    for n in range(0, 6):
        w = int(oracle.dnf("1", n)[0])
        assert w == (1 << (1 << n)) - 1


# ------------------------------------------ Proposition 2.2, independent route

@pytest.mark.parametrize("seed", range(40))
def test_random_formulas_against_python_bigint(seed):
    rng = random.Random(seed)
    n = rng.randrange(0, 11)
    if n == 0:
        n = 1
    stmts, text = random_program(rng, n)
    want = python_dnf(stmts, n)
    got = words_to_int(oracle.dnf(text, n))
    assert got == want, text
    assert words_to_int(oracle.bitpar_dnf(text, n)) == want
    assert oracle.count(text, n) == bin(want).count("1")
    assert models_of(text, n) == [i for i in range(1 << n) if (want >> i) & 1]


def test_precedence_is_pythons():
    # each pair differs only by precedence; Python decides
    for text in ["x0 | x1 & x2", "x0 ^ x1 & x2", "x0 | x1 ^ x2", "~x0 & x1",
                 "x0 & x1 ^ x2 | x3", "~x0 ^ ~x1 | x2 & ~x3", "x3 ^ x2 ^ ~x1 ^ x0"]:
        want = python_dnf([("assert", None, text)], 4)
        assert words_to_int(oracle.dnf(text, 4)) == want, text


def test_eval_at_matches_dnf():
    rng = random.Random(11)
    stmts, text = random_program(rng, 9)
    d = words_to_int(oracle.dnf(text, 9))
    idx = list(range(512))
    got = oracle.eval_at(text, 9, idx)
    assert [int(g) for g in got] == [(d >> i) & 1 for i in idx]


def test_bitpar_matches_valuations_random_3cnf():
    for seed in range(4):
        text, n = workloads.random_3cnf(16, 68, seed)
        assert np.array_equal(oracle.dnf(text, n), oracle.bitpar_dnf(text, n))


def test_random_3cnf_against_brute_force():
    text, n = workloads.random_3cnf(12, 51, 3)
    clauses = []
    for line in text.strip().split("\n"):
        cl = []
        for lit in line.split("|"):
            lit = lit.strip()
            cl.append((int(lit.lstrip("~x")), lit.startswith("~")))
        clauses.append(cl)
    want = [mu for mu in range(1 << n)
            if all(any(((mu >> k) & 1) != neg for k, neg in cl) for cl in clauses)]
    assert models_of(text, n) == want


# ------------------------------------------------------------- theories

def bell(k):
    # Bell triangle
    row = [1]
    for _ in range(k):
        nxt = [row[-1]]
        for v in row:
            nxt.append(nxt[-1] + v)
        row = nxt
    return row[0]


def set_partitions(k):
    """Restricted growth strings: block label of each element."""
    if k == 0:
        yield []
        return
    def rec(prefix, m):
        if len(prefix) == k:
            yield list(prefix)
            return
        for b in range(m + 1):
            yield from rec(prefix + [b], max(m, b + 1))
    yield from rec([0], 1)


@pytest.mark.parametrize("k", range(1, 8))
def test_equivalence_bell(k):
    text, n = workloads.equivalence_relations(k)
    assert oracle.count(text, n) == bell(k)
    text2, _ = workloads.equivalence_relations(k, deduplicate=False)
    assert oracle.count(text2, n) == bell(k)


@pytest.mark.parametrize("k", range(2, 6))
def test_equivalence_models_are_set_partitions(k):
    text, n = workloads.equivalence_relations(k)
    want = []
    for labels in set_partitions(k):
        mu = 0
        for i, j in combinations(range(k), 2):
            if labels[i] == labels[j]:
                mu |= 1 << equivalence_var(k, i, j)
        want.append(mu)
    assert models_of(text, n) == sorted(want)


@pytest.mark.parametrize("k", range(1, 6))
def test_permutation_matrices(k):
    text, n = workloads.permutation_matrices(k)
    want = sorted(sum(1 << (k * r + p[r]) for r in range(k)) for p in permutations(range(k)))
    assert models_of(text, n) == want


def triangle_free_brute(k):
    edges = list(combinations(range(k), 2))
    idx = {e: i for i, e in enumerate(edges)}
    out = []
    for mu in range(1 << len(edges)):
        ok = True
        for i, j, l in combinations(range(k), 3):
            if (mu >> idx[(i, j)]) & 1 and (mu >> idx[(j, l)]) & 1 and (mu >> idx[(i, l)]) & 1:
                ok = False
                break
        if ok:
            out.append(mu)
    return out


@pytest.mark.parametrize("k", range(1, 6))
def test_triangle_free_brute_force(k):
    text, n = workloads.triangle_free(k)
    assert models_of(text, n) == triangle_free_brute(k)


def triangle_free_by_vertex_addition(kmax):
    """Count triangle-free labeled graphs by adding vertices: the new vertex's
    neighbourhood must be an independent set of the graph so far."""
    graphs = [()]   # adjacency bitmasks
    counts = [1]
    for k in range(1, kmax + 1):
        nxt = []
        for g in graphs:
            m = len(g)
            for s in range(1 << m):
                indep = all(not (g[v] & s) for v in range(m) if (s >> v) & 1)
                if indep:
                    ng = tuple(g[v] | ((1 << m) if (s >> v) & 1 else 0) for v in range(m)) + (s,)
                    nxt.append(ng)
        graphs = nxt
        counts.append(len(graphs))
    return counts


def test_triangle_free_counts_k6_k7():
    counts = triangle_free_by_vertex_addition(6)
    for k in (3, 4, 5, 6):
        text, n = workloads.triangle_free(k)
        assert oracle.count(text, n) == counts[k]
    # k = 7 from the same recursion, counting only (no graph list kept)
    text, n = workloads.triangle_free(6)
    graphs6 = triangle_free_by_vertex_addition_graphs(6)
    c7 = 0
    for g in graphs6:
        for s in range(1 << 6):
            if all(not (g[v] & s) for v in range(6) if (s >> v) & 1):
                c7 += 1
    text, n = workloads.triangle_free(7)
    assert oracle.count(text, n) == c7


def triangle_free_by_vertex_addition_graphs(k):
    graphs = [()]
    for _ in range(k):
        nxt = []
        for g in graphs:
            m = len(g)
            for s in range(1 << m):
                if all(not (g[v] & s) for v in range(m) if (s >> v) & 1):
                    nxt.append(tuple(g[v] | ((1 << m) if (s >> v) & 1 else 0) for v in range(m)) + (s,))
        graphs = nxt
    return graphs


@pytest.mark.slow
def test_triangle_free_k8_bitpar_and_valuations_agree():
    text, n = workloads.triangle_free(8)
    c = oracle.bitpar_count(text, n)
    assert c == 4682270  # labeled triangle-free graphs on 8 vertices
    assert oracle.count(text, n) == c


# ------------------------------------------------------ ordered structures

def labeled_posets(m):
    """Partial orders on {0..m-1} by brute force over strict relations."""
    pairs = [(i, j) for i in range(m) for j in range(m) if i != j]
    out = 0
    for bits in range(1 << len(pairs)):
        le = {(i, i) for i in range(m)}
        for t, p in enumerate(pairs):
            if (bits >> t) & 1:
                le.add(p)
        if any((j, i) in le for (i, j) in le if i != j):
            continue
        if any((i, l) not in le for (i, j) in le for (jj, l) in le if j == jj):
            continue
        out += 1
    return out


def special_element_brute(m):
    pairs = list(permutations(range(m), 2))
    out = 0
    for bits in range(1 << len(pairs)):
        le = {(i, i) for i in range(m)}
        for t, p in enumerate(pairs):
            if (bits >> t) & 1:
                le.add(p)
        if any((j, i) in le for (i, j) in le if i != j):
            continue
        if any((i, l) not in le for (i, j) in le for (jj, l) in le if j == jj):
            continue
        if any(all((i, j) in le or (j, i) in le for j in range(m)) for i in range(m)):
            out += 1
    return out


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_special_element_posets(m):
    text, n = workloads.special_element_posets(m)
    assert n == m * m - m
    assert oracle.count(text, n) == special_element_brute(m)


def test_labeled_poset_numbers():
    assert [labeled_posets(m) for m in range(5)] == [1, 1, 3, 19, 219]


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_bounded_posets(m):
    # Section 5.2: l = m(m-1)|K| with |K| the posets on the m-2 inner elements
    text, n = workloads.bounded_posets(m)
    assert n == m * m - 5 * m + 6
    assert oracle.count(text, n) == labeled_posets(m - 2)


# ------------------------------------------------------------------ errors

@pytest.mark.parametrize("bad", ["x0 &", "x0 & (x1", "2", "y0", "t = x0\nt = x1\nt", "x0 = x1", "", "# only\n"])
def test_parse_errors(bad):
    with pytest.raises(oracle.OracleError):
        oracle.count(bad, 3)


def test_variable_out_of_range():
    with pytest.raises(oracle.OracleError):
        oracle.count("x5", 5)


def test_count_range_partitions_the_count():
    text, n = workloads.random_3cnf(16, 50, 2)
    total = oracle.count(text, n)
    cuts = [0, 1, 63, 64, 1000, 4097, 30000, 1 << n]
    parts = sum(oracle.count_range(text, n, a, b) for a, b in zip(cuts, cuts[1:]))
    assert parts == total
    want = oracle.models(text, n)[0]
    assert oracle.count_range(text, n, 1000, 30000) == int(((want >= 1000) & (want < 30000)).sum())
