"""Counting with definable partitions (Section 3.4; bounded partial orders,
Section 5.2): c-partition enumeration against the closed forms, killed
letters against an independent textual substitution, and the formula (ltn)
total against brute force and the oracle's direct count."""

import itertools
import random
import re
from math import comb, factorial

import numpy as np
import pytest

import oracle
import workloads
from paper_1310_6978_amd import fbg, tba
from tests.formula_gen import random_program
from tests.test_oracle_pins import labeled_posets


def substitute(text, n_letters, assume):
    """Killed letters replaced by their constants and the free ones
    renumbered in increasing order, by plain text substitution."""
    renum, f = {}, 0
    for k in range(n_letters):
        if assume[k] < 0:
            renum[k] = f
            f += 1

    def repl(m):
        k = int(m.group(1))
        return str(int(assume[k])) if assume[k] >= 0 else "x%d" % renum[k]
    return re.sub(r"\bx(\d+)\b", repl, text), f


def test_c_partitions_match_the_closed_form():
    for n in range(0, 7):
        for m in range(1, 5):
            brute = sorted(a for a in itertools.product(range(n + 1), repeat=m) if sum(a) == n)
            got = sorted(tba.c_partition_sizes(n, m))
            assert got == brute
            assert tba.c_nm(n, m) == len(brute), (n, m)


def test_weights_count_every_map_to_the_components():
    # every map of an n-set to m labeled components is one labeling of one
    # c-partition: the weights of formula (ltn) sum to m^n
    for n in range(0, 7):
        for m in range(1, 5):
            assert sum(tba.weight(a) for a in tba.c_partition_sizes(n, m)) == m ** n


def test_layerings_number_2_to_the_s_minus_1():
    assert list(tba.layer_sizes(0)) == [()]
    for s in range(1, 12):
        lay = list(tba.layer_sizes(s))
        assert len(lay) == len(set(lay)) == 2 ** (s - 1)       # Proposition posn, s = n - 2
        assert all(min(a) >= 1 and sum(a) == s for a in lay)


def test_layer_weights_count_ordered_set_partitions():
    # sum of multinomials over compositions = ordered set partitions =
    # sum_k k! S(s, k), surjections counted by inclusion-exclusion
    for s in range(0, 9):
        surj = sum(sum((-1) ** j * comb(k, j) * (k - j) ** s for j in range(k + 1)) for k in range(0, s + 1))
        assert sum(tba.weight(a) for a in tba.layer_sizes(s)) == surj


@pytest.mark.parametrize("seed", range(12))
def test_compile_assume_equals_substituted_text(seed):
    rng = random.Random(3300 + seed)
    n = rng.choice([8, 12, 16, 20])
    _, text = random_program(rng, n)
    assume = np.array([rng.choice([-1, -1, 0, 1]) for _ in range(n)], dtype=np.int8)
    sub, f = substitute(text, n, assume)
    p = fbg.compile_assume(text, n, assume)
    assert p.n == f and p.info["n_vars"] == f
    want = oracle.dnf(sub, f)
    for w in (1, 4, 32):
        got, c = p.emulate(w)
        assert np.array_equal(got, want), w


def test_compile_assume_all_free_and_all_killed():
    text = "(x0 | x3) & ~(x1 & x2)\n"
    p = fbg.compile_assume(text, 4, np.full(4, -1, dtype=np.int8))
    q = fbg.Program(text, 4)
    assert np.array_equal(p.emulate(1)[0], q.emulate(1)[0])
    for bits in range(16):
        a = np.array([(bits >> k) & 1 for k in range(4)], dtype=np.int8)
        r = fbg.compile_assume(text, 4, a)
        want = int(bool((a[0] | a[3]) & ~(a[1] & a[2]) & 1))
        assert r.n == 0 and r.emulate(1)[1] == want


def test_compile_assume_errors():
    with pytest.raises(fbg.FbgError) as ei:
        fbg.compile_assume("x0", 2, np.array([-1, 2], dtype=np.int8))
    assert ei.value.status == fbg.FBG_E_INVAL
    with pytest.raises(fbg.FbgError) as ei:
        fbg.compile_assume("x0", 60, np.full(60, -1, dtype=np.int8))
    assert ei.value.status == fbg.FBG_E_RANGE
    with pytest.raises(ValueError):
        fbg.compile_assume("x0", 3, np.full(2, -1, dtype=np.int8))
    # 60 letters of which 40 are killed: fine
    a = np.full(60, -1, dtype=np.int8)
    a[:40] = 1
    assert fbg.compile_assume("x0 & x59", 60, a).n == 20


def parts_total_emulated(n):
    text, nl = workloads.bounded_posets(n)
    total, parts = 0, 0
    for sizes, assume, extra in tba.bounded_poset_parts(n):
        p = fbg.compile_assume(text + extra, nl, assume)
        c = p.emulate(1)[1]
        sub, f = substitute(text + extra, nl, assume)
        assert c == oracle.count(sub, f), sizes
        total += tba.weight(sizes) * c
        parts += 1
    assert parts == max(1, 2 ** (n - 3)) if n >= 3 else parts == 1
    return total


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_bounded_posets_by_layers_equal_brute_force(n):
    assert parts_total_emulated(n) == labeled_posets(n - 2)


def test_bounded_posets_by_layers_equal_direct_count():
    text, nl = workloads.bounded_posets(7)            # 20 letters after the constants
    assert parts_total_emulated(7) == oracle.count(text, nl)
