"""Unlabeled counts (Section 3.2, kappa) by the Frobenius-Burnside lemma:
cycle types and class sizes against closed forms, letter identification
against plain textual substitution, and kappa against the oracle's orbit
count (smallest image of every model under every relabeling)."""

import itertools
import random
import re
from math import factorial

import numpy as np
import pytest

import oracle
from paper_1310_6978_amd import fbg, frontend, unlabeled
from tests.formula_gen import random_program


def partition_numbers(m):
    """p(0..m) by the standard recursion over the largest part."""
    table = [[0] * (m + 1) for _ in range(m + 1)]   # table[n][k]: partitions of n, parts <= k
    for k in range(m + 1):
        table[0][k] = 1
    for n in range(1, m + 1):
        for k in range(1, m + 1):
            table[n][k] = table[n][k - 1] + (table[n - k][k] if k <= n else 0)
    return [table[n][n] for n in range(m + 1)]


def substitute(text, subst):
    def repl(mt):
        v = int(subst[int(mt.group(1))])
        return "0" if v == -1 else "1" if v == -2 else "x%d" % v
    return re.sub(r"\bx(\d+)\b", repl, text)


POSETS = """S = range({n})
S2 = perm(S, 2)
S3 = perm(S, 3)
anti = A[i,j:S2] (~p(i,j) | ~p(j,i))
trans = A[i,j,k:S3] (~(p(i,j) & p(j,k)) | p(i,k))
assumptions = {{p(i,i): 1 for i in S}}
"""

EQUIV = """S = range({n})
S2 = perm(S, 2)
S3 = perm(S, 3)
sym = A[i,j:S2] (~q(i,j) | q(j,i))
trans = A[i,j,k:S3] (~(q(i,j) & q(j,k)) | q(i,k))
assumptions = {{q(i,i): 1 for i in S}}
"""

GRAPHS = """S = range({n})
S2 = perm(S, 2)
sym = A[i,j:S2] (~e(i,j) | e(j,i))
assumptions = {{e(i,i): 0 for i in S}}
"""


def letter_perms(tr, n):
    """The action of every relabeling of range(n) on the free letters."""
    index = {l: k for k, l in enumerate(tr.letters)}
    rows = []
    for sigma in itertools.permutations(range(n)):
        rows.append([index[(rel, tuple(sigma[a] for a in args))] for rel, args in tr.letters])
    return np.array(rows, dtype=np.int32)


def kappa_emulated(tr, n):
    """The lemma's sum with every |Fix| counted by the host emulation of the
    compiled program (the device path runs the same programs)."""
    total = 0
    for lam in unlabeled.partitions(n):
        fs = unlabeled.fixed_substitution(tr.letters, tr.killed, unlabeled.permutation(lam, list(range(n))))
        if fs is None:
            continue
        subst, nfree = fs
        p = fbg.compile_subst(tr.text, tr.n, subst, nfree)
        fixed = p.emulate(1)[1]
        assert fixed == oracle.count(substitute(tr.text, subst), nfree)
        total += unlabeled.class_size(lam) * fixed
    assert total % factorial(n) == 0
    return total // factorial(n)


def test_cycle_types_and_class_sizes():
    p = partition_numbers(10)
    for n in range(0, 11):
        lams = list(unlabeled.partitions(n))
        assert len(lams) == len(set(lams)) == p[n]
        assert all(sum(l) == n for l in lams)
        assert sum(unlabeled.class_size(l) for l in lams) == factorial(n)
    # the class of a cycle type by brute force over S_5
    for lam in unlabeled.partitions(5):
        brute = 0
        for sigma in itertools.permutations(range(5)):
            seen, cyc = set(), []
            for a in range(5):
                if a in seen:
                    continue
                k, b = 0, a
                while b not in seen:
                    seen.add(b)
                    b = sigma[b]
                    k += 1
                cyc.append(k)
            brute += tuple(sorted(cyc, reverse=True)) == lam
        assert brute == unlabeled.class_size(lam)


@pytest.mark.parametrize("seed", range(10))
def test_compile_subst_equals_substituted_text(seed):
    rng = random.Random(5100 + seed)
    n = rng.choice([6, 10, 14])
    _, text = random_program(rng, n)
    nfree = rng.randrange(1, n)
    subst = np.array([rng.choice([-1, -2] + list(range(nfree))) for _ in range(n)], dtype=np.int32)
    p = fbg.compile_subst(text, n, subst, nfree)
    assert p.n == nfree
    want = oracle.dnf(substitute(text, subst), nfree)
    for w in (1, 8):
        assert np.array_equal(p.emulate(w)[0], want)


def test_compile_subst_errors():
    with pytest.raises(fbg.FbgError) as ei:
        fbg.compile_subst("x0", 2, np.array([0, 3], dtype=np.int32), 2)
    assert ei.value.status == fbg.FBG_E_INVAL
    with pytest.raises(fbg.FbgError) as ei:
        fbg.compile_subst("x0", 2, np.array([0, -3], dtype=np.int32), 2)
    assert ei.value.status == fbg.FBG_E_INVAL
    with pytest.raises(fbg.FbgError) as ei:
        fbg.compile_subst("x0", 2, np.array([0, 1], dtype=np.int32), 49)
    assert ei.value.status == fbg.FBG_E_RANGE
    # a variable no letter maps to still doubles the count
    p = fbg.compile_subst("x0 & x1", 2, np.array([0, 0], dtype=np.int32), 3)
    assert p.emulate(1)[1] == 4


def test_oracle_orbits_pins():
    # equivalence relations up to relabeling are integer partitions
    p = partition_numbers(6)
    for n in range(1, 6):
        tr = frontend.translate(EQUIV.format(n=n))
        assert oracle.orbits(tr.text, tr.n, letter_perms(tr, n))[0] == p[n]
    # posets on 1..3 elements: 1, 2, 5 (antichain / chain; for 3: antichain,
    # one comparable pair, V, inverted V, chain)
    for n, want in ((1, 1), (2, 2), (3, 5)):
        tr = frontend.translate(POSETS.format(n=n))
        assert oracle.orbits(tr.text, tr.n, letter_perms(tr, n))[0] == want
    # graphs on 3 vertices: 0, 1, 2 or 3 edges
    tr = frontend.translate(GRAPHS.format(n=3))
    assert oracle.orbits(tr.text, tr.n, letter_perms(tr, 3)) == (4, 8)


@pytest.mark.parametrize("script,n", [(EQUIV, 4), (EQUIV, 5), (POSETS, 3), (POSETS, 4), (GRAPHS, 4),
                                      (GRAPHS, 5)])
def test_kappa_by_the_lemma_equals_orbit_count(script, n):
    tr = frontend.translate(script.format(n=n))
    assert kappa_emulated(tr, n) == oracle.orbits(tr.text, tr.n, letter_perms(tr, n))[0]


def test_fixed_substitution_rejects_asymmetric_assumptions():
    tr = frontend.translate(POSETS.format(n=3).replace("for i in S}", "for i in S} | {p(0,1): 1}"))
    with pytest.raises(ValueError):
        unlabeled.fixed_substitution(tr.letters, tr.killed, unlabeled.permutation((2, 1), [0, 1, 2]))
