"""Front end for TBA-style scripts (Section 4.2): the paper's SO.txt script and
other theories translate to propositional text whose model counts match
brute force over the structures themselves."""

from itertools import permutations

import pytest

import oracle
from paper_1310_6978_amd import frontend
from tests.test_oracle_pins import labeled_posets, special_element_brute


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_so_script_counts(n):
    t = frontend.translate(frontend.so_script(n))
    assert t.n == n * n - n                       # n letters killed (Section 4.2)
    assert sorted(t.axioms) == ["f1", "f2", "f3"]
    assert oracle.count(t.text, t.n) == special_element_brute(n)


def test_so_script_models_decode_to_posets():
    n = 3
    t = frontend.translate(frontend.so_script(n))
    models, total = oracle.models(t.text, t.n)
    assert total == 12
    for m in models:
        le = {args for rel, args in t.decode(m)}
        assert all((i, i) in le for i in range(n))                      # reflexive (killed to 1)
        assert not any((j, i) in le for (i, j) in le if i != j)         # antisymmetric
        assert all((i, l) in le for (i, j) in le for (jj, l) in le if j == jj)  # transitive


def test_partial_orders_without_special_element():
    for n in range(1, 5):
        script = """S = range({n})
S2 = perm(S, 2)
S3 = perm(S, 3)
anti = A[i,j:S2] (~p(i,j) | ~p(j,i))
trans = A[i,j,k:S3] (~(p(i,j) & p(j,k)) | p(i,k))
assumptions = {{p(i,i): 1 for i in S}}
""".format(n=n)
        t = frontend.translate(script)
        assert oracle.count(t.text, t.n) == labeled_posets(n)


def test_exists_forall_chain_and_xor():
    # functions f: S -> S as letters q(a, b) = "f(a) = b": exactly one b per a
    script = """S = range(3)
total = A[a:S] (E[b:S] (q(a,b)))
single = A[a:S] (A[b:S].A[c:S] (~q(a,b) | ~q(a,c) | (1 if b == c else 0)))
"""
    t = frontend.translate(script)
    assert t.n == 9
    assert oracle.count(t.text, t.n) == 27        # 3^3 functions
    t2 = frontend.translate("S = range(4)\nodd = E[i:S] (r(i)) ^ A[i:S] (r(i))\n")
    # "some" xor "all": true unless none or all of the 4 letters hold
    assert oracle.count(t2.text, t2.n) == 16 - 2


def test_killed_letters_fold_to_constants():
    t = frontend.translate("S = range(2)\nf = A[i:S] (p(i) | p(1-i))\nassumptions = {p(0): 0}\n")
    assert t.n == 1 and t.letters == [("p", (1,))]
    assert oracle.count(t.text, t.n) == 1


def test_errors():
    with pytest.raises(ValueError):
        frontend.translate("S = range(2)\n")
    with pytest.raises(SyntaxError):
        frontend.translate("S = range(2)\nf = A[i:S] p(i)\n")
    with pytest.raises(ValueError):
        frontend.translate("S = range(2)\nf = A[i:S] (p(i))\nassumptions = {p(0): 2}\n")
