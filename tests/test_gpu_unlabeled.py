"""GPU: unlabeled counts (Section 3.2, kappa) by the Frobenius-Burnside
lemma, every fixed-point count in one batched launch, against the oracle's
orbit count and the partition numbers."""

import numpy as np
import pytest

import oracle
from paper_1310_6978_amd import frontend, unlabeled
from tests.test_unlabeled import EQUIV, GRAPHS, POSETS, letter_perms, partition_numbers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1310_6978_amd import fbg
    return fbg


@pytest.mark.parametrize("script,n", [(POSETS, 1), (POSETS, 2), (POSETS, 3), (POSETS, 4), (POSETS, 5),
                                      (POSETS, 6), (GRAPHS, 4), (GRAPHS, 5), (GRAPHS, 6)])
def test_kappa_equals_oracle_orbits(F, script, n):
    tr = frontend.translate(script.format(n=n))
    res = unlabeled.count_translation(tr, range(n))
    orbits, models = oracle.orbits(tr.text, tr.n, letter_perms(tr, n))
    assert res.unlabeled == orbits
    assert res.labeled == models


def test_equivalence_relations_up_to_relabeling_are_partitions(F):
    # ordered-pair letters: n(n-1) of them, 42 at n = 7 (the identity term
    # counts the whole theory)
    p = partition_numbers(7)
    for n in range(1, 8):
        tr = frontend.translate(EQUIV.format(n=n))
        res = unlabeled.count_translation(tr, range(n), cofactor=(n % 2 == 0))
        assert res.unlabeled == p[n], n
        assert len(res.terms) == p[n]


def test_cofactor_and_plain_agree(F):
    tr = frontend.translate(POSETS.format(n=6))
    a = unlabeled.count_translation(tr, range(6), cofactor=True)
    b = unlabeled.count_translation(tr, range(6), words_per_lane=4)
    assert [t.fixed for t in a.terms] == [t.fixed for t in b.terms]
    assert (a.unlabeled, a.labeled) == (b.unlabeled, b.labeled)
