"""Unlabeled models: the number kappa_{T,n} of non-isomorphic models of size
n (Section 3.2), by the Frobenius-Burnside counting lemma stated there.

The labeled models of T with domain I_n are permuted by S_n; kappa is the
number of orbits.  Counting orbits by the lemma,

    kappa = (1 / n!) * sum over sigma in S_n of |Fix(sigma)|,

where Fix(sigma) is the set of labeled models that sigma maps onto
themselves: the valuations in which every letter R(a..) has the value of
R(sigma(a)..).  |Fix(sigma)| depends only on the cycle type of sigma, and it
is itself a model count: the theory with the letters of each orbit of sigma
identified (fbg_compile_subst), so the whole sum is one batched count of
p(n) programs on the device -- bit logic like every other count here, with
no isomorphism test.

The theory must be invariant under relabeling: the image of every letter is a
letter of the theory, and killed letters map to killed letters with the same
value (otherwise the labeled models do not form a union of orbits).
"""

from dataclasses import dataclass, field
from math import factorial

import numpy as np

from . import fbg

ZERO, ONE = -1, -2   # FBG_SUBST_ZERO / FBG_SUBST_ONE


def partitions(n, largest=None):
    """The integer partitions of n as non-increasing tuples (cycle types)."""
    if largest is None:
        largest = n
    if n == 0:
        yield ()
        return
    for k in range(min(n, largest), 0, -1):
        for rest in partitions(n - k, k):
            yield (k,) + rest


def class_size(cycle_type):
    """Permutations of n = sum(cycle_type) elements with that cycle type:
    n! / prod_k (k^{m_k} m_k!)."""
    n = sum(cycle_type)
    den = 1
    for k in set(cycle_type):
        m = cycle_type.count(k)
        den *= k ** m * factorial(m)
    return factorial(n) // den


def permutation(cycle_type, domain):
    """A permutation of `domain` with the given cycle type: consecutive
    elements form the cycles.  Returned as a dict element -> image."""
    sigma, pos = {}, 0
    for k in cycle_type:
        cyc = domain[pos:pos + k]
        for i, a in enumerate(cyc):
            sigma[a] = cyc[(i + 1) % k]
        pos += k
    return sigma


def fixed_substitution(letters, killed, sigma):
    """Substitution for fbg_compile_subst whose models are the valuations
    fixed by sigma: letters in one orbit of sigma share a variable, an orbit
    through a killed letter takes its constant.  Returns (subst, n_free), or
    None when an orbit meets both constants (no model is fixed)."""
    index = {l: k for k, l in enumerate(letters)}
    parent = list(range(len(letters)))
    const = {}

    def find(k):
        while parent[k] != k:
            parent[k] = parent[parent[k]]
            k = parent[k]
        return k

    def image(l):
        rel, args = l
        return (rel, tuple(sigma.get(a, a) for a in args))

    for l, v in killed.items():
        img = image(l)
        if img not in killed or killed[img] != v:
            raise ValueError("the killed letters are not invariant under relabeling (%r -> %r)" % (l, img))
    for k, l in enumerate(letters):
        img = image(l)
        if img in index:
            a, b = find(k), find(index[img])
            if a != b:
                parent[a] = b
        elif img in killed:
            r = find(k)
            const.setdefault(r, set()).add(killed[img])
        else:
            raise ValueError("letter %r maps to %r, which is not a letter of the theory" % (l, img))
    # constants bound to a root before a later union moved it
    bound = {}
    for r, vs in const.items():
        bound.setdefault(find(r), set()).update(vs)
    subst = np.zeros(len(letters), dtype=np.int32)
    ids = {}
    for k in range(len(letters)):
        r = find(k)
        vs = bound.get(r)
        if vs:
            if len(vs) > 1:
                return None
            subst[k] = ONE if 1 in vs else ZERO
        else:
            if r not in ids:
                ids[r] = len(ids)
            subst[k] = ids[r]
    return subst, len(ids)


@dataclass
class Term:
    cycle_type: tuple
    class_size: int
    n_free: int
    fixed: int = 0


@dataclass
class Result:
    unlabeled: int
    labeled: int
    terms: list = field(default_factory=list)


def count(text, letters, killed, domain, words_per_lane=0, cofactor=False, stream=None):
    """kappa and l for the theory `text` over `letters` (letters[k] =
    (relation, args) of variable xk; `killed` maps the other letters to
    0/1) with domain `domain`.  One batched launch counts every |Fix|."""
    import torch
    domain = list(domain)
    n = len(domain)
    nl = len(letters)
    terms, progs, where = [], [], []
    for lam in partitions(n):
        t = Term(lam, class_size(lam), 0)
        fs = fixed_substitution(letters, killed, permutation(lam, domain))
        if fs is not None:
            subst, nfree = fs
            t.n_free = nfree
            where.append(len(terms))
            progs.append(fbg.compile_subst(text, nl, subst, nfree))
        terms.append(t)
    if progs:
        b = fbg.Batch(progs, words_per_lane=words_per_lane, cofactor=cofactor)
        out = torch.empty(len(progs), dtype=torch.int64, device="cuda")
        b.count(out=out, stream=stream)
        got = out.cpu().numpy().view(np.uint64).tolist()
        b.free()
        for i, c in zip(where, got):
            terms[i].fixed = int(c)
    total = sum(t.class_size * t.fixed for t in terms)
    if total % factorial(n):
        raise ArithmeticError("the fixed-point counts do not sum to a multiple of n!: the theory is not "
                              "invariant under relabeling")
    labeled = next(t.fixed for t in terms if t.cycle_type == (1,) * n) if n else terms[0].fixed
    return Result(total // factorial(n), labeled, terms)


def count_translation(tr, domain, **kw):
    """count() for a front-end Translation (paper_1310_6978_amd.frontend)."""
    return count(tr.text, tr.letters, tr.killed, domain, **kw)
