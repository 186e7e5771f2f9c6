"""Counting with definable partitions (Section 3.4, the counting procedure,
and its use for bounded partial orders in Section 5.2).

A good definable partition splits every labeled model into components
X_1..X_m.  Up to relabeling, the components can be taken consecutive
(arrangement (c2)); such a c-partition fixes many letters ("killing
variables", step 3), which leaves a much smaller theory T_X.  All T_X are
counted on the device, and the labeled count follows by formula (ltn):

    l_{T,n} = sum over c-partitions X of  C(b_1, a_1) ... C(b_k, a_k) * |K_X|,

with a_i = |X_i|, b_1 = n and b_{i+1} = b_i - a_i.  Every T_X is compiled
with fbg_compile_assume (the killed letters become constants and fold away)
and the |K_X| of all c-partitions are counted in one batched launch.
"""

from dataclasses import dataclass, field
from itertools import permutations
from math import comb

import numpy as np

from . import fbg


def c_partition_sizes(n, m):
    """All size vectors (a_1..a_m), a_i >= 0, sum n: the c-partitions of an
    n-set into m components laid out as in (c2).  Their number is c_{nm} of
    the proposition in Section 3.4."""
    if m == 0:
        if n == 0:
            yield ()
        return
    for a in range(n + 1):
        for rest in c_partition_sizes(n - a, m - 1):
            yield (a,) + rest


def c_nm(n, m):
    """Closed form of the number of c-partitions (Section 3.4): the sum over
    k = 1..m of C(m, k) C(n-1, k-1)."""
    if n == 0:
        return 1
    return sum(comb(m, k) * comb(n - 1, k - 1) for k in range(1, m + 1))


def layer_sizes(s):
    """Size vectors of the layer c-partitions of an s-set (Section 5.2,
    (cpA)): m >= 1 non-empty layers followed by empty ones, i.e. the
    compositions of s.  There are 2^(s-1) of them (Proposition posn with
    s = n - 2); s = 0 has the single empty one."""
    if s == 0:
        yield ()
        return
    for first in range(1, s + 1):
        for rest in layer_sizes(s - first):
            yield (first,) + rest


def weight(sizes):
    """prod_i C(b_i, a_i) of formula (ltn): the labelings that map the
    canonical components onto arbitrary ones."""
    w, left = 1, sum(sizes)
    for a in sizes:
        w *= comb(left, a)
        left -= a
    return w


@dataclass
class Part:
    sizes: tuple
    weight: int
    n_free: int
    count: int = 0


@dataclass
class Result:
    total: int
    parts: list = field(default_factory=list)
    ms: float = 0.0          # device time of the batched count


def run(text, n_letters, parts, words_per_lane=0, cofactor=True, stream=None):
    """Steps 4, 5, 7 and 8 of the counting procedure.  parts: list of
    (sizes, assume, extra) with assume an int8 array of n_letters entries
    (-1 free, 0/1 killed) and extra additional assertion text over the same
    letters (the statement that the partition is the one the formulas
    define).  Returns the total of formula (ltn) and every |K_X|."""
    import torch
    progs, meta = [], []
    for sizes, assume, extra in parts:
        src = text + extra
        p = fbg.compile_assume(src, n_letters, assume)
        progs.append(p)
        meta.append(Part(tuple(sizes), weight(sizes), p.n))
    if not progs:
        return Result(0)
    b = fbg.Batch(progs, words_per_lane=words_per_lane, cofactor=cofactor)
    out = torch.empty(len(progs), dtype=torch.int64, device="cuda")
    s = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    b.count(out=out, stream=s)
    e1.record(s)
    counts = out.cpu().numpy().view(np.uint64).tolist()
    b.free()
    total = 0
    for m, c in zip(meta, counts):
        m.count = int(c)
        total += m.weight * m.count
    return Result(total, meta, e0.elapsed_time(e1))


def inner_letters(n):
    """Letter numbers of the bounded-poset theory on {0..n-1}: p(i, j) for
    distinct i, j in 1..n-2, ordered pairs in lexicographic order (the
    letters that the constants of Section 5.2 leave free)."""
    inner = list(range(1, n - 1))
    return {ij: k for k, ij in enumerate(permutations(inner, 2))}


def bounded_poset_parts(n):
    """The c-partitions of Section 5.2 for partial orders on {0..n-1} with
    least element 0 and greatest n-1: the inner elements 1..n-2 cut into
    consecutive layers of k-minimal elements.  For each layering:
      * killed: p(i, j) = 0 whenever the layer of j is not above the layer
        of i (an element is never below one of an earlier or the same layer);
      * asserted: every element of layer k >= 2 lies above some element of
        layer k-1 (otherwise it would be minimal earlier), which with the
        killed letters says that the layers are exactly the k-minimal sets.
    Yields (sizes, assume, extra)."""
    letters = inner_letters(n)
    s = max(n - 2, 0)
    for sizes in layer_sizes(s):
        layer, el = {}, 1
        for k, a in enumerate(sizes):
            for _ in range(a):
                layer[el] = k
                el += 1
        assume = np.full(len(letters), -1, dtype=np.int8)
        for (i, j), x in letters.items():
            if layer[j] <= layer[i]:
                assume[x] = 0
        extra = []
        for i in range(1, n - 1):
            k = layer[i]
            if k == 0:
                continue
            below = [letters[(j, i)] for j in range(1, n - 1) if layer[j] == k - 1]
            extra.append("(" + " | ".join("x%d" % x for x in below) + ")")
        yield sizes, assume, "".join(e + "\n" for e in extra)


def bounded_posets(n, text, n_letters, **kw):
    """Labeled partial orders on {0..n-1} with least element 0 and greatest
    n-1 (equivalently, labeled partial orders on n-2 elements) by the
    counting procedure.  text, n_letters: the theory of Section 5.2 with its
    constants substituted, over the letters of inner_letters(n)."""
    if n_letters != len(inner_letters(n)):
        raise ValueError("theory has %d letters, expected %d" % (n_letters, len(inner_letters(n))))
    return run(text, n_letters, list(bounded_poset_parts(n)), **kw)
