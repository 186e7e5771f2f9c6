"""Formula text for the workloads: propositional translations of small
first-order theories (Section 3.1), random 3-CNF systems, random DAGs, and the
paper's two worked scripts (Sections 4.2 and 5.1).

Every function returns ``(text, n)``: the formula in the text format of this
package and the number of propositional letters (valuation bits).  Nothing
here evaluates a formula.
"""

from itertools import combinations, permutations

from .splitmix import SplitMix64


def cnf_text(clauses):
    """CNF text, one clause per line.  A clause is a list of literals, a
    literal a pair (k, negated).  No clauses gives the constant 1."""
    lines = []
    for cl in clauses:
        lits = [("~x%d" % k) if neg else ("x%d" % k) for (k, neg) in cl]
        lines.append(" | ".join(lits))
    if not lines:           # the empty conjunction
        lines.append("1")
    return "\n".join(lines) + "\n"


# --------------------------------------------------------------------------
# Equivalence relations on k elements (letters x_ij for i<j; reflexivity and
# symmetry are built into the letter set, transitivity is the theory).
# --------------------------------------------------------------------------

def equivalence_var(k, i, j):
    """Letter index of the pair {i, j}, i != j, in lexicographic order of i<j."""
    if i == j:
        raise ValueError("no letter for i == j")
    if i > j:
        i, j = j, i
    # pairs (a, b) with a < i come first: sum_{a<i} (k-1-a)
    return i * (k - 1) - i * (i - 1) // 2 + (j - i - 1)


def equivalence_relations(k, deduplicate=True):
    """Transitivity x_ij & x_jl -> x_il over distinct i, j, l, as clauses
    ~x_ij | ~x_jl | x_il.  With ``deduplicate`` the clause for (i, j, l) and
    (l, j, i) is emitted once (k * C(k-1, 2) clauses); otherwise once per
    ordered triple (k(k-1)(k-2) clauses).  Both define the same function."""
    n = k * (k - 1) // 2
    clauses = []
    seen = set()
    for i in range(k):
        for j in range(k):
            for l in range(k):
                if len({i, j, l}) < 3:
                    continue
                key = (j, min(i, l), max(i, l))
                if deduplicate:
                    if key in seen:
                        continue
                    seen.add(key)
                clauses.append([(equivalence_var(k, i, j), True),
                                (equivalence_var(k, j, l), True),
                                (equivalence_var(k, i, l), False)])
    return cnf_text(clauses), n


# --------------------------------------------------------------------------
# Permutation matrices: k x k 0/1 matrices with exactly one 1 per row/column.
# --------------------------------------------------------------------------

def permutation_matrices(k):
    """x_rc is letter k*r + c.  Per row and per column: one at-least-one
    clause and C(k,2) pairwise at-most-one clauses."""
    n = k * k
    clauses = []
    lines = [[(k * r + c) for c in range(k)] for r in range(k)]
    lines += [[(k * r + c) for r in range(k)] for c in range(k)]
    for line in lines:
        clauses.append([(v, False) for v in line])
        for a, b in combinations(line, 2):
            clauses.append([(a, True), (b, True)])
    return cnf_text(clauses), n


# --------------------------------------------------------------------------
# Triangle-free labeled graphs on k vertices.
# --------------------------------------------------------------------------

def triangle_free(k):
    """Edge letters x_ij (i<j) in lexicographic order; one ~(x_ij & x_jl & x_il)
    per triple i<j<l, written as the negated conjunction."""
    n = k * (k - 1) // 2
    lines = []
    for i, j, l in combinations(range(k), 3):
        a = equivalence_var(k, i, j)
        b = equivalence_var(k, j, l)
        c = equivalence_var(k, i, l)
        lines.append("~(x%d & x%d & x%d)" % (a, b, c))
    if not lines:
        lines.append("1")
    return "\n".join(lines) + "\n", n


# --------------------------------------------------------------------------
# Random 3-CNF (the system-of-equations form of Section 5.1 with random
# clauses).
# --------------------------------------------------------------------------

def random_3cnf(n, m, seed):
    """m clauses over n >= 3 variables.  Per literal: draw the variable as
    ``below(n)``, redrawing while it repeats one already in the clause, then
    draw its sign with ``coin()`` (1 = negated)."""
    if n < 3:
        raise ValueError("3-CNF needs n >= 3")
    rng = SplitMix64(seed)
    clauses = []
    for _ in range(m):
        cl = []
        used = set()
        while len(cl) < 3:
            v = rng.below(n)
            if v in used:
                continue
            used.add(v)
            cl.append((v, bool(rng.coin())))
        clauses.append(cl)
    return cnf_text(clauses), n


def cnf_clause_count(n):
    """Clauses for ratio 4.25: floor(4.25 n + 1/2)."""
    return int(4.25 * n + 0.5)


# --------------------------------------------------------------------------
# Random Boolean DAGs over {AND, OR, XOR, NOT}.
# --------------------------------------------------------------------------

_DAG_OPS = ("&", "|", "^", "~")


def random_dag(n, size, seed):
    """``size`` op nodes t0..t{size-1}.  Node q draws its op as ``below(4)``
    (AND, OR, XOR, NOT) and each operand as ``below(n + q)``: values below n
    are the generators x0..x{n-1}, the rest are the earlier nodes.  The
    formula is the last node."""
    rng = SplitMix64(seed)
    lines = []

    def operand(q):
        a = rng.below(n + q)
        return ("x%d" % a) if a < n else ("t%d" % (a - n))

    for q in range(size):
        op = _DAG_OPS[rng.below(4)]
        if op == "~":
            lines.append("t%d = ~%s" % (q, operand(q)))
        else:
            a = operand(q)
            b = operand(q)
            lines.append("t%d = %s %s %s" % (q, a, op, b))
    lines.append("t%d" % (size - 1))
    return "\n".join(lines) + "\n", n


def random_dag_batch(count, seed, n_lo=10, n_hi=30, size_lo=50, size_hi=2000):
    """``count`` DAG formulas: per formula draw n, then the size, then a
    64-bit seed for its nodes, all from one stream."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        n = rng.uniform_int(n_lo, n_hi)
        size = rng.uniform_int(size_lo, size_hi)
        fseed = rng.next()
        out.append(random_dag(n, size, fseed))
    return out


# --------------------------------------------------------------------------
# The paper's worked scripts.
# --------------------------------------------------------------------------

def baequ4():
    """The system x + y + ~z + u = 1, x | yz = u of Section 5.1 with
    x, y, z, u as x3, x2, x1, x0 (so the index reads xyzu in binary)."""
    text = "x3 ^ x2 ^ ~x1 ^ x0\n~((x3 | x2 & x1) ^ x0)\n"
    return text, 4


def _pair_letters(elements):
    """Letters p(i, j) for ordered pairs of distinct elements, lexicographic."""
    idx = {}
    for i, j in permutations(elements, 2):
        idx[(i, j)] = len(idx)
    return idx


def special_element_posets(n):
    """The script SO.txt of Section 4.2: partial orders on {0..n-1} with an
    element comparable to all others.  p(i,i) is killed to 1 (reflexivity);
    the killed letters are written as the constant 1 and left to constant
    folding.  The other n^2 - n letters are ordered pairs in lexicographic
    order."""
    S = list(range(n))
    idx = _pair_letters(S)

    def p(i, j):
        return "1" if i == j else "x%d" % idx[(i, j)]

    lines = []
    for i, j in permutations(S, 2):                 # antisymmetry
        lines.append("(~%s | ~%s)" % (p(i, j), p(j, i)))
    for i, j, k in permutations(S, 3):              # transitivity
        lines.append("(~(%s & %s) | %s)" % (p(i, j), p(j, k), p(i, k)))
    disj = []                                        # special element
    for i in S:
        conj = " & ".join("(%s | %s)" % (p(i, j), p(j, i)) for j in S)
        disj.append("(" + conj + ")")
    if disj:
        lines.append(" | ".join(disj))
    return "\n".join(lines) + "\n", len(idx)


def bounded_posets(n):
    """Partial orders on {0..n-1} with least element 0 and greatest n-1
    (Section 5.2), all letters p(i,j), i != j, written out; the letters the
    section kills are replaced by their constants:
    p(0,i) = 1, p(j,0) = 0 (j >= 1), p(i,n-1) = 1, p(n-1,k) = 0 (k <= n-2),
    p(i,i) = 1.  The free letters are p(i,j) for distinct i, j in 1..n-2, in
    lexicographic order: (n-2)(n-3) of them."""
    if n < 2:
        raise ValueError("n >= 2")
    top = n - 1
    inner = list(range(1, n - 1))
    idx = _pair_letters(inner)

    def p(i, j):
        if i == j:
            return "1"
        if i == 0:
            return "1"
        if j == 0:
            return "0"
        if j == top:
            return "1"
        if i == top:
            return "0"
        return "x%d" % idx[(i, j)]

    S = list(range(n))
    lines = []
    for i, j in permutations(S, 2):
        lines.append("(~%s | ~%s)" % (p(i, j), p(j, i)))
    for i, j, k in permutations(S, 3):
        lines.append("(~(%s & %s) | %s)" % (p(i, j), p(j, k), p(i, k)))
    if not lines:
        lines.append("1")
    return "\n".join(lines) + "\n", len(idx)
