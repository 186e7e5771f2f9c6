"""Front end for TBA-style scripts (Section 4.2, "Python-AE"): predicate
formulas over finite domains with bounded quantifiers, translated to
propositional formula text for fbg_compile (the translation * of Section 3.1:
quantifiers over a finite domain become finite conjunctions and disjunctions,
atomic formulas become propositional letters).

A script is Python with two additions:

* bounded quantifiers ``A[i,j:S2] (body)`` (for all (i, j) in S2) and
  ``E[i:S] (body)`` (for some i in S), chained with a dot:
  ``E[i:S].A[j:S] (body)``; the body is a parenthesised Boolean expression;
* ``perm(seq, k)``: the k-tuples of distinct elements of seq.

Relation letters are called like functions, ``p(i, j)``; every name that is
called but not defined by the script is a relation symbol.  ``~ & | ^`` are
not, and, or, and symmetric difference.  Every top-level variable whose value
is a formula is an axiom; the theory is their conjunction.  A dictionary named
``assumptions`` maps letters to 0/1 and kills them (Section 3.3): they are
replaced by constants, which the compiler folds away (the paper's Reduction).

The free letters are numbered in the order (relation name, arguments) sorted;
variable xk of the compiled formula is the k-th free letter.
"""

import itertools
import re

_QUANT = re.compile(r"\b([AE])\[([^\]:]+):([^\]]+)\]\s*(\.)?")


class Term:
    """A propositional term built by the script: a letter, a constant, or an
    operator over terms.  Text is produced on demand."""

    __slots__ = ("op", "args")

    def __init__(self, op, args):
        self.op = op
        self.args = args

    def __invert__(self):
        return _not(self)

    def __and__(self, o):
        return _bin("&", self, o)

    def __rand__(self, o):
        return _bin("&", o, self)

    def __or__(self, o):
        return _bin("|", self, o)

    def __ror__(self, o):
        return _bin("|", o, self)

    def __xor__(self, o):
        return _bin("^", self, o)

    def __rxor__(self, o):
        return _bin("^", o, self)

    def __bool__(self):
        raise TypeError("a formula has no truth value before it is evaluated; "
                        "use ~ & | ^ rather than not/and/or")

    def __hash__(self):
        return hash((self.op, self.args))

    def __eq__(self, o):
        return isinstance(o, Term) and self.op == o.op and self.args == o.args


def _const(v):
    return Term("const", (1 if v else 0,))


def _lift(x):
    if isinstance(x, Term):
        return x
    if x in (0, 1, True, False):
        return _const(x)
    raise TypeError("not a formula: %r" % (x,))


def _not(t):
    t = _lift(t)
    if t.op == "const":
        return _const(1 - t.args[0])
    return Term("~", (t,))


def _bin(op, a, b):
    return Term(op, (_lift(a), _lift(b)))


class Letter(Term):
    """The atomic formula R(a1..ak) over the domain: a propositional letter."""

    __slots__ = ()

    def __init__(self, rel, args):
        Term.__init__(self, "letter", (rel, tuple(args)))


class Relation:
    def __init__(self, name):
        self.name = name

    def __call__(self, *args):
        return Letter(self.name, args)


def perm(seq, k):
    """k-tuples of distinct elements of seq (the paper's perm(range(n), k))."""
    return list(itertools.permutations(list(seq), k))


def _forall(domain, body):
    acc = None
    for elem in domain:
        t = body(*elem) if isinstance(elem, tuple) else body(elem)
        acc = _lift(t) if acc is None else _bin("&", acc, t)
    return _const(1) if acc is None else acc


def _exists(domain, body):
    acc = None
    for elem in domain:
        t = body(*elem) if isinstance(elem, tuple) else body(elem)
        acc = _lift(t) if acc is None else _bin("|", acc, t)
    return _const(0) if acc is None else acc


def _rewrite_quantifiers(src):
    """A[vars:D] (body)  ->  _forall(D, lambda vars: (body)), chains included.
    The body is the parenthesised expression that follows the last
    quantifier of a chain."""
    out = []
    pos = 0
    while True:
        m = _QUANT.search(src, pos)
        if not m:
            out.append(src[pos:])
            return "".join(out)
        out.append(src[pos:m.start()])
        chain = []
        while m:
            chain.append((m.group(1), m.group(2).strip(), m.group(3).strip()))
            pos = m.end()
            if not m.group(4):
                break
            m = _QUANT.match(src, pos)
        # the body: a balanced parenthesised expression
        while pos < len(src) and src[pos] in " \t":
            pos += 1
        if pos >= len(src) or src[pos] != "(":
            raise SyntaxError("a quantifier must be followed by a parenthesised formula")
        depth = 0
        end = pos
        while end < len(src):
            if src[end] == "(":
                depth += 1
            elif src[end] == ")":
                depth -= 1
                if depth == 0:
                    break
            end += 1
        if depth != 0:
            raise SyntaxError("unbalanced parentheses in a quantified formula")
        body = _rewrite_quantifiers(src[pos:end + 1])
        expr = body
        for kind, vars_, dom in reversed(chain):
            fn = "_forall" if kind == "A" else "_exists"
            expr = "%s(%s, lambda %s: %s)" % (fn, dom, vars_, expr)
        out.append(expr)
        pos = end + 1


class _Env(dict):
    """Script globals: unknown names that are called become relations."""

    def __missing__(self, key):
        if key.startswith("__"):
            raise KeyError(key)
        r = Relation(key)
        self[key] = r
        return r


def _letters(t, acc):
    stack = [t]
    seen = set()
    while stack:
        u = stack.pop()
        if id(u) in seen:
            continue
        seen.add(id(u))
        if u.op == "letter":
            acc.add(u.args)
        elif u.op != "const":
            stack.extend(u.args)


def _text(t, index, killed):
    """Formula text with letters as x<k> and killed letters as constants."""
    memo = {}

    def rec(u):
        key = id(u)
        if key in memo:
            return memo[key]
        if u.op == "const":
            s = str(u.args[0])
        elif u.op == "letter":
            s = str(killed[u.args]) if u.args in killed else "x%d" % index[u.args]
        elif u.op == "~":
            s = "~(%s)" % rec(u.args[0])
        else:
            s = "(%s %s %s)" % (rec(u.args[0]), u.op, rec(u.args[1]))
        memo[key] = s
        return s

    import sys
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 100000))
    try:
        return rec(t)
    finally:
        sys.setrecursionlimit(old)


class Translation:
    """The propositional form of a script: `text` and `n` for fbg_compile,
    `letters[k]` = (relation, args) of variable xk, `killed` = the letters
    fixed by the assumptions, `axioms` = names of the conjoined formulas."""

    def __init__(self, text, n, letters, killed, axioms):
        self.text = text
        self.n = n
        self.letters = letters
        self.killed = killed
        self.axioms = axioms

    def decode(self, model):
        """The letters that are true in a model (a valuation index)."""
        true = [self.letters[k] for k in range(self.n) if (int(model) >> k) & 1]
        true += [l for l, v in self.killed.items() if v]
        return sorted(true)


def translate(script, env=None):
    """Execute a TBA-style script and return its Translation."""
    g = _Env()
    g.update({"A": None, "E": None, "perm": perm, "range": range, "_forall": _forall, "_exists": _exists})
    if env:
        g.update(env)
    code = _rewrite_quantifiers(script)
    exec(compile(code, "<script>", "exec"), g)
    axioms = [k for k, v in g.items() if isinstance(v, Term) and not k.startswith("_")]
    if not axioms:
        raise ValueError("the script defines no formula")
    assumptions = g.get("assumptions", {}) or {}
    killed = {}
    for k, v in assumptions.items():
        if not isinstance(k, Letter) or v not in (0, 1, True, False):
            raise ValueError("assumptions map letters to 0 or 1")
        killed[k.args] = 1 if v else 0
    letters = set()
    for name in axioms:
        _letters(g[name], letters)
    free = sorted(l for l in letters if l not in killed)
    index = {l: k for k, l in enumerate(free)}
    text = "\n".join(_text(g[name], index, killed) for name in axioms) + "\n"
    return Translation(text, len(free), free, killed, axioms)


SO_SCRIPT = """n= {n}
S= range(n)
S2= perm(range(n),2)
S3= perm(range(n),3)
f1= A[i,j:S2] (~p(i,j) | ~p(j,i))
f2= A[i,j,k:S3] (~(p(i,j)& p(j,k)) | p(i,k))
f3= E[i:S].A[j:S] (p(i,j) | p(j,i))
assumptions= {{p(i,i): 1 for i in S}}
"""


def so_script(n):
    """The paper's example script SO.txt (Section 4.2) for domain size n."""
    return SO_SCRIPT.format(n=n)
