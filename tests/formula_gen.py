"""Random formula text for tests (Python syntax, the library's format)."""


def random_expr(rng, n, names, depth):
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


def random_program(rng, n, max_defs=6, max_asserts=3, depth=4):
    """(statements, text): statements are (kind, name, expr) with kind
    'def' or 'assert'."""
    stmts = []
    names = []
    for t in range(rng.randrange(0, max_defs)):
        name = "t%d" % t
        stmts.append(("def", name, random_expr(rng, n, names, depth)))
        names.append(name)
    for _ in range(rng.randrange(1, max_asserts + 1)):
        stmts.append(("assert", None, random_expr(rng, n, names, depth)))
    text = "\n".join(("%s = %s" % (nm, tx)) if k == "def" else tx for k, nm, tx in stmts) + "\n"
    return stmts, text


def random_cnf(rng, n, m, width=(1, 5)):
    lines = []
    for _ in range(m):
        w = rng.randint(*width)
        lits = []
        for _ in range(w):
            k = rng.randrange(n)
            lits.append(("~x%d" % k) if rng.random() < 0.5 else ("x%d" % k))
        lines.append(" | ".join(lits))
    return "\n".join(lines) + "\n"


def many_registers(rng, n, k):
    """k shared subterms that are all live at once: each is used once in an
    OR over all of them and again in an XOR over all of them, so the
    compiled program needs about k registers."""
    lines = []
    for i in range(k):
        a, b, c, d = rng.sample(range(n), 4)
        ops = rng.choice([("&", "^", "|"), ("|", "&", "^"), ("^", "|", "&")])
        lines.append("t%d = (x%d %s x%d) %s (x%d %s ~x%d)" % (i, a, ops[0], b, ops[1], c, ops[2], d))
    names = ["t%d" % i for i in range(k)]
    rng.shuffle(names)
    lines.append("(%s) | ~(%s)" % (" | ".join(names), " ^ ".join(reversed(names))))
    return "\n".join(lines) + "\n"
