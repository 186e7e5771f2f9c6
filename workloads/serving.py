"""Seeded request streams for the serving loop: Poisson arrivals and a mix of
model-counting requests.  Formula text and arrival times only."""

from .formulas import cnf_clause_count, equivalence_relations, permutation_matrices, random_3cnf, triangle_free
from .splitmix import SplitMix64

THEORIES = ("equivalence_k9", "permutations_k5", "triangle_free_k8")


def theory(name):
    if name == "equivalence_k9":
        return equivalence_relations(9)
    if name == "permutations_k5":
        return permutation_matrices(5)
    if name == "triangle_free_k8":
        return triangle_free(8)
    raise ValueError(name)


def request_stream(count, qps, seed=0, n_lo=12, n_hi=36, theory_share=0.10):
    """``count`` requests.  Per request, from one SplitMix64 stream: the gap to
    the previous arrival (exponential with rate qps; qps = 0 puts every
    arrival at time 0), then the kind (a theory with probability
    theory_share, the three theories in rotation; otherwise a random 3-CNF
    with n uniform in [n_lo, n_hi], m = floor(4.25 n + 1/2) clauses and its
    own 64-bit seed).  Returns dicts with id, arrival (seconds), kind, text,
    n."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    th = 0
    cache = {}
    for i in range(count):
        if qps > 0:
            t += rng.exponential(qps)
        if rng.unit() < theory_share:
            name = THEORIES[th % len(THEORIES)]
            th += 1
            if name not in cache:
                cache[name] = theory(name)
            text, n = cache[name]
            kind = name
        else:
            n = rng.uniform_int(n_lo, n_hi)
            fseed = rng.next()
            text, n = random_3cnf(n, cnf_clause_count(n), fseed)
            kind = "3cnf"
        out.append({"id": i, "arrival": t, "kind": kind, "text": text, "n": n})
    return out
