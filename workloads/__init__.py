"""Seeded synthetic inputs for the free-Boolean-generator path.

This package only produces formula *text* (and request schedules) from a
seed.  It holds none of the method's arithmetic: no evaluation, no generator
vectors, no counting.  Both the oracle and the GPU path consume its output,
and nothing here imports either of them.

Formula text format (one formula per string):

* statements are separated by newlines or ``;``; ``#`` starts a comment;
* ``name = expr`` defines a temporary (an SSA node of a DAG);
* a bare ``expr`` is an assertion; the formula is the conjunction of all
  assertions (a system of Boolean equations phi_i = 1, Section 5.1);
* operators are the Python ones the paper's scripts use (Section 4.2):
  ``~`` (not), ``&`` (and), ``^`` (symmetric difference, the paper's ``+``),
  ``|`` (or), with Python precedence ``~`` > ``&`` > ``^`` > ``|``;
* atoms are ``0``, ``1``, variables ``x0 .. x{n-1}`` and temporaries.

Variable ``xk`` is bit ``k`` of the valuation index.
"""

from .splitmix import SplitMix64
from .formulas import (
    baequ4,
    equivalence_relations,
    equivalence_var,
    permutation_matrices,
    random_3cnf,
    random_dag,
    special_element_posets,
    bounded_posets,
    triangle_free,
    cnf_text,
)

__all__ = [
    "SplitMix64",
    "baequ4",
    "bounded_posets",
    "cnf_text",
    "equivalence_relations",
    "equivalence_var",
    "permutation_matrices",
    "random_3cnf",
    "random_dag",
    "special_element_posets",
    "triangle_free",
]
