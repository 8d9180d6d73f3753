"""Seeded synthetic #CSP instances (formulas and graphs).

This package holds only input generation: pseudo-random numbers, random
graphs and the formulas built from them. It performs none of the counting
method's arithmetic and imports nothing from the HIP path or the oracle, so
both the oracle and the library binding can draw identical inputs from it.
"""
from .gen import (  # noqa: F401
    Formula,
    Rng,
    instance_seed,
    exactly_one_3,
    cubic_graph,
    vertex_cover_formula,
    perfect_matching_formula,
    cnf_of_exactly_one,
    random_mixed_formula,
    disjoint_union,
    cycle_graph,
    complete_graph,
    complete_bipartite_graph,
    prism_graph,
    petersen_graph,
    cube_graph,
    batch_instance,
    small_1in3,
    cvc,
    large_1in3,
    learned_instance,
    cubic_1in3,
    planar_cubic_graph,
    FAMILY_SMALL_1IN3,
    FAMILY_CVC,
    FAMILY_LARGE_1IN3,
    FAMILY_BATCH,
    FAMILY_LEARNED,
    FAMILY_CUBIC_1IN3,
    OR,
    EXACTLY_ONE,
    XOR,
    exactly_one_k,
    xor_k,
    CSP,
    coloring_csp,
    hardcore_csp,
    random_csp,
    table_csp,
)
