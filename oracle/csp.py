"""Weighted constraint networks with non-boolean domains: the oracle's count.

Test infrastructure only. The generalisation Sec. 4 names (non-boolean or
mixed domains, weighted #CSP) keeps the method of Sec. 2.1: a variable v with
domain size D_v is a COPY tensor of dimension D_v on every index (1 when all
indices hold the same value, the scalar D_v when it occurs nowhere), a
constraint is the tensor of its weights over its scope, and the full
contraction of the network is
    Z = sum over all assignments x of prod over constraints c of w_c(x|scope_c),
the partition function of Eq. 2 with the constraint tensors in place of
exp(-beta E). Two independent computations of Z are given:

``count_brute``     the sum written out over every assignment (exact ints);
``count_contract``  the pairwise contraction of the network in its native
                    dimensions (bonds of dimension D_v, no binary encoding),
                    along any valid order, exactly or modulo a prime.

A CSP (``instances.CSP``) lists per constraint a scope (1-based variables,
repeats allowed) and a flat table, row-major with the first scope variable
slowest.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence, Tuple

import numpy as np

from . import contract, rns


def _table(csp, scope, table, dtype=object) -> np.ndarray:
    shape = tuple(csp.domain[v - 1] for v in scope)
    t = np.array([int(x) for x in table], dtype=dtype)
    if len(t) != int(np.prod(shape, dtype=np.int64)):
        raise ValueError("table size does not match the scope's domains")
    return t.reshape(shape) if shape else t.reshape(())


def count_brute(csp) -> int:
    """Sum over every assignment of the product of the constraint weights."""
    tables = [(scope, _table(csp, scope, table)) for scope, table in csp.constraints]
    total = 0
    for x in itertools.product(*[range(d) for d in csp.domain]):
        prod = 1
        for scope, t in tables:
            prod *= int(t[tuple(x[v - 1] for v in scope)])
            if prod == 0:
                break
        total += prod
    return total


def network(csp, p: int = None) -> List[Tuple[np.ndarray, Tuple[int, ...]]]:
    """Tensors (array, labels) in native dimensions: constraints first get one
    label per scope position; then one COPY tensor per variable over the
    labels of its occurrences."""
    dtype = object if p is None else np.int64
    occ = [[] for _ in range(csp.n_vars)]
    tensors = []
    lab = 0
    for scope, table in csp.constraints:
        labels = []
        for v in scope:
            occ[v - 1].append(lab)
            labels.append(lab)
            lab += 1
        t = _table(csp, scope, table, dtype)
        if p is not None:
            t = t % p
        tensors.append((t, tuple(labels)))
    for v in range(csp.n_vars):
        d = csp.domain[v]
        k = len(occ[v])
        if k == 0:
            c = np.array(d if p is None else d % p, dtype=dtype)
        else:
            c = np.zeros((d,) * k, dtype=dtype)
            for x in range(d):
                c[(x,) * k] = 1
        tensors.append((c, tuple(occ[v])))
    return tensors


def count_contract(csp, order=None, p: int = None) -> int:
    """Pairwise contraction of the native network (exact, or modulo p)."""
    tensors = network(csp, p)
    if order is None:
        order = contract.greedy_order([ls for _, ls in tensors])
    rest = contract.contract_network(tensors, order, p)
    total = 1
    for t, ls in rest:
        if ls:
            raise ValueError("open bonds remain")
        total = total * int(t) if p is None else (total * int(t)) % p
    return total


def log2_bound(csp) -> float:
    """log2 of an upper bound of Z: prod of the domain sizes times the
    product of every constraint's largest weight (Z is a sum of at most
    prod D_v terms, each a product of weights)."""
    b = sum(np.log2(d) for d in csp.domain)
    for _, table in csp.constraints:
        mx = max((int(x) for x in table), default=0)
        b += np.log2(mx) if mx > 1 else 0.0
    return float(b)


def count_rns(csp, order=None) -> int:
    """Contraction per 31-bit prime, recombined by the Chinese remainder
    theorem over enough primes for the bound above."""
    bits = int(np.ceil(log2_bound(csp))) + 1
    primes = rns.primes_for(bits)
    if order is None:
        order = contract.greedy_order([ls for _, ls in network(csp, primes[0])])
    return rns.crt([count_contract(csp, order, p) for p in primes], primes)
