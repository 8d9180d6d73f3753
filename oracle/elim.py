"""O-D: bucket (variable) elimination -- an exact count independent of the
paper's network.

The count is sum_x prod_c sat_c(x) (Eq. 2 at zero temperature). Writing each
clause as a factor over its distinct variables, the sum over one variable v
can be pushed inside the product: multiply every factor that mentions v,
sum the product over v in {0,1}, and put the result back as a factor over
the remaining variables of those factors. Eliminating all variables leaves
scalars whose product is the count. This is the textbook sum-product
(bucket elimination) algorithm; it uses no COPY tensors and no bonds, which
makes it an independent check of the tensor-network contraction.

Elimination order: minimum degree in the interaction graph (two variables
are adjacent when some factor mentions both), ties to the smaller variable.
Arithmetic: exact Python integers, or one pass per prime with CRT.
"""
from __future__ import annotations

import itertools
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import rns

OR = 0
EXACTLY_ONE = 1
XOR = 2

Factor = Tuple[np.ndarray, Tuple[int, ...]]


def clause_factor(kind: int, lits: Sequence[int], dtype=object) -> Factor:
    """Factor of one clause over its distinct variables, sorted ascending."""
    vs = tuple(sorted({abs(l) for l in lits}))
    t = np.zeros((2,) * len(vs), dtype=dtype) if vs else np.zeros((), dtype=dtype)
    for idx in itertools.product((0, 1), repeat=len(vs)):
        val = dict(zip(vs, idx))
        true = sum(1 for l in lits if (val[abs(l)] == 1) == (l > 0))
        ok = (true >= 1) if kind == OR else (true == 1) if kind == EXACTLY_ONE else (true % 2 == 1)
        t[idx] = 1 if ok else 0
    return t, vs


def _align(t: np.ndarray, vs: Tuple[int, ...], scope: Tuple[int, ...]) -> np.ndarray:
    """View factor t (over vs) as broadcastable over scope (ascending order)."""
    perm = sorted(range(len(vs)), key=lambda k: vs[k])
    t = np.transpose(t, perm) if len(vs) > 1 else t
    svs = sorted(vs)
    shape = [2 if v in svs else 1 for v in scope]
    return t.reshape(shape) if scope else t


def _product(factors: List[Factor], p: Optional[int]) -> Factor:
    scope = tuple(sorted(set().union(*[set(vs) for _, vs in factors])))
    acc = None
    for t, vs in factors:
        a = _align(t, vs, scope)
        if acc is None:
            acc = np.broadcast_to(a, (2,) * len(scope)).copy()
        else:
            acc = acc * a
            if p is not None:
                acc %= p
    return acc, scope


def min_degree_order(n: int, scopes: List[Tuple[int, ...]]) -> List[int]:
    adj = {v: set() for v in range(1, n + 1)}
    for vs in scopes:
        for a in vs:
            adj[a].update(x for x in vs if x != a)
    order = []
    alive = set(adj)
    while alive:
        v = min(alive, key=lambda x: (len(adj[x]), x))
        nb = adj[v]
        for a in nb:
            adj[a].discard(v)
            adj[a].update(x for x in nb if x != a)
        alive.discard(v)
        order.append(v)
    return order


def count(formula, p: Optional[int] = None, order: Optional[List[int]] = None) -> int:
    """Count satisfying assignments exactly (p None) or modulo p."""
    dtype = object if p is None else np.int64
    factors: List[Factor] = [clause_factor(k, l, dtype) for k, l in formula.clauses]
    if order is None:
        order = min_degree_order(formula.n_vars, [vs for _, vs in factors])
    for v in order:
        bucket = [f for f in factors if v in f[1]]
        if not bucket:
            # a variable in no clause: both of its values count
            factors.append((np.array(2, dtype=dtype), ()))
            continue
        factors = [f for f in factors if v not in f[1]]
        t, scope = _product(bucket, p)
        k = scope.index(v)
        s = t.take(0, axis=k) + t.take(1, axis=k)
        if p is not None:
            s %= p
        factors.append((s, tuple(x for x in scope if x != v)))
    total = 1
    for t, vs in factors:
        assert not vs
        total = total * int(t) if p is None else (total * int(t)) % p
    return total


def count_rns(formula, primes: Sequence[int] = None) -> int:
    if primes is None:
        primes = rns.primes_for(formula.n_vars)
    factors = [clause_factor(k, l, np.int64) for k, l in formula.clauses]
    order = min_degree_order(formula.n_vars, [vs for _, vs in factors])
    return rns.crt([count(formula, p, order) for p in primes], primes)


def width(formula) -> int:
    """Largest factor scope created by the min-degree order."""
    scopes = [clause_factor(k, l, np.int64)[1] for k, l in formula.clauses]
    order = min_degree_order(formula.n_vars, scopes)
    live = [set(s) for s in scopes]
    w = 0
    for v in order:
        b = [s for s in live if v in s]
        live = [s for s in live if v not in s]
        u = set().union(*b) if b else set()
        w = max(w, len(u))
        u.discard(v)
        live.append(u)
    return w
