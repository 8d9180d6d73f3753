"""The tensors of Sec. 2.1 and Sec. 3.2, written out entry by entry.

Every index is boolean (bond dimension 2). Arrays have shape (2,)*d with
index k of the array being index i_{k+1} of the paper's notation.

* COPY (Eq. 4): 1 when all indices are equal, else 0. For d = 0 the tensor
  stands for a variable that occurs in no clause; reading COPY as
  "sum over the variable's value x of prod_k [i_k = x]" (which is Eq. 4 for
  d >= 1) gives the scalar 2 for d = 0 and [1, 1] for d = 1.
* OR (Eq. 3): 0 when all (effective) indices are 0, else 1.
* exactly-one (Eq. 6): 1 when the (effective) indices sum to 1, else 0.
* parity (XOR, a clause type of Sec. 4): 1 when the (effective) indices sum
  to an odd number, else 0.
* A negated literal reverses the values of its index (Sec. 2.1): the
  effective index is 1 - i.
"""
from __future__ import annotations

import itertools

import numpy as np

OR = 0
EXACTLY_ONE = 1
XOR = 2


def copy_tensor(d: int) -> np.ndarray:
    """COPY tensor of rank d as exact Python integers."""
    if d == 0:
        return np.array(2, dtype=object)
    t = np.zeros((2,) * d, dtype=object)
    for x in (0, 1):
        t[(x,) * d] = 1
    return t


def clause_tensor(kind: int, negated) -> np.ndarray:
    """Clause tensor over len(negated) indices; negated[k] reverses index k."""
    d = len(negated)
    t = np.zeros((2,) * d, dtype=object) if d else np.array(0, dtype=object)
    for idx in itertools.product((0, 1), repeat=d):
        eff = [i ^ int(bool(neg)) for i, neg in zip(idx, negated)]
        if kind == OR:
            val = 0 if all(e == 0 for e in eff) else 1
        elif kind == EXACTLY_ONE:
            val = 1 if sum(eff) == 1 else 0
        elif kind == XOR:
            val = sum(eff) % 2
        else:
            raise ValueError(f"unknown clause kind {kind}")
        t[idx] = val
    return t


def network_of_formula(formula):
    """Tensor network of a formula (Sec. 2.1).

    One COPY tensor per variable with one index per occurrence, one clause
    tensor per clause with one index per literal, and one bond per literal
    occurrence joining the two. Returns ``(tensors, n_bonds)`` where
    ``tensors`` is a list of ``(array, labels)`` and every bond label
    0..n_bonds-1 appears in exactly two tensors. Variables come first
    (tensor v-1 for variable v), clauses after them.
    """
    n = formula.n_vars
    var_bonds = [[] for _ in range(n)]
    clause_tensors = []
    bond = 0
    for kind, lits in formula.clauses:
        labels = []
        neg = []
        for lit in lits:
            v = abs(lit)
            if v < 1 or v > n:
                raise ValueError(f"literal {lit} out of range")
            var_bonds[v - 1].append(bond)
            labels.append(bond)
            neg.append(lit < 0)
            bond += 1
        clause_tensors.append((clause_tensor(kind, neg), tuple(labels)))
    tensors = [(copy_tensor(len(b)), tuple(b)) for b in var_bonds]
    return tensors + clause_tensors, bond
