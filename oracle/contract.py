"""O-B: the paper's method as a plain, slow, pairwise tensor contractor.

The count of a formula is the full contraction (tensor trace, Eq. 2) of its
network (Sec. 2.1): COPY tensors on variables (Eq. 4), OR / exactly-one
tensors on clauses (Eq. 3, Eq. 6), one bond per literal occurrence.
Contracting two tensors sums over every index they share (all parallel
edges at once, Sec. 2.2) the product of their entries, as in the worked
example of Eq. 5; the result keeps the unshared indices. Repeating this on
connected pairs until no bond is left and multiplying the remaining scalars
gives the count. The order of pairs changes only the cost (Sec. 2.1).

Arithmetic is exact: numpy object arrays of Python integers, or -- for
large intermediates -- one pass per prime with entries reduced modulo the
prime and the count recovered by the Chinese remainder theorem.

Order: the paper's tensor-greedy rule (Sec. 3.1.1): among all pairs of
tensors that share at least one bond, contract the pair whose result has the
smallest rank; ties go to the pair with the smallest (first id, second id),
tensor ids being positions in the growing tensor list.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import rns
from .tensors import network_of_formula

Tensor = Tuple[np.ndarray, Tuple[int, ...]]


def _mod_tensordot(A: np.ndarray, B: np.ndarray, axes, p: int) -> np.ndarray:
    """tensordot of residue arrays modulo p, exact in int64.

    Entries are below p < 2^31. Both operands are split into 16-bit halves
    so every partial product is below 2^32 and every sum of at most 2^30 of
    them fits in int64; the four partial results are recombined mod p.
    """
    A = A.astype(np.int64)
    B = B.astype(np.int64)
    a0, a1 = A & 0xFFFF, A >> 16
    b0, b1 = B & 0xFFFF, B >> 16
    s00 = np.tensordot(a0, b0, axes=axes) % p
    s01 = np.tensordot(a0, b1, axes=axes) % p
    s10 = np.tensordot(a1, b0, axes=axes) % p
    s11 = np.tensordot(a1, b1, axes=axes) % p
    two16 = (1 << 16) % p
    two32 = (1 << 32) % p
    mid = (s01 + s10) % p
    return ((s11 * two32) % p + (mid * two16) % p + s00) % p


def contract_pair(A: Tensor, B: Tensor, p: Optional[int] = None) -> Tensor:
    """Sum over all shared labels of A*B; result labels: A's free, then B's free."""
    ta, la = A
    tb, lb = B
    shared = [l for l in la if l in lb]
    ia = [la.index(l) for l in shared]
    ib = [lb.index(l) for l in shared]
    free_a = tuple(l for l in la if l not in shared)
    free_b = tuple(l for l in lb if l not in shared)
    axes = (ia, ib)
    if p is None:
        if ta.ndim == 0 or tb.ndim == 0:
            out = np.multiply(ta, tb, dtype=object)
        else:
            out = np.tensordot(ta, tb, axes=axes)
    else:
        if ta.ndim == 0 or tb.ndim == 0:
            out = (np.asarray(ta, dtype=np.int64) * np.asarray(tb, dtype=np.int64)) % p
        else:
            out = _mod_tensordot(ta, tb, axes, p)
    return np.asarray(out), free_a + free_b


def greedy_order(label_sets: Sequence[Sequence[int]]) -> List[Tuple[int, int]]:
    """tensor-greedy order over a list of label sets (Sec. 3.1.1).

    Returns merges (i, j), i < j, of tensor ids; merge k creates tensor id
    len(label_sets) + k. Only pairs sharing a label are merged.
    """
    live: Dict[int, frozenset] = {i: frozenset(ls) for i, ls in enumerate(label_sets)}
    next_id = len(label_sets)
    order = []
    while True:
        best = None
        ids = sorted(live)
        owner: Dict[int, List[int]] = {}
        for i in ids:
            for l in live[i]:
                owner.setdefault(l, []).append(i)
        pairs = set()
        for l, ts in owner.items():
            if len(ts) == 2:
                pairs.add((min(ts), max(ts)))
        for i, j in pairs:
            r = len(live[i] ^ live[j])
            key = (r, i, j)
            if best is None or key < best:
                best = key
        if best is None:
            break
        _, i, j = best
        live[next_id] = live.pop(i) ^ live.pop(j)
        order.append((i, j))
        next_id += 1
    return order


def contract_network(tensors: List[Tensor], order=None, p: Optional[int] = None):
    """Contract a network along ``order`` (default: tensor-greedy).

    Labels that occur in one tensor only stay open. Returns the final list
    of tensors left after the merges (scalars and open tensors).
    """
    if order is None:
        order = greedy_order([ls for _, ls in tensors])
    work: Dict[int, Tensor] = dict(enumerate(tensors))
    nid = len(tensors)
    for i, j in order:
        work[nid] = contract_pair(work.pop(i), work.pop(j), p)
        nid += 1
    return [work[k] for k in sorted(work)]


def _close(remaining: List[Tensor], p: Optional[int]) -> int:
    """Multiply the scalars left after all bonds are contracted."""
    total = 1
    for t, ls in remaining:
        if ls:
            raise ValueError("open bonds remain in a closed network")
        total = total * int(t) if p is None else (total * int(t)) % p
    return total if p is None else total % p


def count_exact(formula, order=None) -> int:
    """Count with exact Python integers (fine while ranks stay below ~18)."""
    tensors, _ = network_of_formula(formula)
    return _close(contract_network(tensors, order), None)


def count_mod(formula, p: int, order=None) -> int:
    """Count modulo one prime p < 2^31."""
    tensors, _ = network_of_formula(formula)
    tensors = [(np.asarray(t, dtype=np.int64) % p, ls) for t, ls in tensors]
    return _close(contract_network(tensors, order, p), p)


def count_rns(formula, primes: Sequence[int] = None, order=None) -> int:
    """Count by one contraction per prime and CRT (Sec. 3.2 precision remark:
    residues give exactness at a cost linear in the number of primes)."""
    if primes is None:
        primes = rns.primes_for(formula.n_vars)
    if order is None:
        tensors, _ = network_of_formula(formula)
        order = greedy_order([ls for _, ls in tensors])
    res = [count_mod(formula, p, order) for p in primes]
    return rns.crt(res, primes)


def max_rank_of_order(label_sets, order) -> int:
    live = {i: frozenset(ls) for i, ls in enumerate(label_sets)}
    nid = len(label_sets)
    mr = max((len(s) for s in live.values()), default=0)
    for i, j in order:
        live[nid] = live.pop(i) ^ live.pop(j)
        mr = max(mr, len(live[nid]))
        nid += 1
    return mr


def step_entries(A, B, s: int, maskA: int, rC: int, cs, p: Optional[int] = None) -> List[int]:
    """Entries of one contraction step written out from its definition.

    Flat storage: entry index x of a tensor holds bit k of x for its k-th
    bond. A and B hold their s shared bonds as their low s bits, in the same
    order; output bit j of C comes from A's free bits when bit j of maskA is
    set and from B's free bits otherwise, each in increasing order. Then
        C[c] = sum over z < 2^s of A[z + 2^s xA] * B[z + 2^s xB]
    (Eq. 5 form, all shared bonds summed at once), in exact integers, reduced
    mod p when p is given, else mod 2^64 (the wrapping 64-bit mode).
    """
    out = []
    for c in cs:
        xa = xb = 0
        ka = kb = 0
        for j in range(rC):
            bit = (c >> j) & 1
            if (maskA >> j) & 1:
                xa |= bit << ka
                ka += 1
            else:
                xb |= bit << kb
                kb += 1
        acc = 0
        for z in range(1 << s):
            acc += int(A[z + (xa << s)]) * int(B[z + (xb << s)])
        out.append(acc % p if p is not None else acc % (1 << 64))
    return out
