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
    """tensordot of residue arrays modulo p < 2^31, exact.

    Both operands are split into 16-bit halves, a = a0 + 2^16 a1. A product of
    two halves is below 2^32 and a sum of at most 2^21 such products is below
    2^53, so each of the four half-products over a chunk of at most 2^21
    shared entries is an exact float64 matrix product (numpy's BLAS; the
    summation order does not matter for exact integers). The half-products
    are recombined modulo p in int64,
        A.B = s00 + 2^16 (s01 + s10) + 2^32 s11   (mod p),
    and the chunks are added modulo p. The result has A's free axes, then
    B's, as numpy's tensordot.
    """
    ia, ib = list(axes[0]), list(axes[1])
    fa = [d for d in range(A.ndim) if d not in ia]
    fb = [d for d in range(B.ndim) if d not in ib]
    out_shape = tuple(A.shape[d] for d in fa) + tuple(B.shape[d] for d in fb)
    K = 1
    for d in ia:
        K *= A.shape[d]
    A2 = np.transpose(np.asarray(A, dtype=np.int64), fa + ia).reshape(-1, K)
    B2 = np.transpose(np.asarray(B, dtype=np.int64), ib + fb).reshape(K, -1)
    chunk = 1 << 21
    acc = None
    for k0 in range(0, K, chunk):
        a, b = A2[:, k0:k0 + chunk], B2[k0:k0 + chunk, :]
        a0, a1 = (a & 0xFFFF).astype(np.float64), (a >> 16).astype(np.float64)
        b0, b1 = (b & 0xFFFF).astype(np.float64), (b >> 16).astype(np.float64)

        def part(x, y):
            t = x @ y
            np.fmod(t, p, out=t)
            return t.astype(np.int64)

        r = part(a1, b1)
        r *= (1 << 32) % p          # < 2^62
        r %= p
        mid = part(a0, b1)
        mid += part(a1, b0)         # < 2p
        mid %= p
        mid *= (1 << 16) % p        # < 2^47
        r += mid
        del mid
        r += part(a0, b0)
        r %= p
        if acc is None:
            acc = r
        else:
            acc += r
            acc %= p
    return acc.reshape(out_shape)


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
