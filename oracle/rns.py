"""Residue arithmetic for the oracle: prime selection and Chinese remaindering.

Counts are non-negative integers at most 2^n (every term of the sum in Eq. 2
is 0 or 1 and there are 2^n assignments), so residues modulo primes whose
product exceeds 2^n determine the count uniquely (Chinese remainder theorem).
The oracle picks the k largest primes below 2^31 by trial division, with
k = ceil(n/31) + 1: each such prime exceeds 2^30, so their product exceeds
2^(30k) >= 2^n for every n >= 0.
"""
from __future__ import annotations

from typing import List, Sequence


def is_prime(q: int) -> bool:
    if q < 2:
        return False
    if q % 2 == 0:
        return q == 2
    f = 3
    while f * f <= q:
        if q % f == 0:
            return False
        f += 2
    return True


def largest_primes_below(limit: int, k: int) -> List[int]:
    out = []
    q = limit - 1
    while len(out) < k:
        if is_prime(q):
            out.append(q)
        q -= 1
    return out


def n_primes_for(n_vars: int) -> int:
    return (n_vars + 30) // 31 + 1


def primes_for(n_vars: int, k: int = None) -> List[int]:
    return largest_primes_below(1 << 31, n_primes_for(n_vars) if k is None else k)


def crt(residues: Sequence[int], primes: Sequence[int]) -> int:
    """The unique x in [0, prod(primes)) with x = residues[i] mod primes[i]."""
    M = 1
    for p in primes:
        M *= p
    x = 0
    for r, p in zip(residues, primes):
        Mi = M // p
        x += r * Mi * pow(Mi, -1, p)
    return x % M
