"""Closed forms used as pins (derived here, not printed in the paper).

Each closed form is itself checked against brute force on small sizes in
the oracle tests before it is used to check anything at full size.

* Vertex covers of the cycle C_k: walking round the cycle, a vertex may be
  left out only when both neighbours are in, giving the Lucas numbers
  L_1 = 1, L_2 = 3, L_k = L_{k-1} + L_{k-2} (k >= 3).
* Vertex covers of K_{a,b}: the complement of a vertex cover is an
  independent set, and the independent sets of K_{a,b} are the subsets of
  one side (the empty set lying in both), giving 2^a + 2^b - 1.
* Vertex covers of the prism C_k x K_2: transfer matrix over the state of a
  rung (u_i, v_i) in {(1,1), (1,0), (0,1)} (the rung edge forces at least
  one endpoint); consecutive rungs may not both leave out the top or both
  leave out the bottom vertex. The count is the trace of T^k.
* Perfect matchings of the prism, which are the solutions of 1-in-3 with
  one variable per edge and one exactly-one clause per vertex (Sec. 3.2):
  transfer matrix over (top edge, bottom edge) used between rungs i, i+1;
  the rung edge r_i must satisfy t_{i-1} + t_i + r_i = 1 and
  b_{i-1} + b_i + r_i = 1 with r_i in {0, 1}.
* A formula of m disjoint monotone 1-in-3 clauses on n variables has
  3^m 2^(n-3m) solutions; disjoint formulas multiply.
"""
from __future__ import annotations

import numpy as np


def _mat_pow_trace(T, k: int) -> int:
    M = np.array(T, dtype=object)
    R = np.identity(M.shape[0], dtype=object)
    for _ in range(k):
        R = R.dot(M)
    return int(np.trace(R))


def lucas(k: int) -> int:
    a, b = 1, 3
    if k == 1:
        return a
    for _ in range(k - 2):
        a, b = b, a + b
    return b


def cycle_vertex_covers(k: int) -> int:
    return lucas(k)


def complete_bipartite_vertex_covers(a: int, b: int) -> int:
    return 2 ** a + 2 ** b - 1


def prism_vertex_covers(k: int) -> int:
    states = [(1, 1), (1, 0), (0, 1)]
    T = [[1 if (s[0] | t[0]) and (s[1] | t[1]) else 0 for t in states] for s in states]
    return _mat_pow_trace(T, k)


def prism_perfect_matchings(k: int) -> int:
    states = [(0, 0), (0, 1), (1, 0), (1, 1)]
    T = []
    for (tp, bp) in states:
        row = []
        for (t, b) in states:
            row.append(sum(1 for r in (0, 1) if tp + t + r == 1 and bp + b + r == 1))
        T.append(row)
    return _mat_pow_trace(T, k)


def disjoint_1in3(n: int, m: int) -> int:
    return 3 ** m * 2 ** (n - 3 * m)


# ----------------------------------------------- other constraint networks
def chromatic_cycle(n: int, q: int) -> int:
    """Proper q-colourings of the cycle C_n: (q-1)^n + (-1)^n (q-1)."""
    return (q - 1) ** n + (-1) ** n * (q - 1)


def chromatic_complete(n: int, q: int) -> int:
    """Proper q-colourings of K_n: q (q-1) ... (q-n+1)."""
    out = 1
    for i in range(n):
        out *= q - i
    return out


def hardcore_cycle(n: int, lam: int) -> int:
    """Independent sets of C_n weighted by lam^size: the trace of T^n with the
    transfer matrix T[s][t] = lam^t unless both sites are occupied."""
    T = [[1, lam], [1, 0]]
    M = [[1, 0], [0, 1]]
    for _ in range(n):
        M = [[sum(M[i][k] * T[k][j] for k in range(2)) for j in range(2)] for i in range(2)]
    return M[0][0] + M[1][1]


def xorsat_count(formula) -> int:
    """Solutions of a system of parity clauses (an odd number of true
    literals each): 2^(n - rank) over GF(2) when consistent, else 0. A negated
    literal adds 1 to its clause's right-hand side."""
    piv = []
    rank = 0
    for _, lits in formula.clauses:
        mask, rhs = 0, 1
        for l in lits:
            mask ^= 1 << (abs(l) - 1)
            if l < 0:
                rhs ^= 1
        for pm, pr in piv:
            if mask & (pm & -pm):
                mask ^= pm
                rhs ^= pr
        if mask:
            piv.append((mask, rhs))
            rank += 1
        elif rhs:
            return 0
    return 2 ** (formula.n_vars - rank)
