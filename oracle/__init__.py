"""CPU oracle for exact #CSP counting -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import, call, link or run anything in this package. The
library's product path never routes through it: the oracle shares no code,
table or helper with the HIP path, and imports nothing from it. Inputs come
from the ``instances`` package, which holds only input generation.

Parts
-----
``brute``      O-A: the plain definition of the count (Eq. 2 at beta -> inf,
               with the clause semantics of Eq. 3, Eq. 6 and the negation
               rule of Sec. 2.1), enumerated over all 2^n assignments; numpy
               for small n and a plain C loop (``bruteforce.c``) up to n~34.
``tensors``    The tensors of Sec. 2.1 / 3.2 written out entry by entry:
               OR (Eq. 3), COPY (Eq. 4), exactly-one (Eq. 6), negated indices.
``contract``   O-B: the paper's method itself -- build the network, contract
               connected pairs in an order (the paper's tensor-greedy rule,
               Sec. 3.1.1) until one scalar is left (Sec. 2.1, Eq. 5 form),
               in exact integers or per prime with CRT.
``elim``       O-D: bucket (variable) elimination on the clause factors, a
               textbook exact sum-product algorithm independent of the
               paper's network, used for large instances.
``closed``     Closed forms (transfer matrices, Lucas numbers) used as pins.
``rns``        Prime selection and Chinese remaindering in Python integers.
``cost``       Symbolic replay of a contraction order: ranks, bytes, MACs.
``mlp``        float64 reference of the order-scoring MLP and its gradients.

Pinning: every function here is checked by ``tests/test_oracle_*.py``
against values that do not come from itself: the worked example of Eq. 5
(``tests/golden/eq5_worked_example.json``), closed forms checked by brute
force on small cases, invariants (empty formula 2^n, disjoint unions
multiply, the 1-in-3 <-> 5-clause CNF identity of Sec. 3.2) and brute force
on random small formulas. Planted-mistake tests mutate this package on the
CPU and check that a pin fails.
"""
