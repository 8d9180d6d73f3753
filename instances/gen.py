"""Pseudo-random numbers, graphs and formulas for the #CSP workloads.

Formulas follow the usual conjunctive layout: ``n_vars`` boolean variables
numbered 1..n and a list of clauses, each a clause kind plus a list of
DIMACS-style literals (+v for the variable, -v for its negation). Two clause
kinds are used, the OR clause of Eq. 3 and the exactly-one clause of Eq. 6
(Sec. 3.2; there monotone, here negation is allowed as in Sec. 2.1).

Workloads (Sec. 3.2):
* monotone 1-in-3 with clauses of three distinct variables drawn uniformly;
* vertex cover of a random 3-regular graph written as 2-variable OR clauses,
  one per edge, one variable per vertex (the #Cubic-Vertex-Cover encoding);
* 1-in-3 on a cubic graph with one variable per edge and one clause per
  vertex (the paper's own 1-in-3 family, every variable in two clauses).

Random cubic graphs come from the configuration model (3n stubs, uniform
perfect matching of stubs by a Fisher-Yates shuffle) with rejection of the
whole draw on a self-loop or a repeated edge, which samples simple cubic
graphs uniformly. The paper samples with the Viger-Latapy Markov chain
instead; both target the uniform distribution over simple cubic graphs.

Random numbers: SplitMix64 expands a 64-bit seed into the state of
xoshiro256** (Blackman and Vigna); bounded draws use rejection so they are
unbiased.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

OR = 0
EXACTLY_ONE = 1
XOR = 2

_M64 = (1 << 64) - 1


def _splitmix64_next(state: int) -> Tuple[int, int]:
    state = (state + 0x9E3779B97F4A7C15) & _M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return state, z ^ (z >> 31)


def instance_seed(family: int, index: int, master: int = 0) -> int:
    """64-bit seed of instance ``index`` of workload ``family``."""
    _, a = _splitmix64_next((master ^ (family << 40) ^ index) & _M64)
    return a


def _rotl(x: int, k: int) -> int:
    return ((x << k) | (x >> (64 - k))) & _M64


class Rng:
    """xoshiro256** seeded through SplitMix64."""

    def __init__(self, seed: int):
        st = seed & _M64
        s = []
        for _ in range(4):
            st, v = _splitmix64_next(st)
            s.append(v)
        self.s = s

    def next_u64(self) -> int:
        s0, s1, s2, s3 = self.s
        result = (_rotl((s1 * 5) & _M64, 7) * 9) & _M64
        t = (s1 << 17) & _M64
        s2 ^= s0
        s3 ^= s1
        s1 ^= s2
        s0 ^= s3
        s2 ^= t
        s3 = _rotl(s3, 45)
        self.s = [s0, s1, s2, s3]
        return result

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by rejection of the biased low range."""
        if n <= 0:
            raise ValueError("n must be positive")
        limit = (1 << 64) - ((1 << 64) % n)
        while True:
            x = self.next_u64()
            if x < limit:
                return x % n

    def uniform_int(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] inclusive."""
        return lo + self.below(hi - lo + 1)

    def coin(self) -> int:
        return self.next_u64() >> 63


@dataclass
class Formula:
    """A CNF-like formula: ``clauses[i] = (kind, [literals])``."""

    n_vars: int
    clauses: List[Tuple[int, List[int]]] = field(default_factory=list)
    name: str = ""

    @property
    def n_clauses(self) -> int:
        return len(self.clauses)

    def arrays(self):
        """(clause_ptr, lits, kinds) flat lists in the C-ABI layout."""
        ptr = [0]
        lits: List[int] = []
        kinds: List[int] = []
        for kind, cl in self.clauses:
            lits.extend(int(x) for x in cl)
            ptr.append(len(lits))
            kinds.append(int(kind))
        return ptr, lits, kinds

    def occurrences(self) -> List[int]:
        occ = [0] * (self.n_vars + 1)
        for _, cl in self.clauses:
            for lit in cl:
                occ[abs(lit)] += 1
        return occ[1:]


# --------------------------------------------------------------------------
# graphs (vertex labels 0..n-1, edge lists of (u, v) pairs)
# --------------------------------------------------------------------------

def cubic_graph(n: int, rng: Rng, max_tries: int = 100000) -> List[Tuple[int, int]]:
    """Uniform simple 3-regular graph on ``n`` (even) vertices."""
    if n % 2 or n < 4:
        raise ValueError("a cubic graph needs an even n >= 4")
    for _ in range(max_tries):
        stubs = [v for v in range(n) for _ in range(3)]
        for i in range(len(stubs) - 1, 0, -1):
            j = rng.below(i + 1)
            stubs[i], stubs[j] = stubs[j], stubs[i]
        edges = []
        seen = set()
        ok = True
        for i in range(0, len(stubs), 2):
            u, v = stubs[i], stubs[i + 1]
            if u == v:
                ok = False
                break
            key = (min(u, v), max(u, v))
            if key in seen:
                ok = False
                break
            seen.add(key)
            edges.append(key)
        if ok:
            return edges
    raise RuntimeError("configuration model did not produce a simple graph")


def cycle_graph(k: int) -> List[Tuple[int, int]]:
    return [(i, (i + 1) % k) for i in range(k)]


def complete_graph(k: int) -> List[Tuple[int, int]]:
    return [(i, j) for i in range(k) for j in range(i + 1, k)]


def complete_bipartite_graph(a: int, b: int) -> List[Tuple[int, int]]:
    return [(i, a + j) for i in range(a) for j in range(b)]


def prism_graph(k: int) -> List[Tuple[int, int]]:
    """C_k x K_2: two k-cycles (0..k-1 and k..2k-1) joined by rungs."""
    e = [(i, (i + 1) % k) for i in range(k)]
    e += [(k + i, k + (i + 1) % k) for i in range(k)]
    e += [(i, k + i) for i in range(k)]
    return e


def petersen_graph() -> List[Tuple[int, int]]:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, 5 + i) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return outer + spokes + inner


def cube_graph() -> List[Tuple[int, int]]:
    """The 3-cube Q3: vertices 0..7, edges between labels at Hamming distance 1."""
    return [(u, u ^ (1 << b)) for u in range(8) for b in range(3) if u < u ^ (1 << b)]


# --------------------------------------------------------------------------
# formulas
# --------------------------------------------------------------------------

def vertex_cover_formula(edges: Sequence[Tuple[int, int]], n_vertices: int = None,
                         name: str = "") -> Formula:
    """#Vertex-Cover as #2SAT: variable per vertex, OR clause per edge."""
    if n_vertices is None:
        n_vertices = 1 + max(max(u, v) for u, v in edges) if edges else 0
    f = Formula(n_vertices, name=name)
    for u, v in edges:
        f.clauses.append((OR, [u + 1, v + 1]))
    return f


def perfect_matching_formula(edges: Sequence[Tuple[int, int]], n_vertices: int = None,
                             name: str = "") -> Formula:
    """Exactly-one clause per vertex over the variables of its incident edges."""
    if n_vertices is None:
        n_vertices = 1 + max(max(u, v) for u, v in edges) if edges else 0
    inc: List[List[int]] = [[] for _ in range(n_vertices)]
    for i, (u, v) in enumerate(edges):
        inc[u].append(i + 1)
        inc[v].append(i + 1)
    f = Formula(len(edges), name=name)
    for v in range(n_vertices):
        f.clauses.append((EXACTLY_ONE, inc[v]))
    return f


def exactly_one_3(n: int, m: int, rng: Rng, name: str = "") -> Formula:
    """Monotone 1-in-3: m clauses, each 3 distinct variables drawn uniformly."""
    if n < 3 and m > 0:
        raise ValueError("need n >= 3")
    f = Formula(n, name=name)
    for _ in range(m):
        a = rng.below(n)
        b = rng.below(n)
        while b == a:
            b = rng.below(n)
        c = rng.below(n)
        while c == a or c == b:
            c = rng.below(n)
        f.clauses.append((EXACTLY_ONE, [a + 1, b + 1, c + 1]))
    return f


def cnf_of_exactly_one(f: Formula) -> Formula:
    """Rewrite every 3-literal exactly-one clause as the five OR clauses of Sec. 3.2.

    For literals (a, b, c) the clauses are (a|b|c), (a|~b|~c), (~a|~b|c),
    (~a|b|~c), (~a|~b|~c). Other clauses are kept as they are.
    """
    g = Formula(f.n_vars, name=(f.name + "-cnf") if f.name else "")
    for kind, cl in f.clauses:
        if kind == EXACTLY_ONE and len(cl) == 3:
            a, b, c = cl
            g.clauses += [(OR, [a, b, c]), (OR, [a, -b, -c]), (OR, [-a, -b, c]),
                          (OR, [-a, b, -c]), (OR, [-a, -b, -c])]
        else:
            g.clauses.append((kind, list(cl)))
    return g


def random_mixed_formula(n: int, m: int, rng: Rng, max_len: int = 4,
                         allow_repeats: bool = True, name: str = "") -> Formula:
    """Small mixed formulas for property tests: OR and exactly-one clauses of
    length 0..max_len with random negations; repeated and complementary
    literals inside a clause are allowed when ``allow_repeats``."""
    f = Formula(n, name=name)
    for _ in range(m):
        kind = rng.below(2)
        length = rng.below(max_len + 1)
        cl = []
        while len(cl) < length:
            v = rng.below(n) + 1
            if not allow_repeats and any(abs(x) == v for x in cl):
                continue
            cl.append(v if rng.coin() else -v)
        f.clauses.append((kind, cl))
    return f


def disjoint_union(a: Formula, b: Formula) -> Formula:
    """Formula on a.n_vars + b.n_vars variables; b's variables are shifted."""
    f = Formula(a.n_vars + b.n_vars, name=f"{a.name}+{b.name}")
    f.clauses = [(k, list(c)) for k, c in a.clauses]
    sh = a.n_vars
    for k, c in b.clauses:
        f.clauses.append((k, [x + sh if x > 0 else x - sh for x in c]))
    return f


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

FAMILY_SMALL_1IN3 = 0     # monotone 1-in-3, n=20, m=14
FAMILY_CVC = 1            # vertex cover of random cubic graphs
FAMILY_LARGE_1IN3 = 2     # monotone 1-in-3, n=150..300, alpha 0.62..0.70
FAMILY_BATCH = 3          # mixed batch, n in [30, 120]
FAMILY_LEARNED = 4        # training / held-out 1-in-3, n in [100, 250]
FAMILY_CUBIC_1IN3 = 5     # the paper's 1-in-3 family: one variable per edge of a cubic graph


def small_1in3(index: int) -> Formula:
    rng = Rng(instance_seed(FAMILY_SMALL_1IN3, index))
    return exactly_one_3(20, 14, rng, name=f"1in3-n20-m14-s{index}")


def cvc(n: int, index: int) -> Formula:
    rng = Rng(instance_seed(FAMILY_CVC, (n << 20) | index))
    return vertex_cover_formula(cubic_graph(n, rng), n, name=f"cvc-n{n}-s{index}")


def large_1in3(n: int, alpha: float, index: int) -> Formula:
    m = int(round(alpha * n))
    rng = Rng(instance_seed(FAMILY_LARGE_1IN3, (n << 24) | (int(round(alpha * 100)) << 16) | index))
    return exactly_one_3(n, m, rng, name=f"1in3-n{n}-a{alpha:.2f}-s{index}")


def batch_instance(index: int, master: int = 0) -> Formula:
    """Instance ``index`` of the mixed batch: even -> monotone 1-in-3 with
    n ~ U[30,120], m = round(0.66 n); odd -> vertex cover of a random cubic
    graph with n ~ U[30,120] rounded up to even."""
    rng = Rng(instance_seed(FAMILY_BATCH, index, master))
    n = rng.uniform_int(30, 120)
    if index % 2 == 0:
        return exactly_one_3(n, int(round(0.66 * n)), rng, name=f"batch{index}-1in3-n{n}")
    n += n % 2
    return vertex_cover_formula(cubic_graph(n, rng), n, name=f"batch{index}-cvc-n{n}")


def learned_instance(index: int, split: str = "train", n: int = None) -> Formula:
    """1-in-3 at alpha = 0.66 with n ~ U[100, 250] (or a fixed n)."""
    fam_index = index if split == "train" else (1 << 30) | index
    rng = Rng(instance_seed(FAMILY_LEARNED, fam_index))
    if n is None:
        n = rng.uniform_int(100, 250)
    return exactly_one_3(n, int(round(0.66 * n)), rng, name=f"learn-{split}{index}-n{n}")


def cubic_1in3(n_vertices: int, index: int) -> Formula:
    """The paper's 1-in-3 workload (Sec. 3.2): a uniform random cubic graph on
    ``n_vertices`` vertices, one variable per edge (3 n_vertices / 2 of them,
    each in exactly two clauses, clause density 2/3) and one exactly-one
    clause per vertex over its three edges."""
    rng = Rng(instance_seed(FAMILY_CUBIC_1IN3, (n_vertices << 20) | index))
    return perfect_matching_formula(cubic_graph(n_vertices, rng), n_vertices,
                                    name=f"cubic1in3-N{3 * n_vertices // 2}-s{index}")


# --------------------------------------------------------------------------
# other clause types and general weighted constraint networks (Sec. 4)
# --------------------------------------------------------------------------

def exactly_one_k(n: int, m: int, k: int, rng: Rng, name: str = "") -> Formula:
    """Monotone 1-in-k: m clauses, each k distinct variables drawn uniformly
    (a partial Fisher-Yates draw)."""
    if m > 0 and n < k:
        raise ValueError("need n >= k")
    f = Formula(n, name=name)
    for _ in range(m):
        pool = list(range(n))
        cl = []
        for j in range(k):
            t = j + rng.below(n - j)
            pool[j], pool[t] = pool[t], pool[j]
            cl.append(pool[j] + 1)
        f.clauses.append((EXACTLY_ONE, cl))
    return f


def xor_k(n: int, m: int, k: int, rng: Rng, name: str = "") -> Formula:
    """Random k-XORSAT: m parity clauses over k distinct uniform variables,
    each literal negated with probability 1/2 (a random right-hand side)."""
    f = exactly_one_k(n, m, k, rng, name=name)
    f.clauses = [(XOR, [v if rng.coin() else -v for v in cl]) for _, cl in f.clauses]
    return f


@dataclass
class CSP:
    """A weighted constraint network: variable v (1-based) takes values
    0..domain[v-1]-1; constraint c has a scope (variables, repeats allowed)
    and a table of non-negative integer weights over the scope's values,
    row-major with the first scope variable slowest. The count is the sum over
    all assignments of the product of the constraints' weights."""

    n_vars: int
    domain: List[int]
    constraints: List[Tuple[Tuple[int, ...], List[int]]] = field(default_factory=list)
    name: str = ""

    def arrays(self):
        """(domain, scope_ptr, scope, table_ptr, weights) in the C-ABI layout."""
        sp, sc, tp, w = [0], [], [0], []
        for scope, table in self.constraints:
            sc.extend(int(v) for v in scope)
            sp.append(len(sc))
            w.extend(int(x) for x in table)
            tp.append(len(w))
        return list(self.domain), sp, sc, tp, w


def coloring_csp(edges: Sequence[Tuple[int, int]], n: int, q: int, name: str = "") -> CSP:
    """Proper q-colourings of a graph: domain q, one 'differ' table per edge."""
    table = [1 if a != b else 0 for a in range(q) for b in range(q)]
    return CSP(n, [q] * n, [((u + 1, v + 1), list(table)) for u, v in edges], name=name)


def hardcore_csp(edges: Sequence[Tuple[int, int]], n: int, lam: int, name: str = "") -> CSP:
    """Independent sets weighted by lam^size: a unary table [1, lam] per vertex
    and a 'not both' table per edge."""
    cons = [((v + 1,), [1, lam]) for v in range(n)]
    cons += [((u + 1, v + 1), [1, 1, 1, 0]) for u, v in edges]
    return CSP(n, [2] * n, cons, name=name)


def random_csp(n: int, m: int, rng: Rng, max_domain: int = 5, max_arity: int = 3, max_weight: int = 3,
               zero_prob: float = 0.3, name: str = "") -> CSP:
    """Mixed domains 1..max_domain, constraints of arity 0..max_arity over
    uniform variables (repeats allowed), weights uniform in 1..max_weight or
    0 with probability about zero_prob."""
    dom = [1 + rng.below(max_domain) for _ in range(n)]
    cons = []
    zero_thresh = int(zero_prob * 1000)
    for _ in range(m):
        ar = rng.below(max_arity + 1)
        scope = tuple(1 + rng.below(n) for _ in range(ar))
        size = 1
        for v in scope:
            size *= dom[v - 1]
        table = [0 if rng.below(1000) < zero_thresh else 1 + rng.below(max_weight) for _ in range(size)]
        cons.append((scope, table))
    return CSP(n, dom, cons, name=name)


def table_csp(formula: Formula) -> CSP:
    """The boolean CSP of a formula: one 0/1 truth table per clause over its
    literal occurrences' variables (OR, exactly-one and parity rules,
    negation reversing a value)."""
    import itertools
    cons = []
    for kind, lits in formula.clauses:
        scope = tuple(abs(l) for l in lits)
        table = []
        for vals in itertools.product((0, 1), repeat=len(lits)):
            t = sum(1 for l, x in zip(lits, vals) if (x == 1) == (l > 0))
            ok = t >= 1 if kind == OR else t == 1 if kind == EXACTLY_ONE else t % 2 == 1
            table.append(1 if ok else 0)
        cons.append((scope, table))
    return CSP(formula.n_vars, [2] * formula.n_vars, cons, name=formula.name + "-table")


def planar_cubic_graph(n: int, rng: Rng, flips_per_vertex: int = 10) -> List[Tuple[int, int]]:
    """A random simple planar cubic graph on n (even, >= 4) vertices: the dual
    of a random triangulation of the sphere with n/2 + 2 vertices (2V - 4 = n
    triangles). The triangulation starts from K4, grows by inserting a vertex
    into a uniformly chosen triangle, then is mixed by random edge flips that
    keep it simple and every degree at least 3. Vertices of the result are the
    triangles; two are adjacent when they share an edge."""
    if n % 2 or n < 4:
        raise ValueError("need an even n >= 4")
    V = n // 2 + 2
    faces = [[0, 1, 2], [0, 2, 3], [0, 3, 1], [1, 3, 2]]  # consistently oriented
    for v in range(4, V):
        f = faces.pop(rng.below(len(faces)))
        a, b, c = f
        faces += [[a, b, v], [b, c, v], [c, a, v]]

    def edge_map():
        em = {}
        for i, (a, b, c) in enumerate(faces):
            for x, y in ((a, b), (b, c), (c, a)):
                em[(x, y)] = i
        return em

    deg = [0] * V
    for a, b, c in faces:
        for x in (a, b, c):
            deg[x] += 1
    for _ in range(flips_per_vertex * V):
        em = edge_map()
        i = rng.below(len(faces))
        k = rng.below(3)
        a, b = faces[i][k], faces[i][(k + 1) % 3]
        c = faces[i][(k + 2) % 3]
        j = em[(b, a)]
        d = [x for x in faces[j] if x != a and x != b][0]
        if c == d or (c, d) in em or (d, c) in em or deg[a] <= 3 or deg[b] <= 3:
            continue
        # (a, b, c) and (b, a, d) become (c, a, d) and (d, b, c)
        faces[i] = [c, a, d]
        faces[j] = [d, b, c]
        deg[a] -= 1
        deg[b] -= 1
        deg[c] += 1
        deg[d] += 1
    em = edge_map()
    edges = set()
    for (x, y), i in em.items():
        j = em[(y, x)]
        edges.add((min(i, j), max(i, j)))
    return sorted(edges)
