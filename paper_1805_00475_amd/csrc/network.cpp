// Formula -> tensor network (Sec. 2.1): a COPY tensor per variable (Eq. 4),
// a clause tensor per clause (OR, Eq. 3; exactly-one, Eq. 6; parity), and one
// bond per literal occurrence joining the variable's COPY tensor to the
// clause. Weighted constraint networks over any domains (the generalisation
// of Sec. 4) are encoded in the same boolean bonds: a variable of D values
// takes ceil(log2 D) bonds per occurrence, and codes of D or more get weight
// 0 in every tensor that reads them. Optional degree reduction (Sec. 4):
// COPY tensors of rank above 3 become rings of rank-3 COPY tensors, and
// OR / exactly-one / parity clauses of more than 3 literals become chains of
// rank-3 tensors linked by bonds that carry the clause's running state.
#include <algorithm>
#include <cmath>
#include <new>

#include "internal.hpp"

namespace tn {

namespace {

int bits_of(int32_t d) {
    int b = 0;
    while ((int64_t(1) << b) < d) ++b;
    return b;
}

int32_t new_bond(Network& net, int32_t a, int32_t b) {
    net.bond_end.push_back({a, b});
    return int32_t(net.bond_end.size()) - 1;
}

// Bond k of tensor t moved to tensor u (degree reduction keeps every
// original bond and re-homes it).
void rehome(Network& net, int32_t bond, int32_t from, int32_t to) {
    auto& e = net.bond_end[size_t(bond)];
    if (e[0] == from) e[0] = to;
    else if (e[1] == from) e[1] = to;
}

// COPY of rank d > 3 -> ring R_0..R_{d-1}: R_i holds original bond i and
// ring bonds r_{i-1}, r_i (indices mod d); every R_i is a rank-3 COPY, so the
// ring forces one value on all of them. R_0 keeps the original slot.
void ring_copy(Network& net, int32_t t) {
    const std::vector<int32_t> bonds = net.t[size_t(t)].bonds;
    const int d = int(bonds.size());
    std::vector<int32_t> ids(static_cast<size_t>(d));
    ids[0] = t;
    for (int i = 1; i < d; ++i) {
        ids[size_t(i)] = int32_t(net.t.size());
        net.t.push_back(InitTensor{});
        rehome(net, bonds[size_t(i)], t, ids[size_t(i)]);
    }
    std::vector<int32_t> ring(static_cast<size_t>(d));
    for (int i = 0; i < d; ++i) ring[size_t(i)] = new_bond(net, ids[size_t(i)], ids[size_t((i + 1) % d)]);
    for (int i = 0; i < d; ++i) {
        InitTensor r;
        r.kind = T_COPY;
        r.bonds = {bonds[size_t(i)], ring[size_t((i + d - 1) % d)], ring[size_t(i)]};
        net.t[size_t(ids[size_t(i)])] = r;
    }
}

// Clause of k > 3 literals (t_j = value of bond j, reversed when negated) ->
// chain P_1 (t_1, t_2, a_1), P_i (a_{i-1}, t_{i+1}, a_i), P_{k-2}
// (a_{k-3}, t_{k-1}, t_k) where a_i is the running state after i + 1
// literals: "some literal true" (OR), "number true, at most one"
// (exactly-one), parity (XOR). Every piece is a rank-3 table; the a_i are
// functions of the literals, so the count does not change.
void chain_clause(Network& net, int32_t t) {
    const InitTensor c = net.t[size_t(t)];
    const int k = int(c.bonds.size());
    auto lit = [&](int j, int v) { return v ^ int((c.neg >> j) & 1); };
    auto step = [&](int a, int x, int* out) -> bool {  // running state after one more literal
        if (c.kind == T_OR) { *out = a | x; return true; }
        if (c.kind == T_XOR) { *out = a ^ x; return true; }
        *out = a + x;
        return *out <= 1;
    };
    auto final_ok = [](int a) { return a == 1; };  // some true, exactly one, odd
    const int n = k - 2;
    std::vector<int32_t> ids(static_cast<size_t>(n));
    ids[0] = t;
    for (int i = 1; i < n; ++i) {
        ids[size_t(i)] = int32_t(net.t.size());
        net.t.push_back(InitTensor{});
    }
    std::vector<int32_t> aux(static_cast<size_t>(n - 1));
    for (int i = 0; i + 1 < n; ++i) aux[size_t(i)] = new_bond(net, ids[size_t(i)], ids[size_t(i + 1)]);
    for (int i = 0; i < n; ++i) {
        InitTensor p;
        p.kind = T_TABLE;
        p.table.assign(8, 0);
        if (i == 0) {
            p.bonds = {c.bonds[0], c.bonds[1], aux[0]};
            for (int x = 0; x < 8; ++x) {
                int s;
                const bool ok = step(lit(0, x & 1), lit(1, (x >> 1) & 1), &s);
                p.table[size_t(x)] = ok && s == ((x >> 2) & 1) ? 1 : 0;
            }
        } else if (i + 1 < n) {
            p.bonds = {aux[size_t(i - 1)], c.bonds[size_t(i + 1)], aux[size_t(i)]};
            rehome(net, c.bonds[size_t(i + 1)], t, ids[size_t(i)]);
            for (int x = 0; x < 8; ++x) {
                int s;
                const bool ok = step(x & 1, lit(i + 1, (x >> 1) & 1), &s);
                p.table[size_t(x)] = ok && s == ((x >> 2) & 1) ? 1 : 0;
            }
        } else {
            p.bonds = {aux[size_t(i - 1)], c.bonds[size_t(k - 2)], c.bonds[size_t(k - 1)]};
            rehome(net, c.bonds[size_t(k - 2)], t, ids[size_t(i)]);
            rehome(net, c.bonds[size_t(k - 1)], t, ids[size_t(i)]);
            for (int x = 0; x < 8; ++x) {
                int s1, s2;
                const bool ok = step(x & 1, lit(k - 2, (x >> 1) & 1), &s1) &&
                                step(s1, lit(k - 1, (x >> 2) & 1), &s2) && final_ok(s2);
                p.table[size_t(x)] = ok ? 1 : 0;
            }
        }
        net.t[size_t(ids[size_t(i)])] = p;
    }
}

}  // namespace

tn_status reduce_degree(Network& net, uint32_t flags) {
    try {
        const int32_t n0 = int32_t(net.t.size());
        for (int32_t t = 0; t < n0; ++t) {
            const InitTensor& x = net.t[size_t(t)];
            if ((flags & TN_BUILD_RING_COPY) && x.kind == T_COPY && x.bonds.size() > 3) ring_copy(net, t);
            else if ((flags & TN_BUILD_SPLIT_CLAUSES) && (x.kind == T_OR || x.kind == T_EXONE || x.kind == T_XOR) &&
                     x.bonds.size() > 3)
                chain_clause(net, t);
        }
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    return TN_OK;
}

tn_status build_network(const tn_formula* f, Network& net) {
    if (!f || f->n_vars < 0 || f->n_clauses < 0) return TN_EINVAL;
    if (f->n_clauses > 0 && (!f->clause_ptr || !f->kinds)) return TN_EINVAL;
    if (f->n_clauses > 0 && f->clause_ptr[0] != 0) return TN_EINVAL;
    int64_t nl = f->n_clauses > 0 ? f->clause_ptr[f->n_clauses] : 0;
    if (nl > 0 && !f->lits) return TN_EINVAL;
    for (int32_t c = 0; c < f->n_clauses; ++c) {
        if (f->clause_ptr[c + 1] < f->clause_ptr[c]) return TN_EINVAL;
        if (f->kinds[c] > TN_CLAUSE_XOR) return TN_EINVAL;
        if (f->clause_ptr[c + 1] - f->clause_ptr[c] > TN_MAX_INIT_RANK) return TN_ERANK;
    }
    for (int64_t i = 0; i < nl; ++i) {
        int32_t l = f->lits[i];
        if (l == 0 || l > f->n_vars || l < -f->n_vars) return TN_EINVAL;
    }
    try {
        net.n_vars = f->n_vars;
        net.n_clauses = f->n_clauses;
        net.count_bits = f->n_vars;  // every term of the count is 0 or 1: at most 2^n
        net.max_entry = 2;
        net.t.assign(size_t(f->n_vars) + size_t(f->n_clauses), InitTensor{});
        net.bond_end.clear();
        net.bond_end.reserve(size_t(nl));
        for (int32_t v = 0; v < f->n_vars; ++v) net.t[v].kind = T_COPY;
        for (int32_t c = 0; c < f->n_clauses; ++c) {
            InitTensor& ct = net.t[size_t(f->n_vars) + c];
            ct.kind = f->kinds[c] == TN_CLAUSE_OR ? T_OR : f->kinds[c] == TN_CLAUSE_EXACTLY_ONE ? T_EXONE : T_XOR;
            int k = 0;
            for (int32_t i = f->clause_ptr[c]; i < f->clause_ptr[c + 1]; ++i, ++k) {
                int32_t l = f->lits[i];
                int32_t v = (l < 0 ? -l : l) - 1;
                int32_t b = int32_t(net.bond_end.size());
                net.bond_end.push_back({v, f->n_vars + c});
                net.t[v].bonds.push_back(b);
                ct.bonds.push_back(b);
                if (l < 0) ct.neg |= (uint64_t(1) << k);
            }
        }
        for (int32_t v = 0; v < f->n_vars; ++v)
            if (int(net.t[v].bonds.size()) > TN_MAX_INIT_RANK) return TN_ERANK;
        // beyond 63 variables, the elimination bound (count_bound.cpp) sizes the
        // residues; it is kept at 64 bits or more, so such formulas stay
        // with small moduli rather than 64-bit counts
        // (a quick bound within 64 bits settles it without the elimination,
        // as it does for most random 1-in-3 formulas of a few hundred clauses)
        if (f->n_vars > 63)
            net.count_bits = disjoint_clause_bound_bits(f) <= 64.0 - 1e-6
                                 ? 64
                                 : std::max<int32_t>(64, count_bound_bits(f));
        // the formula itself, for the order search's tighter bound
        net.f_ptr.assign(f->clause_ptr, f->clause_ptr + (f->n_clauses > 0 ? f->n_clauses + 1 : 0));
        net.f_lits.assign(f->lits, f->lits + nl);
        net.f_kinds.assign(f->kinds, f->kinds + f->n_clauses);
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    return TN_OK;
}

tn_status build_csp(const tn_csp* c, Network& net) {
    if (!c || c->n_vars < 0 || c->n_cons < 0) return TN_EINVAL;
    if (c->n_cons > 0 && (!c->scope_ptr || !c->table_ptr || c->scope_ptr[0] != 0 || c->table_ptr[0] != 0))
        return TN_EINVAL;
    const int32_t n = c->n_vars;
    std::vector<int32_t> dom(static_cast<size_t>(n), 2);
    for (int32_t v = 0; v < n; ++v) {
        if (c->domain) dom[size_t(v)] = c->domain[v];
        if (dom[size_t(v)] < 1 || dom[size_t(v)] > TN_MAX_DOMAIN) return TN_EINVAL;
    }
    const int64_t ns = c->n_cons > 0 ? c->scope_ptr[c->n_cons] : 0;
    if (ns > 0 && !c->scope) return TN_EINVAL;
    std::vector<int> occ_bits(static_cast<size_t>(n), 0);
    for (int32_t k = 0; k < c->n_cons; ++k) {
        if (c->scope_ptr[k + 1] < c->scope_ptr[k] || c->table_ptr[k + 1] < c->table_ptr[k]) return TN_EINVAL;
        int64_t size = 1;
        int bits = 0;
        for (int32_t i = c->scope_ptr[k]; i < c->scope_ptr[k + 1]; ++i) {
            const int32_t v = c->scope[i];
            if (v < 1 || v > n) return TN_EINVAL;
            bits += bits_of(dom[size_t(v - 1)]);
            occ_bits[size_t(v - 1)] += bits_of(dom[size_t(v - 1)]);
            if (bits > TN_MAX_INIT_RANK) return TN_ERANK;
            size *= dom[size_t(v - 1)];
        }
        if (c->table_ptr[k + 1] - c->table_ptr[k] != size) return TN_EINVAL;
    }
    for (int32_t v = 0; v < n; ++v)
        if (occ_bits[size_t(v)] > TN_MAX_INIT_RANK) return TN_ERANK;
    if (c->n_cons > 0 && c->table_ptr[c->n_cons] > 0 && !c->weights) return TN_EINVAL;
    try {
        net = Network{};
        net.n_vars = n;
        net.n_clauses = c->n_cons;
        net.t.assign(size_t(n) + size_t(c->n_cons), InitTensor{});
        // bonds of every occurrence; occurrence codes are little-endian in them
        std::vector<std::vector<std::vector<int32_t>>> occ(static_cast<size_t>(n));
        double log2_bound = 0.0;
        uint64_t max_entry = 1;
        for (int32_t k = 0; k < c->n_cons; ++k) {
            InitTensor& ct = net.t[size_t(n) + k];
            ct.kind = T_TABLE;
            std::vector<int32_t> scope(c->scope + c->scope_ptr[k], c->scope + c->scope_ptr[k + 1]);
            std::vector<int> sb;  // bits per scope position
            for (int32_t v : scope) {
                const int b = bits_of(dom[size_t(v - 1)]);
                std::vector<int32_t> ob;
                for (int j = 0; j < b; ++j) {
                    const int32_t bond = new_bond(net, v - 1, n + k);
                    net.t[size_t(v - 1)].bonds.push_back(bond);
                    ct.bonds.push_back(bond);
                    ob.push_back(bond);
                }
                occ[size_t(v - 1)].push_back(ob);
                sb.push_back(b);
            }
            const int r = int(ct.bonds.size());
            ct.table.assign(size_t(1) << r, 0);
            const uint32_t* w = c->weights ? c->weights + c->table_ptr[k] : nullptr;
            uint32_t mx = 0;
            for (int64_t i = c->table_ptr[k]; i < c->table_ptr[k + 1]; ++i) mx = std::max(mx, c->weights[i]);
            for (uint64_t x = 0; x < (uint64_t(1) << r); ++x) {
                // codes of the scope positions; the table row-major, first slowest
                int64_t idx = 0;
                bool valid = true;
                int shift = 0;
                for (size_t q = 0; q < scope.size(); ++q) {
                    const int64_t code = int64_t((x >> shift) & ((uint64_t(1) << sb[q]) - 1));
                    shift += sb[q];
                    const int32_t d = dom[size_t(scope[q] - 1)];
                    if (code >= d) valid = false;
                    idx = idx * d + code;
                }
                ct.table[size_t(x)] = valid ? w[idx] : 0;
            }
            max_entry = std::max<uint64_t>(max_entry, mx);
            if (mx > 1) log2_bound += std::log2(double(mx));
        }
        for (int32_t v = 0; v < n; ++v) {
            InitTensor& t = net.t[size_t(v)];
            const int32_t d = dom[size_t(v)];
            log2_bound += std::log2(double(d));
            const int b = bits_of(d);
            const int r = int(t.bonds.size());
            const int nocc = int(occ[size_t(v)].size());
            if (r == 0) {
                // no bond: an unused variable, or one value only
                t.kind = T_TABLE;
                t.table = {uint32_t(d)};
                max_entry = std::max<uint64_t>(max_entry, uint64_t(d));
                continue;
            }
            if (b == 1) {
                t.kind = T_COPY;  // boolean: the COPY of Eq. 4
                continue;
            }
            // COPY over groups of b bonds (each occurrence's bonds are
            // consecutive in t.bonds, in occurrence order): 1 when every group
            // holds the same code and the code names a value
            t.kind = T_TABLE;
            t.table.assign(size_t(1) << r, 0);
            const uint64_t gm = (uint64_t(1) << b) - 1;
            for (uint64_t code = 0; code < uint64_t(d); ++code) {
                uint64_t x = 0;
                for (int o = 0; o < nocc; ++o) x |= code << (o * b);
                t.table[size_t(x)] = 1;
            }
            (void)gm;
        }
        net.max_entry = max_entry;
        net.count_bits = int32_t(std::ceil(log2_bound + 1e-9));
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    return TN_OK;
}

}  // namespace tn
