// Formula -> tensor network (Sec. 2.1): a COPY tensor per variable (Eq. 4),
// a clause tensor per clause (OR, Eq. 3; exactly-one, Eq. 6), and one bond
// per literal occurrence joining the variable's COPY tensor to the clause.
#include <new>

#include "internal.hpp"

namespace tn {

tn_status build_network(const tn_formula* f, Network& net) {
    if (!f || f->n_vars < 0 || f->n_clauses < 0) return TN_EINVAL;
    if (f->n_clauses > 0 && (!f->clause_ptr || !f->kinds)) return TN_EINVAL;
    if (f->n_clauses > 0 && f->clause_ptr[0] != 0) return TN_EINVAL;
    int64_t nl = f->n_clauses > 0 ? f->clause_ptr[f->n_clauses] : 0;
    if (nl > 0 && !f->lits) return TN_EINVAL;
    for (int32_t c = 0; c < f->n_clauses; ++c) {
        if (f->clause_ptr[c + 1] < f->clause_ptr[c]) return TN_EINVAL;
        if (f->kinds[c] > TN_CLAUSE_EXACTLY_ONE) return TN_EINVAL;
        if (f->clause_ptr[c + 1] - f->clause_ptr[c] > TN_MAX_INIT_RANK) return TN_ERANK;
    }
    for (int64_t i = 0; i < nl; ++i) {
        int32_t l = f->lits[i];
        if (l == 0 || l > f->n_vars || l < -f->n_vars) return TN_EINVAL;
    }
    try {
        net.n_vars = f->n_vars;
        net.n_clauses = f->n_clauses;
        net.t.assign(size_t(f->n_vars) + size_t(f->n_clauses), InitTensor{});
        net.bond_end.clear();
        net.bond_end.reserve(size_t(nl));
        for (int32_t v = 0; v < f->n_vars; ++v) net.t[v].kind = T_COPY;
        for (int32_t c = 0; c < f->n_clauses; ++c) {
            InitTensor& ct = net.t[size_t(f->n_vars) + c];
            ct.kind = f->kinds[c] == TN_CLAUSE_OR ? T_OR : T_EXONE;
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
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    return TN_OK;
}

}  // namespace tn
