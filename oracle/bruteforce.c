/* O-A in plain C: enumerate every assignment x in {0,1}^n and count those
 * satisfying every clause -- the zero-temperature partition function of
 * Eq. 2 (Sec. 2.1) with OR clauses (Eq. 3), exactly-one clauses (Eq. 6),
 * parity clauses (kind 2: an odd number of true literals) and negated
 * literals (Sec. 2.1). Test infrastructure only.
 *
 * Variable v (1-based) is bit v-1 of x. For clause c, pos_c / neg_c are the
 * bit masks of its positive / negated literals; the literals true under x are
 * counted as popcount(x & pos) + popcount(~x & neg), each occurrence of a
 * repeated literal counted separately (a clause lists literals, not a set).
 * So a clause is handled as a list of literal masks, one per occurrence.
 */
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

int bf_count(int n, int m, const int32_t* clause_ptr, const int32_t* lits,
             const uint8_t* kinds, int threads, uint64_t* out) {
    if (n < 0 || n > 40 || m < 0 || !out) return -1;
    int nl = m ? clause_ptr[m] : 0;
    /* one entry per literal occurrence: bit mask and polarity */
    uint64_t* lmask = (uint64_t*)malloc(sizeof(uint64_t) * (nl + 1));
    uint8_t* lneg = (uint8_t*)malloc(nl + 1);
    if (!lmask || !lneg) { free(lmask); free(lneg); return -2; }
    for (int i = 0; i < nl; ++i) {
        int v = lits[i] < 0 ? -lits[i] : lits[i];
        if (v < 1 || v > n) { free(lmask); free(lneg); return -1; }
        lmask[i] = 1ull << (v - 1);
        lneg[i] = lits[i] < 0;
    }
    for (int c = 0; c < m; ++c)
        if (kinds[c] > 2 || clause_ptr[c + 1] < clause_ptr[c]) { free(lmask); free(lneg); return -1; }
    /* clauses whose variables are all distinct use a popcount test on two
     * masks; a clause naming one variable twice keeps the per-literal loop */
    uint64_t* pos = (uint64_t*)calloc(m + 1, sizeof(uint64_t));
    uint64_t* neg = (uint64_t*)calloc(m + 1, sizeof(uint64_t));
    uint8_t* simple = (uint8_t*)malloc(m + 1);
    if (!pos || !neg || !simple) { free(lmask); free(lneg); free(pos); free(neg); free(simple); return -2; }
    for (int c = 0; c < m; ++c) {
        simple[c] = 1;
        for (int i = clause_ptr[c]; i < clause_ptr[c + 1]; ++i) {
            if ((pos[c] | neg[c]) & lmask[i]) simple[c] = 0;
            if (lneg[i]) neg[c] |= lmask[i]; else pos[c] |= lmask[i];
        }
    }
    uint64_t total = 0;
    int64_t N = (int64_t)1 << n;
    int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(static, 1 << 14) reduction(+ : total) if (n > 14) num_threads(nt)
    for (int64_t xi = 0; xi < N; ++xi) {
        uint64_t x = (uint64_t)xi;
        int ok = 1;
        for (int c = 0; c < m && ok; ++c) {
            int t = 0;
            if (simple[c]) {
                t = __builtin_popcountll((x & pos[c]) | (~x & neg[c]));
            } else {
                for (int i = clause_ptr[c]; i < clause_ptr[c + 1]; ++i) {
                    int bit = (x & lmask[i]) != 0;
                    t += lneg[i] ? !bit : bit;
                }
            }
            ok = kinds[c] == 0 ? (t >= 1) : kinds[c] == 1 ? (t == 1) : (t & 1);
        }
        total += (uint64_t)ok;
    }
    free(pos);
    free(neg);
    free(simple);
    free(lmask);
    free(lneg);
    *out = total;
    return 0;
}
