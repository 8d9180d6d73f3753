/*
 * tn.h -- exact model counting of #CSP formulas by tensor-network
 * contraction on one AMD Instinct MI355X (gfx950).
 *
 * The method (Kourtis, Chamon, Mucciolo, Ruckenstein, "Fast counting with
 * tensor networks", Sec. 2.1 and Sec. 3): a formula becomes a network of
 * boolean tensors -- a COPY tensor on every variable (Eq. 4), an OR (Eq. 3)
 * or exactly-one (Eq. 6) tensor on every clause, one bond of dimension 2 per
 * literal occurrence, a negated literal reversing its index -- and the full
 * contraction of the network (Eq. 2 at zero temperature) is the number of
 * satisfying assignments. A host-side order (Sec. 3.1.1: tensor-greedy,
 * tensor-METIS style recursive bisection, tensor-GN community detection, or
 * a learned scorer) fixes the sequence of pairwise contractions; HIP kernels
 * run them on the GPU. Counts are exact (the paper's floating-point counts
 * lose precision from about 100 vertices, Sec. 3.2): 64-bit unsigned
 * arithmetic while the count is below 2^64 (at most 63 boolean variables);
 * otherwise residues modulo the fewest small pairwise coprime moduli
 * (<= 255, one signed byte per residue) whose product exceeds twice the
 * largest possible count, or, beyond about 332 bits, modulo 16-bit primes;
 * the residues are combined on the host by the Chinese remainder theorem at
 * a cost linear in the number of moduli.
 *
 * Conventions for every call:
 *  - Plain C ABI, no exceptions cross it; every call returns a tn_status.
 *  - Host arrays passed in are borrowed for the call and copied; nothing the
 *    caller passes is retained unless stated.
 *  - Opaque handles are owned by the caller and released with *_free.
 *  - Device memory on the contraction path is never allocated by the
 *    library: it sub-allocates the caller's workspace (device pointer).
 *  - GPU work is queued on the caller's stream (hipStream_t passed as
 *    void*; NULL = the null stream); calls that return host results
 *    synchronize that stream before returning.
 *  - Distinct handles may be used from different threads; one handle must
 *    not be used by two threads at once.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TN_OK = 0,
    TN_EINVAL = -1,        /* malformed argument (bad literal, null pointer, ...) */
    TN_ENOMEM = -2,        /* host allocation failed */
    TN_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    TN_ETOOBIG = -4,       /* the plan's peak memory exceeds the workspace */
    TN_ERANK = -5,         /* a tensor rank exceeds TN_MAX_RANK */
    TN_EBUFSIZE = -6,      /* output buffer too small; the needed size is returned */
    TN_EUNSUPPORTED = -7   /* a valid request the library does not handle */
} tn_status;

/* Largest tensor rank the contraction kernels accept: 2^34 entries. */
#define TN_MAX_RANK 34
/* Largest rank of an initial (clause or COPY) tensor. */
#define TN_MAX_INIT_RANK 24
/* Most primes one contraction may use (counts up to ~2^2000). */
#define TN_MAX_PRIMES 128

/* Clause kinds: OR (Eq. 3), exactly-one (Eq. 6, with negation allowed; any
 * number of literals: #1-in-k SAT) and parity (#XORSAT, one of the other
 * clause types Sec. 4 names: satisfied when an odd number of literals is
 * true). Literals are counted per occurrence. */
typedef enum { TN_CLAUSE_OR = 0, TN_CLAUSE_EXACTLY_ONE = 1, TN_CLAUSE_XOR = 2 } tn_clause_kind;
/* Largest domain of a variable of a constraint network (tn_build_csp). */
#define TN_MAX_DOMAIN 256

/* A formula. Variables are 1..n_vars. Clause c owns literals
 * lits[clause_ptr[c] .. clause_ptr[c+1]-1]; a literal is +v or -v
 * (negated). kinds[c] is a tn_clause_kind. A clause may repeat a variable
 * or hold complementary literals (each occurrence is its own bond). An empty
 * clause is unsatisfiable; a variable in no clause doubles the count. */
typedef struct {
    int32_t n_vars;
    int32_t n_clauses;
    const int32_t* clause_ptr;  /* n_clauses + 1 entries, clause_ptr[0] = 0 */
    const int32_t* lits;        /* clause_ptr[n_clauses] entries */
    const uint8_t* kinds;       /* n_clauses entries */
} tn_formula;

typedef struct tn_network tn_network;
typedef struct tn_plan tn_plan;
typedef struct tn_model tn_model;

typedef enum {
    TN_ORDER_GREEDY = 0,     /* Sec. 3.1.1 tensor-greedy: smallest result rank first */
    TN_ORDER_PARTITION = 1,  /* Sec. 3.1.1 tensor-METIS: recursive best-of-2 bisection */
    TN_ORDER_COMMUNITY = 2,  /* Sec. 3.1.1 tensor-GN: Girvan-Newman split tree */
    TN_ORDER_LEARNED = 3,    /* MLP pair scorer judged against greedy; plans predicted above
                                50 ms go on to the full judge as its incumbent */
    TN_ORDER_BEST = 4,       /* cheapest of greedy, community and randomized partitions (rounds
                                of 16 over the host threads), searched while the host time
                                spent stays below twice the best plan's predicted device time */
    TN_ORDER_LEARNED_RAW = 5 /* the learned order alone, not judged (evaluation) */
} tn_order_kind;

/* Predicted cost of a plan, known before any tensor entry is touched (the
 * "lazy" evaluation of Sec. 4). Entries and multiply-adds are per residue
 * plane; log2_cost is the log2 of the predicted device time in microseconds
 * of the whole contraction in the default residue arithmetic (64-bit counts
 * for n_vars <= 63, else small moduli when they hold the count, else 16-bit
 * primes; all planes and launches). */
typedef struct {
    int32_t n_steps;
    int32_t max_rank;              /* largest rank of any tensor in the plan */
    double entries;                /* sum over steps of 2^rA + 2^rB + 2^rC */
    double macs;                   /* sum over steps of 2^(rA + rB - s) */
    double log2_cost;              /* log2 of the predicted device time (us) used to judge orders */
    uint64_t peak_elems;           /* arena high-water mark in entries, one prime */
    int32_t chosen;                /* tn_order_kind that produced the plan */
    int32_t fallback;              /* TN_ORDER_LEARNED: 1 when the plan kept is not the learned one */
    int32_t refined;               /* 1 when local tree reconfiguration improved the plan */
} tn_plan_stats;

typedef enum { TN_ARITH_AUTO = 0, TN_ARITH_U64 = 1, TN_ARITH_RNS = 2 } tn_arith;

typedef struct {
    int32_t arith;            /* tn_arith; AUTO = U64 if n_vars <= 63 else RNS */
    int32_t n_primes;         /* RNS: 0 = the fewest small moduli (see tn_moduli) or, if those do
                                 not hold 2^(n_vars + 1), the fewest primes of tn_primes that do;
                                 k > 0 = the first k primes of tn_primes */
    void* workspace;          /* device memory owned by the caller */
    size_t workspace_bytes;
    void* stream;             /* hipStream_t; NULL = null stream */
    int32_t prime_group;      /* primes resident at once; 0 = as many as fit */
    int32_t flags;            /* TN_FLAG_* */
} tn_contract_opts;

#define TN_FLAG_GENERIC_ONLY 1   /* use only the generic kernel (testing) */
#define TN_FLAG_NO_MFMA 2        /* never use the int8 matrix-core kernels */
#define TN_FLAG_TIMING 4         /* record per-kernel-class device times */
#define TN_FLAG_NO_GRAPH 8       /* batch: launch waves directly, no hipGraph */
#define TN_FLAG_WIDE_RNS 16      /* RNS with 16-bit primes even where small moduli suffice */

/* ------------------------------------------------------------------ build
 * Formula -> network (Sec. 2.1). Validates every literal and clause kind;
 * returns TN_EINVAL on malformed input and TN_ERANK when a variable occurs
 * more than TN_MAX_INIT_RANK times or a clause has more literals. */
tn_status tn_build(const tn_formula* f, tn_network** out);
void tn_network_free(tn_network* net);

/* Degree reduction (Sec. 4: splitting long clauses, COPY tensors as rings of
 * rank-3 tensors), flags of tn_build_ex and tn_build_csp. RING_COPY: a
 * boolean COPY tensor of rank d > 3 becomes d rank-3 COPY tensors on a ring
 * of d new bonds, each holding one of the original bonds. SPLIT_CLAUSES: an
 * OR, exactly-one or parity clause of k > 3 literals becomes a chain of k - 2
 * rank-3 tensors linked by k - 3 new bonds that carry the clause's running
 * state ("some literal true", "one literal true so far", parity); the count
 * is unchanged and no initial tensor keeps a rank above 3 (other than
 * tables of tn_build_csp). New tensors follow the original ones. */
#define TN_BUILD_RING_COPY 1
#define TN_BUILD_SPLIT_CLAUSES 2
/* tn_build, then the degree reduction of ``flags``. */
tn_status tn_build_ex(const tn_formula* f, uint32_t flags, tn_network** out);

/* A weighted constraint network over variables of any domain (Sec. 4:
 * non-boolean and mixed domains, weighted #CSP): variable v (1..n_vars)
 * takes the values 0..domain[v-1]-1, 1 <= domain[v-1] <= TN_MAX_DOMAIN (NULL:
 * every variable boolean). Constraint c has a scope scope[scope_ptr[c] ..
 * scope_ptr[c+1]-1] of variables (a variable may repeat; an empty scope is
 * a constant weight) and a table of non-negative integer weights
 * weights[table_ptr[c] .. table_ptr[c+1]-1], one per joint value of its
 * scope, row-major with the first scope variable slowest. The count is the
 * sum over all assignments of the product of the constraints' weights (the
 * partition function of Eq. 2 with the constraint tensors in place of
 * exp(-beta E)); it is exact for any weights. The network keeps the boolean
 * bonds of Sec. 2.1: a variable of D values has ceil(log2 D) bonds per
 * occurrence (its value in binary), its COPY tensor is 1 where every
 * occurrence holds the same value below D (the scalar D when it has no bond),
 * and a constraint's tensor is 0 wherever an occurrence holds a code of D or
 * more. Host arrays are borrowed and copied. TN_EINVAL on a malformed
 * network or a table of the wrong size; TN_ERANK when a constraint's or a
 * variable's bonds exceed TN_MAX_INIT_RANK. flags: TN_BUILD_* (boolean COPY
 * tensors only). */
typedef struct {
    int32_t n_vars;
    const int32_t* domain;      /* n_vars entries, or NULL */
    int32_t n_cons;
    const int32_t* scope_ptr;   /* n_cons + 1 entries, scope_ptr[0] = 0 */
    const int32_t* scope;       /* scope_ptr[n_cons] entries */
    const int64_t* table_ptr;   /* n_cons + 1 entries, table_ptr[0] = 0 */
    const uint32_t* weights;    /* table_ptr[n_cons] entries */
} tn_csp;
tn_status tn_build_csp(const tn_csp* c, uint32_t flags, tn_network** out);
/* Largest rank among the initial tensors, and the bound the arithmetic is
 * sized for: every count of the network is at most 2^count_bits. */
tn_status tn_network_ranks(const tn_network* net, int32_t* max_init_rank, int32_t* count_bits);
/* Number of tensors (n_vars COPY tensors first, then one per clause) and
 * bonds (one per literal occurrence). */
tn_status tn_network_info(const tn_network* net, int32_t* n_tensors, int32_t* n_bonds);

/* ------------------------------------------------------------------ order
 * Host-only: chooses a pairwise contraction order and lays out the plan
 * (bit order of every tensor, arena offsets, kernel choice) and its
 * predicted cost. ``seed`` drives the randomized bisections. ``model`` is
 * used by TN_ORDER_LEARNED (may be NULL otherwise; with NULL the learned
 * order falls back to the judge's choice). With several host threads the
 * judge (TN_ORDER_BEST, and TN_ORDER_LEARNED when it hands its plan on)
 * also computes a tighter count bound for a boolean formula whose
 * network's bound exceeds 64 bits, and the plan carries it: its
 * contraction may then use fewer residue planes than tn_network_ranks'
 * count_bits implies (never fewer than for 64 bits). */
tn_status tn_order(const tn_network* net, tn_order_kind kind, uint64_t seed,
                   const tn_model* model, tn_plan** out, tn_plan_stats* stats);
/* tn_order with a fixed search (Sec. 4: lazy evaluation, spending search where
 * the predicted contraction is costly): with rounds > 0, TN_ORDER_BEST (and
 * TN_ORDER_LEARNED when it hands its plan to the judge) runs exactly that
 * many rounds of 16 randomized bisections (spread over the host threads),
 * instead of stopping at twice the best plan's predicted device time or 24
 * rounds (one on a single thread), and reconfigures the best quarter of
 * them until each settles, with no time budget: the plan then depends only
 * on the seed.
 * rounds = 0 is tn_order; rounds outside [0, 256] give TN_EINVAL. */
tn_status tn_order_rounds(const tn_network* net, tn_order_kind kind, uint64_t seed,
                          const tn_model* model, int32_t rounds, tn_plan** out,
                          tn_plan_stats* stats);
void tn_plan_free(tn_plan* plan);
/* Copy the merges of a plan: pairs[2k], pairs[2k+1] are the tensor ids of
 * step k, which creates tensor id n_tensors + k. cap = pair capacity. */
tn_status tn_plan_steps(const tn_plan* plan, int32_t* pairs, int32_t cap, int32_t* n_steps);
/* Self-check of a plan's memory layouts: TN_OK when no two tensors that are
 * alive at the same time overlap in the arena, both for one-step-at-a-time
 * execution and for execution in waves of equal level; TN_EINVAL otherwise. */
tn_status tn_plan_verify(const tn_plan* plan);

/* --------------------------------------------------------------- contract
 * Device workspace needed for a plan under opts (arith, n_primes,
 * prime_group, flags; workspace fields ignored). With prime_group = 0 the
 * answer is for one residue plane resident at a time. */
tn_status tn_workspace_bytes(const tn_network* net, const tn_plan* plan,
                             const tn_contract_opts* opts, size_t* bytes);

/* Runs the plan on the GPU: the ordered pairwise contractions of Sec. 2.1
 * (each step sums over every bond its two tensors share, Eq. 5 form; all
 * parallel bonds at once, Sec. 2.2) until the network is one scalar, the
 * full trace of Eq. 2 at zero temperature. RNS: writes the count modulo each modulus that
 * tn_moduli lists for the same plan and opts, in that order, to
 * residues[0..k-1]. U64: writes the exact count to *u64. Either output
 * pointer may be NULL when unused. Returns TN_ETOOBIG before any device work
 * when the workspace cannot hold one residue plane's arena. */
tn_status tn_contract(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts,
                      uint32_t* residues, int32_t residues_cap, uint64_t* u64);

/* tn_contract without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the workspace is a file-scope device array of
 * tn_noalloc_max_bytes() bytes (64 MiB) that the library holds on every GPU
 * it runs on until the process ends; opts->workspace and
 * opts->workspace_bytes are ignored, every other field is used as by
 * tn_contract, and the outputs are tn_contract's. Returns TN_ETOOBIG before
 * any device work when the plan's initial tensors, one residue plane's
 * arena and its scratch do not fit the array (tn_workspace_bytes with
 * prime_group = 0 gives the need), TN_EUNSUPPORTED with TN_FLAG_TIMING.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind (nothing in it needs to start at zero): calls that overlap on one
 * GPU, from two threads or on two streams, race and must not be made. */
tn_status tn_contract_noalloc(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts,
                              uint32_t* residues, int32_t residues_cap, uint64_t* u64);
/* Size in bytes of tn_contract_noalloc's device array. */
size_t tn_noalloc_max_bytes(void);

/* Exact count (Sec. 2.1: the full contraction of the network is the number
 * of satisfying assignments; exact integers instead of the floating-point
 * counts of Sec. 3.2) as little-endian base-2^32 limbs: the CRT of
 * tn_contract's residues, or its 64-bit value. limbs is a host buffer of cap
 * entries; TN_EBUFSIZE with *n_limbs set when cap is too small. */
tn_status tn_count(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts,
                   uint32_t* limbs, size_t cap, size_t* n_limbs);

/* Batched counting of n formulas: build and order on host threads, then
 * contract all instances together in waves (one persistent launch per wave,
 * captured in a hipGraph). limbs holds cap_per limbs per instance; n_limbs
 * receives each instance's limb count. The workspace is split into
 * sub-batches that fit. stats (nullable) receives n entries. */
tn_status tn_count_batch(const tn_formula* fs, int32_t n, tn_order_kind kind, uint64_t seed,
                         const tn_contract_opts* opts, uint32_t* limbs, size_t cap_per,
                         size_t* n_limbs, tn_plan_stats* stats);

/* Device time per kernel class recorded by the last tn_contract / tn_count /
 * tn_count_batch call of the calling thread made with TN_FLAG_TIMING
 * (hipEvents around every launch, on the caller's stream). bytes and macs
 * are the algorithmic totals of those launches: 2^rA + 2^rB + 2^rC entries
 * of 1 (small-modulus residues), 4 or 8 bytes and 2^(rA + rB - s)
 * multiply-adds per step and residue plane. */
typedef enum {
    TN_KC_GENERIC = 0, TN_KC_STREAM = 1, TN_KC_ROWDOT = 2, TN_KC_MFMA = 3, TN_KC_BATCH = 4, TN_KC_DOT = 5,
    TN_KC_DIGITS = 6,  /* in-place digit pass before TN_KC_MFMA */
    TN_KC_NARROW = 7   /* int8 matrix cores, B side of at most 64 rows: streams A once */
} tn_kernel_class;
#define TN_KERNEL_CLASSES 8
typedef struct {
    int64_t launches;
    double ms;
    double bytes;
    double macs;
} tn_kernel_profile;
tn_status tn_profile_get(tn_kernel_profile* out /* TN_KERNEL_CLASSES entries */);
/* The individual launches of that record (at most 2^20), in launch order:
 * kernel class, step shape and device time. *n receives the count. */
typedef struct {
    int32_t kernel_class;
    int32_t rA, rB, s, rC;
    int32_t planes;
    double ms;
} tn_launch_record;
tn_status tn_profile_launches(tn_launch_record* out, int64_t cap, int64_t* n);

/* One contraction step from host buffers (test and measurement hook):
 *     C[c] = sum over z < 2^s of A[z + 2^s xA] * B[z + 2^s xB]
 * where xA gathers the bits of c selected by maskA and xB the remaining bits
 * of c below 2^(rA + rB - 2s) (the shared bonds are the low s bits of both
 * operands, Sec. 2.1 / Eq. 5 form). Entries are uint32 residues modulo
 * ``prime`` (arith TN_ARITH_RNS; a prime in (2^16 - 2^11, 65280), as
 * tn_primes returns, or a small modulus 2 <= m <= 255, computed on the
 * device as centred int8 residues; inputs are taken modulo m, outputs are
 * in [0, m)) or uint64 wrapping (TN_ARITH_U64). ``kernel`` forces a
 * tn_kernel_class (-1 = the library's choice); TN_EUNSUPPORTED if that kernel
 * cannot run this shape. The workspace (device) must hold the three tensors,
 * each rounded up to 256 bytes, plus 4 MiB of scratch; A and B may be
 * overwritten on the device. */
tn_status tn_step(const void* A, int32_t rA, const void* B, int32_t rB, int32_t s, uint64_t maskA,
                  int32_t arith, uint32_t prime, int32_t kernel, void* C, void* workspace,
                  size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------- learned order
 * A 3-layer perceptron scores candidate pairs of live tensors from 10
 * features (ranks, shared bonds, result rank, neighbour counts; see
 * order_learned.cpp): h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
 * y = w3 . h2 + b3 with hidden width 128, fp32. The learned order contracts
 * the best-scoring pair at every step; tn_order(TN_ORDER_LEARNED) keeps it
 * when its predicted cost is at most greedy's, else greedy's plan, and hands
 * the kept plan to the full judge as its incumbent when it is predicted to
 * take more than 50 ms on the device (Sec. 4: portfolio and lazy evaluation).
 * Parameters are packed as W1 [128 x 10], b1 [128], W2 [128 x 128], b2 [128],
 * w3 [128], b3 (tn_model_param_count() floats). */
int32_t tn_model_param_count(void);
/* Host-side model for ordering; params (host, nullable = zeros) are copied. */
tn_status tn_model_create(const float* params, tn_model** out);
void tn_model_free(tn_model* model);
tn_status tn_model_get(const tn_model* model, float* params);
/* Host forward pass over n rows of 10 features (row-major) -> n scores. */
tn_status tn_model_score(const tn_model* model, const float* x, int32_t n, float* y);
/* Imitation data along a teacher plan's merge sequence: before each merge,
 * one row of features per connected pair of live tensors (plus the teacher's
 * pair if it shares no bond), label 1 for pairs the teacher merges while both
 * are alive. groups[g] .. groups[g+1]-1 are the rows of state g. Host
 * buffers; TN_EBUFSIZE with the needed sizes when a capacity is too small. */
tn_status tn_trace(const tn_network* net, const tn_plan* teacher, float* feats, uint8_t* labels, int32_t* groups,
                   int64_t cap_rows, int32_t cap_groups, int64_t* n_rows, int32_t* n_groups);
/* GPU training kernels (all pointers device memory owned by the caller,
 * queued on ``stream``). Forward: H1, H2 [n x 128], y [n]. Backward: the
 * listwise loss L_g = log sum_{rows of g} exp(y) - log sum_{label 1} exp(y),
 * averaged over the n_groups groups (device offsets, n_groups + 1 entries),
 * into *loss; parameter gradients into grad (overwritten); dZ2, dZ1
 * [n x 128] and dy [n] are scratch. Adam: one step (step >= 1) on the packed
 * parameters with moment buffers m, v. */
tn_status tn_mlp_forward(const float* params, const float* x, int64_t n, float* h1, float* h2, float* y,
                         void* stream);
tn_status tn_mlp_backward(const float* params, const float* x, const float* h1, const float* h2, const float* y,
                          const uint8_t* labels, const int32_t* groups, int32_t n_groups, int64_t n, float* grad,
                          float* dz2, float* dz1, float* dy, float* loss, void* stream);
tn_status tn_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                      float beta2, float eps, void* stream);

/* -------------------------------------------------------------- autotuner
 * tn_autotune times every configuration of the tunable kernels over a grid
 * of step shapes on the current device (hipEvents on ``stream``, the best of
 * ``reps`` timed launches after one warm-up): the tile shape (256 x 256,
 * 256 x 128, 128 x 128, 256 x 64, 128 x 64) of the tiled int8 matrix-core
 * kernel, and the B rows per thread (1..16) of the streaming kernel for int8
 * residues and 64-bit counts. The fastest configuration per shape is used by
 * every later launch in the process (the nearest tuned shape of the same
 * kernel and element kind whose configuration fits the step), and the table
 * is written to ``out_path`` (nullable) as JSON: one entry per shape with the
 * measured microseconds per residue plane of every configuration.
 * ``workspace`` (device, at least 64 MiB; larger shapes are skipped when it
 * is small) is overwritten. TN_EHIP if a launch fails. */
tn_status tn_autotune(const char* out_path, void* workspace, size_t workspace_bytes, void* stream, int32_t reps);
/* Installs the table of a cache written by tn_autotune (replacing any table
 * in use; launches in flight keep the old one). ``arch`` (nullable): refuse
 * with TN_EUNSUPPORTED a cache measured on another architecture, e.g.
 * "gfx950". path = NULL removes the table (built-in rules everywhere).
 * TN_EINVAL if the file cannot be read or parsed. */
tn_status tn_tune_load(const char* path, const char* arch);

/* -------------------------------------------------------------- utilities */
/* The k largest primes below 65280, descending, as used by the RNS path
 * (k <= TN_MAX_PRIMES; all lie above 2^16 - 2^11). */
tn_status tn_primes(int32_t k, uint32_t* out);
/* Number of primes the RNS path uses by default for a formula with n_vars
 * variables: the fewest leading primes of tn_primes whose product exceeds
 * 2^(n_vars + 1) (every count is at most 2^n_vars). TN_EINVAL if n_vars < 0
 * or more than TN_MAX_PRIMES primes would be needed. */
tn_status tn_primes_for(int32_t n_vars, int32_t* k);
/* Residue moduli of a contraction of ``plan`` under ``opts`` (RNS): the
 * first k small moduli -- pairwise coprime integers of at most 255 taken
 * greedily from 255 down (255, 254, 253, 251, 247, ...), whose centred
 * residues are single int8 values -- when their product exceeds
 * 2^(n_vars + 1) (n_vars up to about 332) and neither opts->n_primes nor
 * TN_FLAG_WIDE_RNS asks for primes; otherwise the primes of tn_primes the
 * contraction uses. tn_contract's residues are modulo these, in order.
 * *k = 0 for 64-bit arithmetic; TN_EBUFSIZE (with *k set) if cap < *k. */
tn_status tn_moduli(const tn_plan* plan, const tn_contract_opts* opts, uint32_t* out, int32_t cap, int32_t* k);
/* Chinese remaindering of residues modulo the first k primes of tn_primes
 * into little-endian base-2^32 limbs. */
tn_status tn_crt(const uint32_t* residues, int32_t k, uint32_t* limbs, size_t cap, size_t* n_limbs);
/* Chinese remaindering of residues[i] modulo moduli[i] (i < k; any pairwise
 * coprime moduli >= 2, such as those tn_moduli returns for a plan, so that
 * tn_contract's residues recombine into the count) into the unique integer
 * below their product, as little-endian base-2^32 limbs (host buffers).
 * TN_EINVAL if a residue is not below its modulus or two moduli share a
 * factor; TN_EBUFSIZE with *n_limbs set when cap is too small. */
tn_status tn_crt_moduli(const uint32_t* residues, const uint32_t* moduli, int32_t k, uint32_t* limbs, size_t cap,
                        size_t* n_limbs);
const char* tn_status_str(tn_status s);

/* ------------------------------------------------------------- generators
 * Seeded synthetic instances shaped like the paper's workloads (Sec. 3.2):
 * random cubic graphs, #Cubic-Vertex-Cover as 2-variable OR clauses (one
 * variable per vertex, one clause per edge), monotone 1-in-3 with uniform
 * clauses, and the paper's own 1-in-3 family on cubic graphs (one variable
 * per edge, one exactly-one clause per vertex: every variable occurs in two
 * clauses, the solutions are the perfect matchings). Random numbers:
 * SplitMix64 seeding xoshiro256**, bounded draws by rejection; cubic graphs by
 * the configuration model, the whole draw rejected on a loop or repeated
 * edge (uniform over simple cubic graphs; the paper samples the same
 * distribution with the Viger-Latapy method). Outputs are caller-owned host
 * arrays in the tn_formula layout; a formula's sizes are fixed by its
 * arguments, as stated per call. TN_EINVAL on a bad size or NULL output,
 * TN_EUNSUPPORTED if no simple graph was drawn in 100000 tries. */
/* Seed of instance ``index`` of workload ``family`` under ``master``
 * (SplitMix64 of master ^ family << 40 ^ index). */
uint64_t tn_instance_seed(int32_t family, uint64_t index, uint64_t master);
/* Simple cubic graph on n (even, >= 4) vertices 0..n-1: edges[2i], edges[2i+1]
 * for i < 3n/2, each pair (smaller, larger). */
tn_status tn_gen_cubic_graph(int32_t n, uint64_t seed, int32_t* edges);
/* Monotone 1-in-3: n variables, m clauses of 3 distinct variables drawn
 * uniformly. clause_ptr: m + 1, lits: 3m, kinds: m entries. */
tn_status tn_gen_exactly_one_3(int32_t n, int32_t m, uint64_t seed, int32_t* clause_ptr, int32_t* lits,
                               uint8_t* kinds);
/* Vertex cover of a random cubic graph on n vertices (OR clause per edge,
 * in tn_gen_cubic_graph's edge order). clause_ptr: 3n/2 + 1, lits: 3n,
 * kinds: 3n/2 entries. */
tn_status tn_gen_cubic_vc(int32_t n, uint64_t seed, int32_t* clause_ptr, int32_t* lits, uint8_t* kinds);
/* The paper's 1-in-3 family on a random cubic graph with n_vertices vertices:
 * 3 n_vertices / 2 variables (variable i + 1 = edge i), one exactly-one clause
 * per vertex over its three edges in increasing order. clause_ptr:
 * n_vertices + 1, lits: 3 n_vertices, kinds: n_vertices entries. */
tn_status tn_gen_cubic_1in3(int32_t n_vertices, uint64_t seed, int32_t* clause_ptr, int32_t* lits, uint8_t* kinds);

/* Library version string. */
const char* tn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TN_H */
