/*
 * fmm.h -- C ABI of the MI355X (gfx950) fast multipole library.
 *
 * The library evaluates, on one GPU, the per-rank part of the fast multipole
 * method of AbdulJabbar, Yokota & Keyes, "Asynchronous Execution of the Fast
 * Multipole Method Using Charm++" (arXiv 1405.7487): for N bodies with
 * coordinates x and charges q it returns the Laplace potential and field
 *
 *     phi_i = sum_{j: x_j != x_i} q_j / |x_i - x_j|,
 *     E_i   = -grad_i phi_i = sum_j q_j (x_i - x_j) / |x_i - x_j|^3,
 *
 * approximated with the paper's six operators P2M, M2M, M2L, L2L, L2P and
 * P2P (Section II.A), a local octree built from the rank's own bounding box
 * with 64-bit Morton keys (Section II.B), an upward pass, a dual tree
 * traversal and a downward pass (Section II.C), under the parameters P
 * (expansion order), theta (acceptance criterion) and N_crit (maximum bodies
 * per leaf) of Table I.  Expansions are solid spherical harmonics of degree
 * n < p; the error falls as O(theta^p) (Section III.A).  The kernel carries
 * no 1/(4 pi) factor and coincident bodies do not interact.
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers on the current HIP device,
 *     contiguous, in the caller's original body order.  x and field are
 *     N x 3 row-major; q, phi, grad_phi, dq are length N; dx is N x 3.
 *   - The element type of every caller array is given by fmm_dtype (float64
 *     or float32).  Tree geometry is always computed in float64; float32
 *     coordinates are widened exactly.
 *   - The caller owns every array it passes.  The library never keeps a
 *     caller pointer after a call returns.  A plan owns its internal device
 *     buffers, obtained through the fmm_allocator given to fmm_build (or an
 *     internal caching pool when that pointer is NULL) and released by
 *     fmm_destroy.
 *   - Work is enqueued on hip_stream (a hipStream_t; NULL = default stream).
 *     fmm_build synchronises that stream, because the tree's sizes depend on
 *     the data.  fmm_evaluate_plan and fmm_adjoint are asynchronous.
 *   - Every entry point returns a status; no C++ exception crosses the ABI.
 *     fmm_last_error() returns a thread-local message about the last failure.
 *   - Calls on one plan must not overlap; distinct plans are independent.
 */
#ifndef FMM_H_
#define FMM_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define FMM_API __attribute__((visibility("default")))
#else
#define FMM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FMM_OK = 0,
    FMM_ERR_INVALID = 1,     /* bad argument: NULL pointer, n < 0, p, theta or ncrit out of range */
    FMM_ERR_NOMEM = 2,       /* an allocation failed; everything already allocated was released   */
    FMM_ERR_DEVICE = 3,      /* a HIP runtime call failed                                        */
    FMM_ERR_UNSUPPORTED = 4, /* n >= 2^31 (indices are 32-bit) or a list would overflow         */
    FMM_ERR_NONFINITE = 5    /* a coordinate is NaN or infinite                                  */
} fmm_status;

typedef enum { FMM_F64 = 0, FMM_F32 = 1 } fmm_dtype;

typedef enum {
    FMM_PREC_FP64 = 0,  /* every stage in float64 (the plain FP64 GPU FMM)                       */
    FMM_PREC_MIXED = 1  /* P2P, P2M, L2P and the bulk of M2L in float32 with float32 accumulation;
                           float64 for M2M/L2L and coefficient accumulation at coarse levels      */
} fmm_precision;

/* Method parameters (Table I: P, theta, N_crit). */
typedef struct {
    int32_t p;                  /* expansion order: degrees 0 <= n < p, 1 <= p <= 16             */
    double theta;               /* acceptance: R_A + R_B < theta |c_A - c_B|, 0 < theta < 1,
                                   R = radius of the cell's bounding sphere                      */
    int32_t ncrit;              /* a cell holding more than ncrit bodies is split (>= 1)         */
    int32_t precision;          /* fmm_precision                                                 */
    int32_t coarse_fp64_levels; /* MIXED: levels 0 .. coarse_fp64_levels-1 keep float64
                                   multipole/local coefficients and translations (default 3)    */
    int32_t kahan;              /* MIXED: compensated P2P sums across source batches (default 1) */
    int32_t tight;              /* 1: a pair is also accepted when the cells' radii about their
                                   lattice centers, tight to their bodies (boxes squeezed to the
                                   bodies, Section II.B, Fig. `orb2'), meet the criterion; the radius
                                   is the farthest corner of a member body's 2^-21 lattice cell,
                                   rounded up to units of S 2^-22 (default 0: cube radii only)     */
    int32_t m2l_sparse;         /* same-level M2L runs as dense products over tiles of targets that
                                   share one offset; a tile row (one offset) with fewer than
                                   m2l_sparse sources per 64 targets is evaluated pair by pair with
                                   the cross-level pairs instead (same sums up to rounding order).
                                   0: never; -1 (default): 24 in plans with at least 1024 tiles,
                                   else never (small plans pay more to set up the pairs than the
                                   rows cost)                                                      */
    int32_t m2l_rotation;       /* 1: every M2L pair by rotation, O(p^3) per pair (the O(P^3) end of
                                   the operator cost range, Section III.A): the offset is turned onto
                                   +z, the expansion translated along z and turned back, in float64
                                   on the vector units; 0 (default): dense operators, O(p^4) on the
                                   matrix cores                                                    */
    int32_t mutual;             /* 1: mutual P2P (Section II.C lists mutual interactions among the
                                   features of the underlying code): each unordered pair of
                                   different leaves is evaluated once and both leaves gain their
                                   sums, a leaf's own pairs one-sided; the sums of every (pair,
                                   body) are kept and added per body in a fixed order, so results
                                   stay bit-reproducible; needs 16 B (32 B in FP64) per source body
                                   of every such pair in the plan.  0 (default): every list entry
                                   one-sided                                                       */
} fmm_params;

/* Fills defaults: p=8, theta=0.4, ncrit=64, MIXED, coarse_fp64_levels=3,
 * kahan=1, tight=0, m2l_sparse=-1, m2l_rotation=0, mutual=0.  P, theta and N_crit are the method parameters of Table I
 * (Section III.A); the values are this library's defaults, not the paper's.
 * A NULL prm is ignored. */
FMM_API void fmm_params_default(fmm_params *prm);

/* Device memory provider (no passage of the paper: plumbing of this library).
 * alloc returns a device pointer of at least `bytes` bytes usable on
 * `stream`, or NULL on failure (the library then returns FMM_ERR_NOMEM after
 * handing back everything it had obtained); free returns it.  Both are called
 * from the thread that calls the library. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} fmm_allocator;

typedef struct fmm_plan fmm_plan; /* opaque: tree, lists, operators, buffers */

/* Counts and timings of a plan (host struct filled by fmm_plan_stats).  The
 * list sizes are the interaction counts of Section II.C (l_i of Eq. (1)
 * summed over a rank's bodies); the phases follow the runtime breakdown of
 * Section III.A (tree build, traversal, the M2L and P2P kernels). */
typedef struct {
    int64_t n, ncell, nleaf;
    int32_t depth, p;
    int64_t n_m2l;           /* all M2L pairs                                  */
    int64_t n_m2l_same;      /* M2L pairs between cells of one level            */
    int64_t n_m2l_cross;     /* M2L pairs between cells of different levels     */
    int64_t n_p2p;           /* P2P leaf pairs                                 */
    int64_t p2p_body_pairs;  /* sum over P2P pairs of |A| * |B|, -1 until
                                fmm_count_body_pairs has counted it            */
    int64_t m2l_stencil;     /* same-level offsets per target octant class     */
    int64_t m2l_offsets;     /* distinct same-level offsets (operators)        */
    int64_t m2l_slots;       /* slot entries scanned by the batched M2L         */
    int64_t device_bytes;    /* bytes held by the plan                          */
    /* build: host wall clock of fmm_build and of its parts (tree = box, keys,
     * sort, cells, geometry; traverse = stencils, tiles, dual traversal, lists;
     * ops = operator tables and M2L schedule) */
    double ms_build, ms_tree, ms_traverse, ms_ops;
    /* milliseconds of the last evaluation, per phase (HIP events on the stream) */
    double ms_p2m, ms_m2m, ms_m2l, ms_l2l, ms_l2p, ms_p2p, ms_evaluate, ms_adjoint;
    double ms_m2l_cross;     /* cross-level M2L (ms_m2l: same-level, batched) */
    int64_t m2l_cross_keys;     /* (level difference, offset) keys of the pair list (cross-level
                                   pairs and the same-level pairs of sparse rows) with an operator */
    int64_t m2l_cross_batched;  /* pairs of that list run as shared-operator products            */
    int64_t p2p_cut_leaves;     /* leaves whose P2P list is split over several work items */
    int64_t n_m2l_sparse;       /* same-level pairs evaluated pair by pair (fmm_params.m2l_sparse) */
    int64_t m2l_rows;           /* (tile, offset) rows the batched M2L multiplies: m2l_rows x the
                                   tile width slots, of which n_m2l_same - n_m2l_sparse hold a pair */
    int64_t p2p_mutual_pairs;   /* unordered leaf pairs evaluated once for both leaves (mutual) */
} fmm_stats;

/* Host buffers for fmm_export_tree; any pointer may be NULL.  Lists are
 * (target, source) cell pairs in ascending (target, source) order.  Keys and
 * cells as in Section II.B, lists as emitted by the dual tree traversal of
 * Section II.C. */
typedef struct {
    uint64_t *keys;      /* [n] sorted Morton keys                           */
    int32_t *perm;       /* [n] sorted position -> original body index       */
    int32_t *level;      /* [ncell] cells in (level, key) order              */
    uint64_t *cell_key;  /* [ncell] key >> 3*(21 - level)                    */
    int32_t *begin, *end;/* [ncell] body range in sorted order               */
    int32_t *parent;     /* [ncell] -1 for the root                          */
    int32_t *child_begin;/* [ncell] first child (children are contiguous)    */
    int32_t *nchild;     /* [ncell]                                          */
    double *centers;     /* [3*ncell] lattice centers                        */
    int32_t *m2l;        /* [2*n_m2l]                                        */
    int32_t *p2p;        /* [2*n_p2p]                                        */
} fmm_tree_export;

/* Builds the tree, the interaction lists and the work schedule for the
 * coordinates x (N x 3, dtype).  Steps: root cube from the local bounding
 * box; 21-bit lattice coordinates and 64-bit Morton keys (Section II.B);
 * stable radix sort; cells split while they hold more than ncrit bodies;
 * lattice centers; dual tree traversal emitting M2L and P2P pairs (Section
 * II.C).  Synchronises hip_stream.  On success *out holds a plan that must be
 * released with fmm_destroy.  n == 0 gives a valid empty plan.
 * Errors: FMM_ERR_INVALID (x or out NULL with n > 0, n < 0, bad params),
 * FMM_ERR_UNSUPPORTED (n >= 2^31), FMM_ERR_NONFINITE, FMM_ERR_NOMEM,
 * FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_build(const void *x, fmm_dtype dtype, int64_t n, const fmm_params *prm,
                     const fmm_allocator *alloc, void *hip_stream, fmm_plan **out);

/* Evaluates potential and field for charges q (length N, the plan's dtype)
 * on the plan's tree: the six operators of Section II.A in the order of
 * Section II.C -- P2M and M2M (upward pass), M2L and P2P over the traversal's
 * lists, L2L and L2P (downward pass) -- then scatters the results to the
 * caller's order.  phi (length N) is required; field (N x 3) may be NULL.
 * Asynchronous on hip_stream; allocates nothing.
 * Errors: FMM_ERR_INVALID (NULL plan/q/phi), FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_evaluate_plan(fmm_plan *plan, const void *q, void *phi, void *field, void *hip_stream);

/* One call = fmm_build + fmm_evaluate_plan + fmm_destroy (Sections II.B,
 * II.C and II.A as for those calls), with the method parameters of Table I
 * given as scalars (kahan on, coarse_fp64_levels 3).  Synchronises
 * hip_stream.  Errors: those of fmm_build and fmm_evaluate_plan. */
FMM_API fmm_status fmm_evaluate(const void *x, const void *q, fmm_dtype dtype, int64_t n, int32_t p,
                        double theta, int32_t ncrit, int32_t precision, const fmm_allocator *alloc,
                        void *phi, void *field, void *hip_stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * evaluation as fmm_evaluate (build, evaluate, release), but every device
 * buffer of the plan, including the operator and stencil tables that other
 * plans cache per device, comes from one static array of
 * FMM_NOALLOC_SCRATCH_BYTES bytes that the library holds on each GPU it runs
 * on until the process ends.  The call allocates no device memory (host-side
 * bookkeeping uses the C++ heap) and returns after its work on hip_stream is
 * complete.  Calls on one device share that array and are serialised by the
 * library; calls from several threads on one device therefore never overlap,
 * but each waits for the previous one to finish.
 * Limits: n <= FMM_NOALLOC_MAX_N, else FMM_ERR_UNSUPPORTED; a tree whose plan
 * does not fit the array (deep adaptive trees, large p with small theta)
 * fails with FMM_ERR_NOMEM and a message giving the bytes in use and asked
 * for.  Uniform bodies at p <= 8, theta >= 0.4, ncrit >= 64 fit up to the
 * maximum n in either precision.
 * Other errors: those of fmm_evaluate (without the allocator's). */
#define FMM_NOALLOC_MAX_N (1 << 17)
#define FMM_NOALLOC_SCRATCH_BYTES (512ull << 20)
FMM_API fmm_status fmm_evaluate_noalloc(const void *x, const void *q, fmm_dtype dtype, int64_t n, int32_t p,
                                        double theta, int32_t ncrit, int32_t precision, void *phi, void *field,
                                        void *hip_stream);

/* Adjoint of L = sum_i w_i phi_i with w = grad_phi (the paper computes only
 * the forward potential and field of Section II.A; this is the reverse mode
 * of that computation).  The plan's lists are symmetric (the traversal of
 * Section II.C splits both cells of a pair alike), so the FMM operator is
 * symmetric and
 *     dL/dq = FMM potential with charges w,
 *     dL/dx = -(w * E^q + q * E^w)   (E^q, E^w: FMM fields of q and of w).
 * field_q is E^q from the forward call (N x 3) or NULL, in which case it is
 * recomputed on the same tree.  dq (N) and dx (N x 3) are outputs; either may
 * be NULL.  Asynchronous on hip_stream.
 * Errors: FMM_ERR_INVALID (NULL plan/q/grad_phi), FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_adjoint(fmm_plan *plan, const void *q, const void *grad_phi, const void *field_q,
                       void *dq, void *dx, void *hip_stream);

/* Statistics of fmm_let_evaluate (host struct), summed over the ordered rank
 * pairs (receiver r, sender s != r) unless stated.  let_bytes is what the
 * LETs would occupy as messages: per cell its center, side and structure
 * (40 B) and its p^2 multipole coefficients (compute type), per body its
 * coordinates and charge (32 B). */
typedef struct {
    int32_t nrank;
    int64_t let_cells;        /* cells sent                                        */
    int64_t let_far;          /* ... of them accepted against the receiver's cube   */
    int64_t let_body_leaves;  /* ... leaves sent with their bodies                  */
    int64_t let_bodies;       /* bodies sent                                       */
    int64_t let_bytes;        /* message bytes as above                             */
    int64_t n_m2l_local, n_p2p_local;                  /* each rank's own lists      */
    int64_t n_m2l_remote, n_p2p_remote, n_m2p_remote;  /* lists against grafted LETs */
    int64_t device_bytes;     /* bytes held by the ranks' plans                      */
    double ms_partition, ms_build, ms_let, ms_evaluate, ms_total;  /* host wall clock */
} fmm_let_stats;

/* The evaluation split over nrank virtual ranks on one GPU, as the paper's
 * distributed code splits it over processes (Section II.B: orthogonal
 * recursive bisection weighted by the work of Eq. (1); Section II.C: local
 * trees from local bounding boxes, the local essential tree (LET), Fig.
 * `tree').
 *   Partition: the box of a set of bodies is split across its longest side
 *   (the first of the longest on a tie), bodies taken in ascending
 *   (coordinate, index) order, the lower part getting the fewest bodies
 *   whose weight reaches floor(m/2)/m of the box's weight for m ranks (at
 *   least one body a side when there are two), recursively; weights
 *   (device, int64, 0 <= w < 2^40; NULL = all 1; all 0 in a box = 1 each)
 *   are typically l_i + alpha r_i from a previous call's work outputs.
 *   Each rank builds its own tree from its own bodies (fmm_build rules).
 *   LET of sender s for receiver r: top-down over s's cells, a cell meeting
 *   the acceptance criterion against r's whole root cube (R_B < theta d, d
 *   the distance from the cell's center to the cube) is sent with its
 *   multipole only, a leaf that does not with its bodies, any other cell is
 *   sent and opened.  Receiver r walks its tree against each grafted LET:
 *   accepted pairs (R_A + R_B < theta |c_A - c_B|) are M2L, a leaf against
 *   a sent leaf is P2P (bodies) or M2P (multipole only, evaluated at the
 *   leaf's bodies), otherwise the sent leaf splits A, a leaf A splits B, or
 *   the larger cube is split (both when equal).  Remote work is float64.
 * Outputs (device, caller's order; all but phi may be NULL): phi (N), field
 * (N x 3); rank (N, int32) of every body; work_local / work_remote (N,
 * int64) the l_i / r_i of Eq. (1) -- bodies of the leaves in the body's
 * P2P list plus cells in the M2L lists of its leaf and its leaf's
 * ancestors, over the local lists / the remote lists (M2P cells included).
 * pair_stats (HOST, nrank^2 x 11 int64, receiver-major): per (r, s != r)
 * [cells sent, multipole-only cells, body leaves, bodies, remote M2L, remote
 * P2P, M2P, three list digests, LET digest], per (r, r) [0, 0, 0, 0, local
 * M2L, local P2P, 0, local M2L digest, local P2P digest, 0, 0] (digests as
 * in fmm_list_digest; the LET digest sums mix64(cell << 8 | kind) with kind
 * 1 opened, 2 multipole only, 3 leaf with bodies).  Synchronises hip_stream.
 * Errors: FMM_ERR_INVALID (NULL x/q/phi with n > 0, nrank outside
 * [1, 1024], bad params or weights), FMM_ERR_UNSUPPORTED (n >= 2^31),
 * FMM_ERR_NONFINITE, FMM_ERR_NOMEM, FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_let_evaluate(const void *x, const void *q, fmm_dtype dtype, int64_t n, int32_t nrank,
                                    const int64_t *weights, const fmm_params *prm, const fmm_allocator *alloc,
                                    void *phi, void *field, int32_t *rank, int64_t *work_local,
                                    int64_t *work_remote, int64_t *pair_stats, fmm_let_stats *stats,
                                    void *hip_stream);

/* Copies counts and the last per-phase timings into *out (host): the
 * interaction counts of Section II.C and the phase breakdown of Section
 * III.A (event timings only when fmm_set_timing enabled them).
 * Errors: FMM_ERR_INVALID (NULL argument). */
FMM_API fmm_status fmm_plan_stats(const fmm_plan *plan, fmm_stats *out);

/* Copies the tree (Section II.B: keys, permutation, cells, centers) and the
 * canonical lists of the dual tree traversal (Section II.C) to the host
 * buffers of *out (synchronises the plan's stream).  The caller sizes the
 * buffers from fmm_plan_stats (n, ncell, n_m2l, n_p2p).
 * Errors: FMM_ERR_INVALID (NULL argument), FMM_ERR_NOMEM (host staging),
 * FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_export_tree(const fmm_plan *plan, const fmm_tree_export *out);

/* Order-independent digests of the plan's two lists (dual tree traversal,
 * Section II.C): out_host[0] for the M2L pairs (same- and cross-level),
 * out_host[1] for the P2P pairs, each the sum mod 2^64 over the pairs
 * (A <- B) of mix64(A << 32 | B), with A and B cell indices in (level, key)
 * order and mix64 the output finaliser of SplitMix64 (Steele, Lea & Flood
 * 2014).  Equal digests mean equal lists without copying them to the host.
 * out_host is a HOST array of 2 uint64.  Synchronises the plan's stream.
 * Errors: FMM_ERR_INVALID (NULL argument), FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_list_digest(const fmm_plan *plan, uint64_t *out_host);

/* Body pairs of the P2P list: the sum over P2P leaf pairs (A <- B) of
 * |A| |B| (the near-field work of Section II.A, self pairs included), into
 * *out_host (a HOST int64).  A statistic kept apart from fmm_plan_stats,
 * which reports it once counted: the count walks the whole list and
 * synchronises the plan's stream.
 * Errors: FMM_ERR_INVALID (NULL argument), FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_count_body_pairs(const fmm_plan *plan, int64_t *out_host);

/* Per-phase event timing (the breakdown of Section III.A) on (1) or off (0,
 * default).  Timing adds one event pair per phase to the stream.
 * Errors: FMM_ERR_INVALID (NULL plan). */
FMM_API fmm_status fmm_set_timing(fmm_plan *plan, int32_t on);

/* Releases the plan and its device buffers (synchronises its stream); no
 * passage of the paper.  NULL is a no-op. */
FMM_API void fmm_destroy(fmm_plan *plan);

/* Thread-local description of the last failure ("" if none); no passage of
 * the paper. */
FMM_API const char *fmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H_ */
