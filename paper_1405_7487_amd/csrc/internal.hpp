// internal.hpp -- shared declarations of the gfx950 FMM library (not installed).
//
// Layout of the data in HBM (one plan):
//   bodies   : sorted by Morton key; float4/double4 (u_x, u_y, u_z, q) with u
//              the offset from the body's leaf center (small magnitudes keep
//              float32 differences accurate deep in the tree)
//   cells    : structure of arrays in (level, key) order; a level is a
//              contiguous index range
//   coefs    : per cell P2pad = roundup(p^2, 16) reals, real solid-harmonic
//              basis scaled per level (multipole / h^n, local * h^{n+1})
//   lists    : same-level M2L as a slot table [tile][k][TW] (source cell of
//              stencil entry k for each of TW targets of one octant class);
//              cross-level M2L and P2P as CSR by target cell
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "../../include/fmm_diag.h"

namespace fmm {

constexpr int kLevels = 21;       // 64-bit Morton key: 3 bits x 21 levels
constexpr int kMaxP = 16;

struct Error : std::runtime_error {
    fmm_status code;
    Error(fmm_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define FMM_HIP(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            throw ::fmm::Error(FMM_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define FMM_CHECK(cond, code, msg)                   \
    do {                                             \
        if (!(cond)) throw ::fmm::Error(code, msg);  \
    } while (0)

inline int p2pad_of(int p) { return ((p * p + 15) / 16) * 16; }

// ------------------------------------------------- M2L operator table layout
// An operator (P2pad output rows, RT = P2pad / 16 row tiles; 4 Q input
// columns, Q input steps per k-group) is stored as NC stages of SCH input
// steps; a stage holds the 4 k-groups one after another, GST elements apart,
// each group SCH rows of P2pad values in MFMA fragment order:
//     op[(c 4 + g) GST + ss P2pad + (row % 16) RT + row / 16] = T[row][g Q + c SCH + ss].
// A stage is contiguous so that four waves copy it straight into LDS, 1 KiB
// per wave and instruction; the groups are padded apart (m2l_gst) so that the
// fragment reads of a step fall in different LDS banks.  SCH is the
// largest divisor of Q (a multiple of 4, else of 2, when one exists) whose
// stage fits 16 KiB (32 KiB for float64, whose fragments are half as long),
// i.e. SCH RT <= 64.
__host__ __device__ constexpr int m2l_sch(int RT, int Q, int esz)
{
    int b4 = 0, b2 = 0, b1 = 1;
    for (int sc = 1; sc <= Q; ++sc)
        if (Q % sc == 0 && 4 * sc * 16 * RT * esz <= (esz == 8 ? 32768 : 16384)) {
            if (sc % 4 == 0) b4 = sc;
            if (sc % 2 == 0) b2 = sc;
            b1 = sc;
        }
    return b4 ? b4 : (b2 ? b2 : b1);
}
// Input steps per k-group for order p: ceil(p^2 / 4), so that the operator
// carries no padded input columns (the MFMA needs the inputs in fours only),
// when that count has a divisor of at least 4 (or is itself small) whose
// stage fits; else 4 RT, the padded count.  p = 10: 25 steps of 4 inputs for
// 100 coefficients instead of 28.
__host__ __device__ constexpr int m2l_q(int p)
{
    const int RT = (p * p + 15) / 16, q0 = (p * p + 3) / 4;
    int best = 0;
    for (int sc = 1; sc <= q0; ++sc)
        if (q0 % sc == 0 && sc * RT <= 64) best = sc;
    return (best >= 4 || best == q0) ? q0 : 4 * RT;
}
__host__ __device__ constexpr int m2l_rt(int p) { return (p * p + 15) / 16; }
// Coefficient rows in the last row tile when there are at most 4 of them
// and p <= 10 (p = 1, 2, 6, 7, 9, 10), else 0.  In float32 such a tile runs
// as one 4x4x1 MFMA (sixteen 4x4 blocks) per step instead of a 16x16x4 one:
// its operator rows are stored as row 16 (RT - 1) + (j & 3) in fragment lane
// j, so block (g, j / 4) multiplies those rows by the inputs of k-group g for
// columns 4 (j / 4) .. + 3, a quarter of the matrix-core passes.  (At p = 14
// and 15 the same change costs the kernel half its waves per SIMD, for 5 %
// of the passes.)
__host__ __device__ constexpr int m2l_tail_rows(int p)
{
    const int v = p * p - 16 * (m2l_rt(p) - 1);
    return (p <= 10 && v >= 1 && v <= 4) ? v : 0;
}
// Whether the fragment reads of a step, lane (g, j) at word g G + j RT, fall
// in 64 different LDS banks.
__host__ __device__ constexpr bool m2l_banks_distinct(int G, int RT)
{
    bool seen[64] = {};
    for (int g = 0; g < 4; ++g)
        for (int j = 0; j < 16; ++j) {
            const int b = (g * G + j * RT) % 64;
            if (seen[b]) return false;
            seen[b] = true;
        }
    return true;
}
// Elements from one k-group of a stage to the next: SCH rows of P2pad values
// plus padding.  float32 with RT odd (fragment reads of single words): the
// smallest pad that spreads the 64 lanes' reads over 64 banks.  RT even
// keeps the groups 16-byte aligned (wide fragment reads); float64: 64 bytes
// when RT is odd.
__host__ __device__ constexpr int m2l_gst(int RT, int Q, int esz)
{
    const int base = m2l_sch(RT, Q, esz) * 16 * RT;
    if (esz == 4 && (RT & 1))
        for (int pad = 0; pad < 64; ++pad)
            if (m2l_banks_distinct(base + pad, RT)) return base + pad;
    return base + ((RT & 1) ? 64 / esz : 0);
}
// elements per operator, and the zero tail a table needs after its last operator
// (the last stage copy is rounded up to whole 4 KiB block rounds)
__host__ __device__ constexpr int64_t m2l_opsz(int RT, int Q, int esz)
{
    return (int64_t)(Q / m2l_sch(RT, Q, esz)) * 4 * m2l_gst(RT, Q, esz);
}
// rounds of WV KiB (WV waves copying 1 KiB each) that copy one stage
__host__ __device__ constexpr int m2l_rounds(int RT, int Q, int esz, int WV)
{
    return (4 * m2l_gst(RT, Q, esz) * esz + 1024 * WV - 1) / (1024 * WV);
}
__host__ __device__ constexpr int64_t m2l_tail(int RT, int Q, int esz) { return (int64_t)m2l_rounds(RT, Q, esz, 8) * 8192 / esz; }
// Tiles of the batched M2L: CG column groups of 16 targets per wave, WV waves
// per block.  Two groups per wave where the accumulators allow (float32,
// P2pad <= 64), else one; four waves (eight measured slower at P = 10 and 12).
__host__ __device__ constexpr int m2l_cg(int RT, bool f64) { return f64 ? 1 : (RT <= 4 ? 2 : 1); }
__host__ __device__ constexpr int m2l_wv(int RT, bool f64) { return 4; }

// Sum of n values p[0], p[stride], ..., in float64, in index order; eight
// loads are issued before they are added, so a thread keeps eight in flight
// (the order of the additions, hence the result, is that of a plain loop).
template <class T>
__device__ __forceinline__ double strided_sum(const T *p, int64_t n, int64_t stride)
{
    double acc = 0.0;
    int64_t k = 0;
    for (; k + 8 <= n; k += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(k + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; k < n; ++k) acc += (double)p[k * stride];
    return acc;
}

// ---------------------------------------------------------------- memory
// Device memory of a plan: the caller's callbacks, the library's caching pool,
// or (for the entry point that allocates nothing) blocks carved from a fixed
// device range: first fit over the free ranges in address order, freed blocks
// merged with their free neighbours; no fitting range is FMM_ERR_NOMEM.
struct Allocator {
    fmm_allocator user{};
    bool has_user = false;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    size_t arena_cap = 0, arena_peak = 0;
    std::map<size_t, size_t> arena_free;            // offset -> bytes
    std::map<size_t, size_t> arena_used;            // offset -> bytes
    void *alloc(size_t bytes);
    void free(void *p);
};

// A device buffer owned by a plan.
struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// ---------------------------------------------------------------- plan
struct Level {
    int64_t start = 0, count = 0;   // cells [start, start + count)
    int64_t tile0 = 0, ntile = 0;   // batched-M2L tiles of this level
};

struct Timer;

// One chunk of the batched cross-level M2L: tiles [t0, t1) cover the pairs at
// positions [p0, p1); reduction segments [s0, s1).
struct XChunk {
    int64_t t0 = 0, t1 = 0, p0 = 0, p1 = 0, s0 = 0, s1 = 0;
};

}  // namespace fmm

struct fmm_plan {
    // parameters
    int64_t n = 0;
    int p = 8, P2 = 64, P2pad = 64;
    double theta = 0.4, t4 = 0.64;
    int ncrit = 64, precision = FMM_PREC_MIXED, cfl = 3, kahan = 1;
    int tight = 0;                   // acceptance also by the cells' own radii (c_rad)
    int m2l_sparse = 0;              // slot rows below this many sources per 64 targets run as pairs
    int m2l_rotation = 0;            // every M2L pair by the O(p^3) rotation kernel
    int mutual = 0;                  // P2P: each unordered leaf pair once, both leaves updated
    double *rot_x = nullptr;         // its table d^n(pi/2), n < p
    fmm_dtype dtype = FMM_F64;
    int timing = 0;
    fmm::Allocator al;
    bool noalloc = false;            // tables that are cached per device elsewhere come from al
    std::vector<fmm::Buf> owned;
    int64_t bytes_held = 0;

    // root box
    double lo[3] = {0, 0, 0}, S = 1.0, scale = 1.0;

    // tree
    int64_t ncell = 0, nleaf = 0, ncoarse = 0;
    int depth = 0;
    std::vector<fmm::Level> lv;
    uint64_t *keys = nullptr;      // [n]
    int32_t *perm = nullptr;       // [n]
    int32_t *leaf_of = nullptr;    // [n] sorted body -> leaf cell
    int32_t *c_lvl = nullptr, *c_beg = nullptr, *c_end = nullptr, *c_par = nullptr;
    int32_t *c_cbeg = nullptr, *c_nch = nullptr;
    uint64_t *c_key = nullptr;
    int32_t *c_ix = nullptr;       // [3*ncell] lattice coords at own level
    double *c_ctr = nullptr;       // [3*ncell]
    int64_t *c_rad = nullptr;      // [ncell] radius tight to the bodies, units S 2^-22 (tight only)
    int32_t *leaves = nullptr;     // [nleaf] leaf cell indices (ascending)
    void *ubody = nullptr;         // [n] float4 or double4 (u, q)
    void *ulo = nullptr;           // [n] float4: float32 rounding residuals of ubody (mixed path)

    // lists
    int64_t n_m2l_same = 0, n_m2l_cross = 0, n_p2p = 0, p2p_body_pairs = 0;
    int64_t n_m2l_sparse = 0;  // same-level pairs moved from sparse slot rows to the pair list
    int64_t n_m2lx = 0;        // entries of the m2lx CSR: cross-level plus moved same-level pairs
    int64_t m2l_rows = 0;      // (tile, entry) rows left to the batched kernel
    unsigned long long *d_m2l_rows = nullptr;  // its device copy (plan memory)
    int64_t *p2p_off = nullptr;  int32_t *p2p_src = nullptr;   // CSR over cells
    int64_t *p2p_near = nullptr;     // [ncell + 1] end of each list's leading run of touching leaves
    // P2P work items: (leaf, list range, output); long lists are cut into items
    int64_t p2p_nitem = 0, p2p_ncut = 0, p2p_npart = 0;
    int32_t *p2p_it_leaf = nullptr;
    int64_t *p2p_it_k0 = nullptr, *p2p_it_k1 = nullptr;
    int64_t *p2p_it_out = nullptr;   // >= 0: first body index; < 0: -(partial slot) - 1
    int32_t *p2p_cl_leaf = nullptr, *p2p_cl_n = nullptr;   // cut leaves, their item counts
    int64_t *p2p_cl_part = nullptr;  // first partial slot of each cut leaf
    void *p2p_part = nullptr;        // [4 npart] partial phi, then partial E (3 per slot)
    // mutual P2P: the upper entries (source > target) of every leaf's list in
    // list order, the first slot of each entry's source-side sums, the entries
    // ordered by source, and work items over the upper entries
    int64_t mu_nup = 0, mu_nitem = 0, mu_nslot = 0, mu_nabody = 0;
    int32_t *mu_src = nullptr;       // [nup] source leaf of each upper entry
    int64_t *mu_pb = nullptr;        // [nup] first source-side slot of each upper entry
    uint64_t *mu_tkey = nullptr;     // [nup] sources ascending (stable: entries ascending within one source)
    int32_t *mu_tval = nullptr;      // [nup] the upper entry of each
    int32_t *mu_it_leaf = nullptr;   // [nitem] target leaf
    int64_t *mu_it_u = nullptr;      // [4 nitem] first entry, end of the touching run, end, first target-side slot
    int64_t *mu_li = nullptr;        // [nleaf + 1] first item of each leaf (leaf order)
    int32_t *mu_order = nullptr;     // [nitem] launch order of the items: most work first
    void *mu_bufA = nullptr;         // [nabody] target-side sums per item (phi, E) as 4-vectors
    void *mu_bufB = nullptr;         // [nslot] source-side sums per (upper entry, source body)
    int64_t *m2lx_off = nullptr; int32_t *m2lx_src = nullptr;  // cross-level M2L
    // batched same-level M2L
    int K = 0, nops = 0, R = 0;      // stencil size per class, #operators, offset radius
    int st_reach = 0;                // largest |component| of a stencil offset
    int TW = 64;                     // targets per batched-M2L tile (64 or 128)
    int E = 0;                       // stencil entries per chunk
    int NCH = 0;                     // chunks of the stencil (launched chunk after chunk)
    int G = 1;                       // chunks per launch (partial sums when > 1)
    int TPC = 0;                     // tile slots per octant class in the interleaved order
    int32_t *tile_order = nullptr;   // [8*TPC] tile in slot i (class i % 8) or -1
    std::vector<int32_t> h_tile_cls, h_tile_order;  // host copies (sources of async copies)
    int64_t ntile = 0;
    int32_t *tile_tgt = nullptr;     // [ntile*TW] target cell or -1
    int32_t *tile_cls = nullptr;     // [ntile] octant class
    int32_t *slots = nullptr;        // [ntile*K*TW] source cell or -1
    void *m2l_part = nullptr;        // [G][ntile*TW][P2pad] partial sums when G > 1
    int32_t *tile_kl = nullptr;      // [ntile][K] stencil entries with a source, per tile
    int32_t *tile_nk = nullptr;      // [ntile] length of that list
    int32_t *slot_none = nullptr;    // [TW] all -1 (source row of an entry past the list)
    uint8_t *tile_kflag = nullptr;   // [ntile][K] 1 where the entry has a source in the tile
    int32_t *st_op = nullptr;        // [8*K] operator index of stencil entry
    int32_t *st_kidx = nullptr;      // [8*(2R+1)^3] stencil entry of (class, t) or -1
    std::vector<int32_t> h_st_t;     // [8*K*3] offsets (host copy)
    std::vector<int32_t> h_ops_t;    // [nops*3]
    void *ops = nullptr;             // M2L operators, fragment layout, compute type
    // batched cross-level M2L: pairs grouped by key (level difference, offset)
    int nxk = 0;                     // keys with their own operator
    void *xops = nullptr;            // [nxk] operators, fragment layout, compute type
    int64_t nxb = 0;                 // batched pairs, in (key, target) order
    int64_t nxt = 0;                 // tiles of TW pairs of one key
    int32_t *xt_op = nullptr;        // [nxt] key of the tile
    int64_t *xt_first = nullptr;     // [nxt] position of its first pair
    int32_t *xt_cnt = nullptr;       // [nxt] pairs in the tile
    int32_t *xp_src = nullptr;       // [nxb] source cell of each batched pair
    int32_t *xr_inv = nullptr;       // [nxb] position of each pair in (chunk, target, key) order
    int64_t *xs_off = nullptr;       // [nseg + 1] segment starts in that order (one target of one chunk)
    int32_t *xs_tgt = nullptr;       // [nseg] target cell of the segment
    std::vector<fmm::XChunk> xchunks;
    void *xbuf = nullptr;            // per-pair products of one chunk
    int64_t n_gx = 0;                // cross pairs left to the generic kernel
    int64_t *gx_off = nullptr; int32_t *gx_src = nullptr;  // their CSR by target
    int64_t n_gchunk = 0;            // chunks of those pairs (a target's list split in order)
    int32_t *gx_ctgt = nullptr;      // [n_gchunk] target cell
    int64_t *gx_ck0 = nullptr;       // [n_gchunk] first pair
    int64_t *gx_cofs = nullptr;      // [ncell + 1] chunks of each cell
    double *gx_part = nullptr;       // [n_gchunk][P2pad] float64 sums of a chunk
    void *m2m_c = nullptr, *l2l_c = nullptr;   // [8][P2pad][P2pad] compute type
    double *m2m_d = nullptr, *l2l_d = nullptr; // float64 versions

    // coefficients
    void *Mc = nullptr, *Lc = nullptr;    // [(ncell+1)*P2pad] compute type; row ncell stays zero
    double *M64 = nullptr, *L64 = nullptr;// [ncoarse*P2pad]
    // evaluation outputs in sorted order, compute type
    void *phi_s = nullptr, *E_s = nullptr;    // [n], [3n]
    void *phi_s2 = nullptr, *E_s2 = nullptr;  // second right-hand side (adjoint)
    void *ubody2 = nullptr;

    // stats
    fmm_stats st{};
};

namespace fmm {

// ---------------------------------------------------------------- launchers
// sort.hip
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, Allocator &al, hipStream_t s);
void scan_exclusive_i32to64(const int32_t *in, int64_t *out, int64_t n, int64_t *total_dev, Allocator &al, hipStream_t s);
// Stable LSD sort of keys (and vals, when given) by key bits [lo_bit, bits).
// The result lands in keys, unless sorted is given and there are no values:
// then *sorted points at the sorted keys, either keys or a buffer from al
// that the caller frees.
void radix_sort_u64(uint64_t *keys, int32_t *vals, int64_t n, int bits, Allocator &al, hipStream_t s,
                    int lo_bit = 0, uint64_t **sorted = nullptr);

// tree.hip
void tree_build(fmm_plan *P, const void *x, hipStream_t s);
// traverse.hip
void traverse(fmm_plan *P, hipStream_t s);
int64_t p2p_body_pairs(fmm_plan *P, hipStream_t s);
void list_digest(fmm_plan *P, uint64_t out[2], hipStream_t s);
// expansions.hip
void make_operators(fmm_plan *P, hipStream_t s);
void make_m2l_ops(fmm_plan *P, const double4 *tr_dev, int nops, void *out, hipStream_t s);
void upward(fmm_plan *P, const void *ub, hipStream_t s);
void downward_l2l(fmm_plan *P, hipStream_t s);
void l2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s);
// m2l.hip
int m2l_tile_width(int p, bool f64);
void m2l_prepare(fmm_plan *P, hipStream_t s);
void m2l_same(fmm_plan *P, hipStream_t s);
void m2l_cross(fmm_plan *P, hipStream_t s);
void m2l_cross_prepare(fmm_plan *P, hipStream_t s);
// p2p.hip
void p2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s);
void p2p_prepare(fmm_plan *P, hipStream_t s);
// api.hip helpers
void gather_bodies(fmm_plan *P, const void *q, void *ub, hipStream_t s);
// the evaluation's phases: charges + upward pass; M2L (local expansions
// zeroed first); downward pass + P2P + L2P
void eval_up(fmm_plan *P, const void *q, void *ub, hipStream_t s);
void eval_m2l(fmm_plan *P, hipStream_t s);
void eval_down(fmm_plan *P, void *ub, void *phi_s, void *E_s, hipStream_t s);
// hands back every block an allocator still holds
// M2L by rotation (rotation.hip): the table d^n(pi/2) and the kernel over
// the plan's pair list, adding into the local expansions.
void rotation_prepare(fmm_plan *P, hipStream_t s);
void rotation_m2l(fmm_plan *P, hipStream_t s);
void allocator_done(Allocator &a);
// let.hip: the virtual-rank evaluation behind fmm_let_evaluate
void let_evaluate(const void *x, const void *q, fmm_dtype dtype, int64_t n, int R, const int64_t *w,
                  const fmm_params &prm, const fmm_allocator *ualloc, void *phi, void *field, int32_t *rank_out,
                  int64_t *work_l, int64_t *work_r, int64_t *pair_stats, fmm_let_stats *stats, hipStream_t s);

void *plan_alloc(fmm_plan *P, size_t bytes);
// One work-item per element.  A dispatch counts its work-items in 32 bits, so
// larger ranges must use grid-stride kernels instead.
inline dim3 grid1(int64_t n, int bs)
{
    const int64_t nb = (n + bs - 1) / bs;
    FMM_CHECK(nb * bs < (1ll << 32), FMM_ERR_UNSUPPORTED, "launch of more than 2^32 work-items");
    return dim3((unsigned)nb);
}

}  // namespace fmm
