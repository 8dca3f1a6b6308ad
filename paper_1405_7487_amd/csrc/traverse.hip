// traverse.hip -- dual tree traversal on gfx950 (Section II.C of the paper,
// after Dehnen 2002).
//
// The walk starts from the pair (root, root).  A pair whose cells satisfy the
// acceptance criterion R_A + R_B < theta |c_A - c_B| becomes an M2L pair; a
// pair of two leaves becomes a P2P pair; otherwise the coarser cell is split
// (both when they share a level; a leaf is never split).  The rule treats
// both sides alike, so every list is symmetric.
//
// The GPU walks the pair frontier one generation at a time: each frontier
// pair expands into its child pairs, which are classified at once; counts,
// scan and write passes keep the output deterministic.  Unlike the paper's
// code, which never forms lists, the lists are materialised here so that the
// translation work can be regrouped:
//   * same-level M2L pairs go to a slot table.  For a target of octant class c
//     (its position inside its parent) the offsets t = i_A - i_B of its
//     same-level sources form a fixed stencil S_c, the same at every level;
//     slot [tile][k][lane] holds the source of stencil entry k of the lane's
//     target, or -1;
//   * cross-level M2L pairs and P2P pairs are sorted into CSR by target.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <array>
#include <map>
#include <mutex>

namespace fmm {

namespace {

// Exact acceptance test on the lattice of half-units of the finer cell:
// 3 (s_A + s_B)^2 < (4 theta^2) * D^2 with sides s = 2^{f-l+1} and center
// coordinates 2^{f-l} (2 i + 1), D^2 the squared distance of the centers.
__device__ __forceinline__ bool mac_dev(int la, int ax, int ay, int az, int lb, int bx, int by, int bz, double t4)
{
#pragma clang fp contract(off)
    const int f = la > lb ? la : lb;
    const int64_t sa = 1ll << (f - la + 1), sb = 1ll << (f - lb + 1);
    const int64_t dx = ((2ll * ax + 1) << (f - la)) - ((2ll * bx + 1) << (f - lb));
    const int64_t dy = ((2ll * ay + 1) << (f - la)) - ((2ll * by + 1) << (f - lb));
    const int64_t dz = ((2ll * az + 1) << (f - la)) - ((2ll * bz + 1) << (f - lb));
    const int64_t d2 = dx * dx + dy * dy + dz * dz;
    const double lhs = (double)(3 * (sa + sb) * (sa + sb));
    return lhs < t4 * (double)d2;
}

struct TreeView {
    const int32_t *lvl, *nch, *cbeg, *ix;
    const int64_t *rad;       // radii tight to the bodies (tight criterion) or null
    const uint64_t *key;
    const int32_t *tile_pos;  // cell -> tile*64 + lane (or -1)
    const int32_t *kidx;      // [8][(2R+1)^3]
    int32_t *slots;
    uint8_t *kflag;  // [ntile][K]: sources of the entry in the tile (set after the traversal)
    int K, R, TW;
    double t4;
};

// A cell as the expansion kernels see it: level, lattice coordinates at that
// level and child count.
struct CellG {
    int l, x, y, z, n;
    int64_t r;  // tight radius (units S 2^-22), or -1 without the tight criterion
};

__device__ __forceinline__ CellG load_cell(const TreeView &T, int c)
{
    CellG g;
    g.l = T.lvl[c];
    g.x = T.ix[3 * c];
    g.y = T.ix[3 * c + 1];
    g.z = T.ix[3 * c + 2];
    g.n = T.nch[c];
    g.r = T.rad ? T.rad[c] : -1;
    return g;
}

// The criterion with the cells' own radii about their lattice centers, in
// units u = S 2^-22 (centers at (2 i + 1) 2^(21 - l) u):
// 4 (r_A + r_B)^2 < (4 theta^2) D^2, all integers below 2^53.
__device__ __forceinline__ bool mac_tight(const CellG &A, const CellG &B, double t4)
{
#pragma clang fp contract(off)
    const int64_t dx = ((2ll * A.x + 1) << (kLevels - A.l)) - ((2ll * B.x + 1) << (kLevels - B.l));
    const int64_t dy = ((2ll * A.y + 1) << (kLevels - A.l)) - ((2ll * B.y + 1) << (kLevels - B.l));
    const int64_t dz = ((2ll * A.z + 1) << (kLevels - A.l)) - ((2ll * B.z + 1) << (kLevels - B.l));
    const int64_t d2 = dx * dx + dy * dy + dz * dz;
    const int64_t rs = A.r + B.r;
    return (double)(4 * rs * rs) < t4 * (double)d2;
}

// Classification of one child pair: 0 = same-level M2L, 1 = cross-level M2L,
// 2 = P2P, 3 = split further.  For two cells of one level the lattice test
// reduces to sides 2 and center differences 2 (i_A - i_B): the same integers,
// hence the same decision, as the general form.
__device__ __forceinline__ int classify(const CellG &A, const CellG &B, double t4)
{
#pragma clang fp contract(off)
    bool acc;
    if (A.l == B.l) {
        const int64_t dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
        acc = 48.0 < t4 * (double)(4 * (dx * dx + dy * dy + dz * dz));
    } else {
        acc = mac_dev(A.l, A.x, A.y, A.z, B.l, B.x, B.y, B.z, t4);
    }
    if (!acc && A.r >= 0) acc = mac_tight(A, B, t4);
    if (acc) return A.l == B.l ? 0 : 1;
    if (A.n == 0 && B.n == 0) return 2;
    return 3;
}

// Whether the cubes of two cells share at least a corner: along each axis
// their extents, in units of the finer cell's side, overlap or abut.
__device__ __forceinline__ bool touching(const CellG &A, const CellG &B)
{
    const int f = A.l > B.l ? A.l : B.l;
    const int64_t sa = 1ll << (f - A.l), sb = 1ll << (f - B.l);
    const int64_t a[3] = {A.x, A.y, A.z}, b[3] = {B.x, B.y, B.z};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (a[d] * sa > (b[d] + 1) * sb || b[d] * sb > (a[d] + 1) * sa) return false;
    return true;
}

// The split rule of the traversal for a pair that was not accepted and is
// not two leaves.
__device__ __forceinline__ void split_rule(const CellG &A, const CellG &B, bool &sa, bool &sb)
{
    const bool leafa = A.n == 0, leafb = B.n == 0;
    if (leafa) { sa = false; sb = true; }
    else if (leafb) { sa = true; sb = false; }
    else if (A.l < B.l) { sa = true; sb = false; }
    else if (B.l < A.l) { sa = false; sb = true; }
    else { sa = true; sb = true; }
}

// Child pairs of frontier pair (a, b): the source side's (at most 8) cells are
// loaded into registers once; the target side's one at a time.  The visiting
// order (target child outer, source child inner) fixes the order of the
// emitted pairs.
struct Expansion {
    int na, nb, a0, b0;
    CellG ys[8];
};

__device__ __forceinline__ void expansion(const TreeView &T, int a, int b, Expansion &E)
{
    const CellG A = load_cell(T, a), B = load_cell(T, b);
    bool sa, sb;
    split_rule(A, B, sa, sb);
    E.na = sa ? A.n : 1;
    E.nb = sb ? B.n : 1;
    E.a0 = sa ? T.cbeg[a] : a;
    E.b0 = sb ? T.cbeg[b] : b;
#pragma unroll
    for (int v = 0; v < 8; ++v)
        if (v < E.nb) E.ys[v] = sb ? load_cell(T, E.b0 + v) : B;
}

__global__ __launch_bounds__(256) void k_expand_count(TreeView T, const int2 *F, int64_t nf, int32_t *c_cross,
                                                      int32_t *c_p2p, int32_t *c_next, unsigned long long *n_same)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    Expansion E;
    expansion(T, F[i].x, F[i].y, E);
    int cx = 0, cp = 0, cn = 0, cs = 0;
    for (int u = 0; u < E.na; ++u) {
        const CellG X = load_cell(T, E.a0 + u);
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (v < E.nb) {
                const int k = classify(X, E.ys[v], T.t4);
                cs += k == 0;
                cx += k == 1;
                cp += k == 2;
                cn += k == 3;
            }
    }
    c_cross[i] = cx;
    c_p2p[i] = cp;
    c_next[i] = cn;
    if (cs) atomicAdd(n_same, (unsigned long long)cs);
}

__global__ __launch_bounds__(256) void k_expand_write(TreeView T, const int2 *F, int64_t nf, const int64_t *o_cross,
                                                      const int64_t *o_p2p, const int64_t *o_next, uint64_t *cross,
                                                      uint64_t *p2p, int2 *next, int cbits, int *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    Expansion E;
    expansion(T, F[i].x, F[i].y, E);
    // one scan covers the three count arrays back to back: each list's
    // offsets start at its own first entry
    int64_t ox = o_cross[i] - o_cross[0], op = o_p2p[i] - o_p2p[0], on = o_next[i] - o_next[0];
    const int W = 2 * T.R + 1;
    for (int u = 0; u < E.na; ++u) {
        const int x = E.a0 + u;
        const CellG X = load_cell(T, x);
        const int cls = (int)(T.key[x] & 7u);
        const int pos = T.tile_pos[x];
        const int64_t tile = pos / T.TW, lane = pos % T.TW;
        const int32_t *kx = T.kidx + cls * W * W * W;
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (v < E.nb) {
                const CellG &Y = E.ys[v];
                const int y = E.b0 + v;
                const int k = classify(X, Y, T.t4);
                if (k == 0) {
                    const int tx = X.x - Y.x, ty = X.y - Y.y, tz = X.z - Y.z;
                    int kk = -1;
                    if (abs(tx) <= T.R && abs(ty) <= T.R && abs(tz) <= T.R)
                        kk = kx[((tx + T.R) * W + (ty + T.R)) * W + (tz + T.R)];
                    if (kk < 0 || pos < 0) atomicOr(err, 1);
                    else T.slots[(tile * T.K + kk) * T.TW + lane] = y;
                } else if (k == 1) {
                    cross[ox++] = ((uint64_t)x << cbits) | (uint64_t)y;
                } else if (k == 2) {
                    // a bit below the target orders the sources of leaves that
                    // touch the target first (they get compensated offsets)
                    const uint64_t far = touching(X, Y) ? 0u : 1u;
                    p2p[op++] = ((uint64_t)x << (cbits + 1)) | (far << cbits) | (uint64_t)y;
                } else {
                    next[on++] = make_int2(x, y);
                }
            }
    }
}

// Totals of the three lists from the scan over their concatenated counts.
__global__ void k_list_totals(const int64_t *offs, int64_t nf, int64_t *tot)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t all = tot[3];
        tot[0] = offs[nf];
        tot[1] = offs[2 * nf] - offs[nf];
        tot[2] = all - offs[2 * nf];
    }
}

// Squared radius of every cell tight to its bodies: a body's lattice cell
// (side 2 in units u = S 2^-22) has its farthest corner from a cell's
// center (2 i + 1) 2^(21 - l) at sum_d max(|2 v_d - C_d|, |2 v_d + 2 - C_d|)^2;
// each body raises the maximum of its leaf and of every ancestor.
// Level by level from the deepest: the lanes of a wave hold consecutive
// sorted bodies, so their ancestors at one level are non-decreasing across
// the lanes; a segmented maximum over lanes with the same ancestor leaves one
// atomic per (wave, cell), skipped when it cannot raise the value.
__global__ __launch_bounds__(256) void k_tight_r2(const uint64_t *keys, const int32_t *leaf_of, const int32_t *par,
                                                  const int32_t *lvl, const int32_t *ix, int64_t n, int depth,
                                                  unsigned long long *r2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool act = i < n;
    int64_t v[3] = {0, 0, 0};
    int c = -1;
    if (act) {
        const uint64_t k = keys[i];
        for (int b = 0; b < kLevels; ++b)
            for (int d = 0; d < 3; ++d) v[d] |= (int64_t)((k >> (3 * b + 2 - d)) & 1ull) << b;
        c = leaf_of[i];
    }
    for (int l = depth; l >= 0; --l) {
        // this lane's cell at level l (its leaf may be coarser: then none yet)
        const int a = (c >= 0 && lvl[c] == l) ? c : -1;
        unsigned long long s = 0;
        if (a >= 0) {
            for (int d = 0; d < 3; ++d) {
                const int64_t C = (2ll * ix[3 * a + d] + 1) << (kLevels - l);
                const int64_t lo = 2 * v[d] - C, hi = 2 * v[d] + 2 - C;
                const int64_t m = max(lo < 0 ? -lo : lo, hi < 0 ? -hi : hi);
                s += (unsigned long long)(m * m);
            }
        }
        // segmented maximum towards the first lane of each run of equal a
        for (int w = 1; w < 64; w <<= 1) {
            const unsigned long long so = __shfl_down(s, w, 64);
            const int ao = __shfl_down(a, w, 64);
            if (lane + w < 64 && ao == a && so > s) s = so;
        }
        const int ap = __shfl_up(a, 1, 64);
        if (a >= 0 && (lane == 0 || ap != a) && s > r2[a]) atomicMax(&r2[a], s);
        if (a >= 0) c = par[a];
    }
}

// r = the smallest integer with r^2 >= r2 (exact; the float64 root is only a start)
__global__ __launch_bounds__(256) void k_tight_rad(const unsigned long long *r2, int64_t nc, int64_t *rad)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int64_t v = (int64_t)r2[c];
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r < v) ++r;
    while (r > 0 && (r - 1) * (r - 1) >= v) --r;
    rad[c] = r;
}

// Tile order keys: level and octant class (the tiles; bits 16 and up), then,
// inside a class, the cell's place relative to the faces of the root box
// along each axis -- its distance to the nearer face when below CAP, signed by
// face, else CAP; three digits of base 2 CAP + 1 -- and finally Morton order
// (the cell order, kept by the stable sort).  Cells
// that share these face classes have sources at the same stencil entries, so
// grouping them leaves fewer empty target columns in the batched products.
__device__ __forceinline__ uint32_t face_class(int v, int n, int cap)
{
    if (v < cap) return (uint32_t)v;
    if (n - 1 - v < cap) return (uint32_t)(2 * cap - (n - 1 - v));
    return (uint32_t)cap;
}

__global__ __launch_bounds__(256) void k_class_keys(const int32_t *lvl, const uint64_t *key, const int32_t *ix,
                                                    int64_t nc, int cap, uint64_t *ck, int32_t *idx, int32_t *cnt)
{
    __shared__ int32_t h[(kLevels + 1) * 8];
    for (int t = threadIdx.x; t < (kLevels + 1) * 8; t += blockDim.x) h[t] = 0;
    __syncthreads();
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc) {
        const int l = lvl[c];
        const int g = l * 8 + (int)(key[c] & 7u);
        const int n = 1 << l;
        const uint32_t F = 2 * cap + 1;
        const uint32_t code = (face_class(ix[3 * c], n, cap) * F + face_class(ix[3 * c + 1], n, cap)) * F +
                              face_class(ix[3 * c + 2], n, cap);
        ck[c] = ((uint64_t)g << 16) | code;
        idx[c] = (int32_t)c;
        atomicAdd(&h[g], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < (kLevels + 1) * 8; t += blockDim.x)
        if (h[t]) atomicAdd(&cnt[t], h[t]);
}

__global__ __launch_bounds__(256) void k_fill_tiles(const uint64_t *ck, const int32_t *idx, int64_t nc,
                                                    const int64_t *gstart, const int64_t *gtile, int TW,
                                                    int32_t *tile_tgt, int32_t *tile_pos)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nc) return;
    const int g = (int)(ck[j] >> 16);
    const int c = idx[j];
    if (gtile[g] < 0) {  // level 0: no same-level partner
        tile_pos[c] = -1;
        return;
    }
    const int64_t r = j - gstart[g];
    const int64_t p = (gtile[g] + r / TW) * TW + r % TW;
    tile_tgt[p] = c;
    tile_pos[c] = (int32_t)p;
}

// Grid-stride fill: the slot table can hold more than 2^32 entries, beyond
// what one dispatch can cover with one work-item per entry.
__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

dim3 grid_fill(int64_t n) { return dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16)); }

// CSR offsets: off[c] = first position whose key is >= (c << shift) | low.
__global__ __launch_bounds__(256) void k_csr_offsets(const uint64_t *keys, int64_t np, int shift, uint64_t low,
                                                     int64_t nc, int64_t *off)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc) return;
    const uint64_t want = ((uint64_t)c << shift) | low;
    int64_t lo = 0, hi = np;
    while (lo < hi) {
        int64_t m = lo + ((hi - lo) >> 1);
        if (keys[m] < want) lo = m + 1;
        else hi = m;
    }
    off[c] = lo;
}

__global__ __launch_bounds__(256) void k_csr_sources(const uint64_t *keys, int64_t np, int cbits, int32_t *src)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < np) src[k] = (int32_t)(keys[k] & ((1ull << cbits) - 1));
}

// Body pairs of one target's list: |A| * sum_B |B| (one thread per cell).
// |A| * sum over A's P2P sources of |B|, one wave per cell (lists reach
// thousands of entries in dense regions, so lanes share a list).
__global__ __launch_bounds__(256) void k_body_pairs(const int64_t *off, const int32_t *src, const int32_t *beg,
                                                    const int32_t *end, int64_t nc, int64_t *out)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= nc) return;
    long long s = 0;
    for (int64_t k = off[c] + lane; k < off[c + 1]; k += 64) s += end[src[k]] - beg[src[k]];
    for (int w = 32; w >= 1; w >>= 1) s += __shfl_xor(s, w, 64);
    if (lane == 0) out[c] = (int64_t)s * (int64_t)(end[c] - beg[c]);
}

// List digests: the sum, mod 2^64, of mix64(target << 32 | source) over the
// pairs, mix64 being the output finaliser of SplitMix64 (Steele, Lea & Flood
// 2014).  Integer addition commutes, so the result is the same for any order
// of the pairs or of the atomic adds.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_digest_slots(const int32_t *slots, const int32_t *tile_tgt, int64_t nslot,
                                                      int K, int TW, unsigned long long *out)
{
    uint64_t h = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslot; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t sv = slots[i];
        if (sv < 0) continue;
        const int64_t tile = i / ((int64_t)K * TW);
        const int32_t tg = tile_tgt[tile * TW + (int)(i % TW)];
        if (tg >= 0) h += mix64(((uint64_t)(uint32_t)tg << 32) | (uint32_t)sv);
    }
    atomicAdd(out, (unsigned long long)h);
}

__global__ __launch_bounds__(256) void k_digest_csr(const int64_t *off, const int32_t *src, int64_t nc,
                                                    unsigned long long *out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    uint64_t h = 0;
    for (int64_t k = off[c]; k < off[c + 1]; ++k) h += mix64(((uint64_t)(uint32_t)c << 32) | (uint32_t)src[k]);
    atomicAdd(out, (unsigned long long)h);
}

// Same-level acceptance as the traversal evaluates it (equal sides: s = 2,
// D = 2 |t| in half-units).
bool mac_same_level(int64_t t2, double t4) { return 48.0 < t4 * (double)(4 * t2); }

int ceil_div2(int v) { return (v >= 0) ? (v + 1) / 2 : -((-v) / 2); }

}  // namespace

// The stencils S_c depend only on theta; they are computed once per device
// and kept for the life of the process.
namespace {
struct StencilCache {
    int K = 0, R = 0, nops = 0, reach = 0;
    std::vector<int32_t> ops_t, st_t;
    int32_t *d_op = nullptr, *d_kidx = nullptr;
};
std::mutex g_stencil_mu;
std::map<std::tuple<int, uint64_t, int>, StencilCache> g_stencils;

// Host part: the stencils, and the device tables' contents in op and kidx.
// An offset t is in S_c when the parents' offset fails the cube criterion
// (else the pair is never reached) and, without the tight criterion, t itself
// passes it; with the tight criterion any t != 0 can pass.
StencilCache make_stencils(double t4, int tight, std::vector<int32_t> &op, std::vector<int32_t> &kidx)
{
    StencilCache C;
    // parent offsets that fail the criterion satisfy |T|^2 <= 12 / t4
    const int rT = (int)std::floor(std::sqrt(12.0 / t4)) + 1;
    const int R = 2 * rT + 1;
    std::vector<std::vector<std::array<int, 3>>> S(8);
    std::map<std::array<int, 3>, int> uni;
    for (int c = 0; c < 8; ++c) {
        const int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
        for (int tx = -R; tx <= R; ++tx)
            for (int ty = -R; ty <= R; ++ty)
                for (int tz = -R; tz <= R; ++tz) {
                    const int64_t t2 = (int64_t)tx * tx + (int64_t)ty * ty + (int64_t)tz * tz;
                    if (tight ? t2 == 0 : !mac_same_level(t2, t4)) continue;
                    const int Tx = ceil_div2(tx - cx), Ty = ceil_div2(ty - cy), Tz = ceil_div2(tz - cz);
                    if (mac_same_level((int64_t)Tx * Tx + (int64_t)Ty * Ty + (int64_t)Tz * Tz, t4)) continue;
                    S[c].push_back({tx, ty, tz});
                    uni[{tx, ty, tz}] = 0;
                    C.reach = std::max({C.reach, std::abs(tx), std::abs(ty), std::abs(tz)});
                }
    }
    int id = 0;
    for (auto &kv : uni) {
        kv.second = id++;
        C.ops_t.insert(C.ops_t.end(), kv.first.begin(), kv.first.end());
    }
    size_t K = 0;
    for (int c = 0; c < 8; ++c) K = std::max(K, S[c].size());
    C.K = (int)K;
    C.R = R;
    C.nops = id;
    // stencil entries in lexicographic offset order (= operator order), so
    // that all classes sweep the operator table alike
    op.assign(std::max<size_t>(1, 8 * K), -1);
    kidx.assign((size_t)8 * (2 * R + 1) * (2 * R + 1) * (2 * R + 1), -1);
    C.st_t.assign(8 * K * 3, 0);
    const int W = 2 * R + 1;
    for (int c = 0; c < 8; ++c) {
        std::sort(S[c].begin(), S[c].end());
        for (size_t k = 0; k < S[c].size(); ++k) {
            const auto &t = S[c][k];
            op[c * K + k] = uni[t];
            for (int d = 0; d < 3; ++d) C.st_t[(c * K + k) * 3 + d] = t[d];
            kidx[(size_t)c * W * W * W + ((t[0] + R) * W + (t[1] + R)) * W + (t[2] + R)] = (int32_t)k;
        }
    }
    return C;
}

// Stencils with their device tables, cached per (device, theta).
StencilCache make_stencils_cached(double t4, int tight)
{
    std::vector<int32_t> op, kidx;
    StencilCache C = make_stencils(t4, tight, op, kidx);
    FMM_HIP(hipMalloc(&C.d_op, sizeof(int32_t) * op.size()));
    FMM_HIP(hipMalloc(&C.d_kidx, sizeof(int32_t) * kidx.size()));
    FMM_HIP(hipMemcpy(C.d_op, op.data(), sizeof(int32_t) * op.size(), hipMemcpyHostToDevice));
    FMM_HIP(hipMemcpy(C.d_kidx, kidx.data(), sizeof(int32_t) * kidx.size(), hipMemcpyHostToDevice));
    return C;
}
}  // namespace

static void build_stencils(fmm_plan *P, hipStream_t s)
{
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    uint64_t bits;
    std::memcpy(&bits, &P->t4, sizeof(bits));
    StencilCache own;
    const StencilCache *Cp = nullptr;
    std::unique_lock<std::mutex> lk(g_stencil_mu, std::defer_lock);
    if (P->noalloc) {
        // a plan that may not allocate keeps its own copy of the tables
        std::vector<int32_t> op, kidx;
        own = make_stencils(P->t4, P->tight, op, kidx);
        own.d_op = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * op.size()));
        own.d_kidx = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * kidx.size()));
        FMM_HIP(hipMemcpyAsync(own.d_op, op.data(), sizeof(int32_t) * op.size(), hipMemcpyHostToDevice, s));
        FMM_HIP(hipMemcpyAsync(own.d_kidx, kidx.data(), sizeof(int32_t) * kidx.size(), hipMemcpyHostToDevice, s));
        FMM_HIP(hipStreamSynchronize(s));
        Cp = &own;
    } else {
        lk.lock();
        auto key = std::make_tuple(dev, bits, P->tight);
        auto it = g_stencils.find(key);
        if (it == g_stencils.end()) it = g_stencils.emplace(key, make_stencils_cached(P->t4, P->tight)).first;
        Cp = &it->second;
    }
    const StencilCache &C = *Cp;
    P->K = C.K;
    P->R = C.R;
    P->st_reach = C.reach;
    P->nops = C.nops;
    P->h_ops_t = C.ops_t;
    P->h_st_t = C.st_t;
    P->st_op = C.d_op;
    P->st_kidx = C.d_kidx;
}

static int bits_for(int64_t v)
{
    int b = 1;
    while ((1ll << b) <= v) ++b;
    return b;
}

// Keys are target << (cbits + obits) | order bits << cbits | source.  With
// one order bit (P2P), near_end[c] is where target c's entries with the bit
// set begin.
static void sort_to_csr(fmm_plan *P, uint64_t *keys, int64_t np, int cbits, int obits, int64_t **off,
                        int32_t **src, int64_t **near_end, int64_t *body_pairs_dev, hipStream_t s)
{
    // grouped by target (and order bits) only: within a group the pairs keep
    // the traversal's order, which is fixed, so the lists are deterministic
    uint64_t *const in = keys;
    uint64_t *sk = nullptr;  // the sorted keys: keys, or the sort's own buffer
    radix_sort_u64(keys, nullptr, np, 2 * cbits + obits, P->al, s, cbits, &sk);
    keys = sk;
    *off = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * (P->ncell + 1)));
    *src = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, np)));
    k_csr_offsets<<<grid1(P->ncell + 1, 256), 256, 0, s>>>(keys, np, cbits + obits, 0, P->ncell, *off);
    FMM_HIP(hipGetLastError());
    if (near_end) {
        *near_end = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * (P->ncell + 1)));
        k_csr_offsets<<<grid1(P->ncell + 1, 256), 256, 0, s>>>(keys, np, cbits + obits, 1ull << cbits, P->ncell,
                                                               *near_end);
        FMM_HIP(hipGetLastError());
    }
    if (np > 0) {
        k_csr_sources<<<grid1(np, 256), 256, 0, s>>>(keys, np, cbits, *src);
        FMM_HIP(hipGetLastError());
    }
    if (body_pairs_dev) {
        int64_t *per = static_cast<int64_t *>(P->al.alloc(sizeof(int64_t) * P->ncell));
        int64_t *scn = static_cast<int64_t *>(P->al.alloc(sizeof(int64_t) * P->ncell));
        k_body_pairs<<<grid1(P->ncell * 64, 256), 256, 0, s>>>(*off, *src, P->c_beg, P->c_end, P->ncell, per);
        FMM_HIP(hipGetLastError());
        scan_exclusive_i64(per, scn, P->ncell, body_pairs_dev, P->al, s);
        P->al.free(scn);
        P->al.free(per);
    }
    if (sk != in) P->al.free(sk);
}

// Sum over P2P pairs of |A| |B| (a statistic; computed when asked for).
int64_t p2p_body_pairs(fmm_plan *P, hipStream_t s)
{
    if (P->p2p_body_pairs >= 0 || P->ncell == 0) return std::max<int64_t>(0, P->p2p_body_pairs);
    int64_t *per = static_cast<int64_t *>(P->al.alloc(sizeof(int64_t) * P->ncell));
    int64_t *scn = static_cast<int64_t *>(P->al.alloc(sizeof(int64_t) * P->ncell));
    int64_t *tot = static_cast<int64_t *>(P->al.alloc(sizeof(int64_t)));
    k_body_pairs<<<grid1(P->ncell * 64, 256), 256, 0, s>>>(P->p2p_off, P->p2p_src, P->c_beg, P->c_end, P->ncell, per);
    FMM_HIP(hipGetLastError());
    scan_exclusive_i64(per, scn, P->ncell, tot, P->al, s);
    int64_t h = 0;
    FMM_HIP(hipMemcpyAsync(&h, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    P->al.free(tot);
    P->al.free(scn);
    P->al.free(per);
    P->p2p_body_pairs = h;
    return h;
}

// Sparse rows of the slot table.  A row is one stencil entry of one tile: the
// batched M2L multiplies it for all TW targets of the tile, so a row whose
// sources are few costs nearly as much as a full one.
// Pass 1 streams the table, 4 slots per lane (TW / 4 lanes per row): each
// row's source count goes to its flag byte (0 for an empty row), and, when
// spc is given, spc[r] = the count if 0 < count * 64 < thr * TW (a sparse
// row), else 0.  An
// exclusive scan of spc gives each sparse row its first output position.
// Pass 2, 64 rows per wave, moves the pairs of each sparse row to out, in row
// then lane order, as pair-list keys (target << cbits | source) and clears
// the row (slots -1, flag 0).  No atomics: the output is the same on every
// run.
__global__ __launch_bounds__(256) void k_sparse_count(const int4 *slots4, uint8_t *kflag, int64_t nrow, int TW,
                                                      int thr, int32_t *spc)
{
    const int lane = threadIdx.x & 63;
    const int LPR = TW >> 2;  // lanes per row (16 or 32)
    const int64_t n4 = nrow * LPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane of a wave runs the same trip count
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; i < n4; i += stride) {
        const int64_t k = i + lane;
        int o = 0;
        if (k < n4) {
            const int4 v = slots4[k];
            o = (v.x >= 0) + (v.y >= 0) + (v.z >= 0) + (v.w >= 0);
        }
        for (int w = 1; w < LPR; w <<= 1) o += __shfl_xor(o, w, 64);
        if (k < n4 && (lane & (LPR - 1)) == 0) {
            const int64_t r = k / LPR;
            kflag[r] = (uint8_t)o;
            if (spc) spc[r] = (o > 0 && o * 64 < thr * TW) ? o : 0;
        }
    }
}

template <int TWC>
__global__ __launch_bounds__(256) void k_sparse_move(int32_t *slots, uint8_t *kflag, const int32_t *tile_tgt,
                                                     const int32_t *spc, const int64_t *off, int64_t nrow, int K,
                                                     int cbits, uint64_t *out)
{
    constexpr int TW = 64 * TWC;
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r0 = w0 * 64; r0 < nrow; r0 += nw * 64) {
        const int64_t rl = r0 + lane;
        const int c_l = rl < nrow ? spc[rl] : 0;
        const int64_t o_l = c_l ? off[rl] : 0;
        uint64_t todo = __ballot(c_l > 0);
        while (todo) {
            const int jl = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int64_t r = r0 + jl, tile = r / K;
            unsigned long long base = (unsigned long long)__shfl(o_l, jl, 64);
            int32_t *row = slots + r * TW;
#pragma unroll
            for (int c = 0; c < TWC; ++c) {
                const int32_t sv = row[64 * c + lane];
                const uint64_t m = __ballot(sv >= 0);
                if (sv >= 0) {
                    const int32_t tg = tile_tgt[tile * TW + 64 * c + lane];
                    out[base + __popcll(m & ((1ull << lane) - 1))] = ((uint64_t)tg << cbits) | (uint64_t)sv;
                    row[64 * c + lane] = -1;
                }
                base += __popcll(m);
            }
            if (lane == 0) kflag[r] = 0;
        }
    }
}

// Digests of the M2L list (same-level slots and cross-level CSR) and of the
// P2P list; synchronises the stream.
void list_digest(fmm_plan *P, uint64_t out[2], hipStream_t s)
{
    out[0] = out[1] = 0;
    if (P->ncell == 0) return;
    unsigned long long *d = static_cast<unsigned long long *>(P->al.alloc(2 * sizeof(unsigned long long)));
    FMM_HIP(hipMemsetAsync(d, 0, 2 * sizeof(unsigned long long), s));
    const int64_t nslot = P->ntile * (int64_t)P->K * P->TW;
    if (nslot > 0) {
        k_digest_slots<<<2048, 256, 0, s>>>(P->slots, P->tile_tgt, nslot, P->K, P->TW, d);
        FMM_HIP(hipGetLastError());
    }
    if (P->m2lx_off) {
        k_digest_csr<<<grid1(P->ncell, 256), 256, 0, s>>>(P->m2lx_off, P->m2lx_src, P->ncell, d);
        FMM_HIP(hipGetLastError());
    }
    if (P->p2p_off) {
        k_digest_csr<<<grid1(P->ncell, 256), 256, 0, s>>>(P->p2p_off, P->p2p_src, P->ncell, d + 1);
        FMM_HIP(hipGetLastError());
    }
    unsigned long long h[2] = {0, 0};
    FMM_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    P->al.free(d);
    out[0] = h[0];
    out[1] = h[1];
}

void traverse(fmm_plan *P, hipStream_t s)
{
    Allocator &al = P->al;
    const int64_t nc = P->ncell;
    build_stencils(P, s);
    if (P->tight) {
        unsigned long long *r2 = static_cast<unsigned long long *>(al.alloc(sizeof(unsigned long long) * nc));
        FMM_HIP(hipMemsetAsync(r2, 0, sizeof(unsigned long long) * nc, s));
        k_tight_r2<<<grid1(P->n, 256), 256, 0, s>>>(P->keys, P->leaf_of, P->c_par, P->c_lvl, P->c_ix, P->n, P->depth,
                                                    r2);
        FMM_HIP(hipGetLastError());
        P->c_rad = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * nc));
        k_tight_rad<<<grid1(nc, 256), 256, 0, s>>>(r2, nc, P->c_rad);
        FMM_HIP(hipGetLastError());
        al.free(r2);
    }

    // Octant-class tiles per level (levels >= 1).
    const int G = (kLevels + 1) * 8;
    uint64_t *ck = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * nc));
    int32_t *idx = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nc));
    int32_t *gcnt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * G));
    FMM_HIP(hipMemsetAsync(gcnt, 0, sizeof(int32_t) * G, s));
    // face classes are capped one cell short of the stencil's reach
    const int cap = std::max(1, P->st_reach - 1);
    FMM_CHECK((int64_t)(2 * cap + 1) * (2 * cap + 1) * (2 * cap + 1) <= 65536, FMM_ERR_UNSUPPORTED,
              "traversal: stencil reach too large");
    FMM_CHECK(G <= 256, FMM_ERR_UNSUPPORTED, "traversal: too many levels");
    k_class_keys<<<grid1(nc, 256), 256, 0, s>>>(P->c_lvl, P->c_key, P->c_ix, nc, cap, ck, idx, gcnt);
    FMM_HIP(hipGetLastError());
    radix_sort_u64(ck, idx, nc, 24, al, s);
    std::vector<int32_t> hcnt(G);
    FMM_HIP(hipMemcpyAsync(hcnt.data(), gcnt, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> gstart(G), gtile(G);
    int64_t acc = 0, tiles = 0;
    for (int g = 0; g < G; ++g) {
        gstart[g] = acc;
        acc += hcnt[g];
        const int l = g / 8;
        if (l == 0 || hcnt[g] == 0) {
            gtile[g] = -1;
            continue;
        }
        gtile[g] = tiles;
        tiles += (hcnt[g] + P->TW - 1) / P->TW;
    }
    for (int l = 0; l <= P->depth; ++l) {
        P->lv[l].tile0 = (l == 0) ? 0 : -1;
        P->lv[l].ntile = 0;
        for (int c = 0; c < 8; ++c) {
            const int g = l * 8 + c;
            if (gtile[g] < 0) continue;
            if (P->lv[l].tile0 < 0) P->lv[l].tile0 = gtile[g];
            P->lv[l].ntile += (hcnt[g] + P->TW - 1) / P->TW;
        }
        if (P->lv[l].tile0 < 0) P->lv[l].tile0 = tiles;
    }
    P->ntile = tiles;
    int64_t *d_gs = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 2 * G));
    FMM_HIP(hipMemcpyAsync(d_gs, gstart.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, s));
    FMM_HIP(hipMemcpyAsync(d_gs + G, gtile.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, s));
    P->tile_tgt = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, tiles * P->TW)));
    P->tile_cls = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, tiles)));
    int32_t *tile_pos = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nc));
    if (tiles > 0) {
        k_fill_i32<<<grid_fill(tiles * P->TW), 256, 0, s>>>(P->tile_tgt, tiles * P->TW, -1);
        FMM_HIP(hipGetLastError());
    }
    k_fill_tiles<<<grid1(nc, 256), 256, 0, s>>>(ck, idx, nc, d_gs, d_gs + G, P->TW, P->tile_tgt, tile_pos);
    FMM_HIP(hipGetLastError());
    {
        // the plan keeps the host copy: it is the copy's source and the M2L
        // schedule reads it
        std::vector<int32_t> &tc = P->h_tile_cls;
        tc.assign(std::max<int64_t>(1, tiles), 0);
        for (int g = 0; g < G; ++g)
            if (gtile[g] >= 0)
                for (int64_t t = 0; t < (hcnt[g] + P->TW - 1) / P->TW; ++t) tc[gtile[g] + t] = g % 8;
        FMM_HIP(hipMemcpyAsync(P->tile_cls, tc.data(), sizeof(int32_t) * tc.size(), hipMemcpyHostToDevice, s));
    }
    al.free(d_gs);
    al.free(gcnt);
    al.free(idx);
    al.free(ck);

    // (every byte is written by the row count after the traversal)
    P->tile_kflag = static_cast<uint8_t *>(plan_alloc(P, std::max<int64_t>(1, tiles * (int64_t)P->K)));
    const int64_t nslots = tiles * (int64_t)P->K * P->TW;
    P->slots = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, nslots)));
    if (nslots > 0) {
        k_fill_i32<<<grid_fill(nslots), 256, 0, s>>>(P->slots, nslots, -1);
        FMM_HIP(hipGetLastError());
    }

    TreeView T;
    T.lvl = P->c_lvl;
    T.nch = P->c_nch;
    T.cbeg = P->c_cbeg;
    T.ix = P->c_ix;
    T.rad = P->tight ? P->c_rad : nullptr;
    T.key = P->c_key;
    T.tile_pos = tile_pos;
    T.kidx = P->st_kidx;
    T.slots = P->slots;
    T.kflag = P->tile_kflag;
    T.K = P->K;
    T.R = P->R;
    T.TW = P->TW;
    T.t4 = P->t4;

    const int cbits = bits_for(nc);
    FMM_CHECK(2 * cbits + 1 <= 64, FMM_ERR_UNSUPPORTED, "too many cells");
    // Growable outputs.
    std::vector<std::pair<uint64_t *, int64_t>> cross_parts, p2p_parts;
    int64_t ncross = 0, np2p = 0;
    unsigned long long *d_cnt = static_cast<unsigned long long *>(al.alloc(sizeof(unsigned long long) * 2));
    FMM_HIP(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long) * 2, s));
    int *d_err = static_cast<int *>(al.alloc(sizeof(int)));
    FMM_HIP(hipMemsetAsync(d_err, 0, sizeof(int), s));

    int2 *F = nullptr;
    int64_t nf = 0;
    if (P->depth == 0) {
        // the root is a leaf: the only pair is P2P(root, root)
        uint64_t *pp = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t)));
        FMM_HIP(hipMemsetAsync(pp, 0, sizeof(uint64_t), s));
        p2p_parts.push_back({pp, 1});
        np2p = 1;
    } else {
        // the frontier starts from (root, root) = (0, 0)
        F = static_cast<int2 *>(al.alloc(sizeof(int2)));
        FMM_HIP(hipMemsetAsync(F, 0, sizeof(int2), s));
        nf = 1;
    }
    int64_t *d_tot = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 4));
    while (nf > 0) {
        int32_t *cnts = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * 3 * nf));
        int64_t *offs = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 3 * nf));
        k_expand_count<<<grid1(nf, 256), 256, 0, s>>>(T, F, nf, cnts, cnts + nf, cnts + 2 * nf, d_cnt);
        FMM_HIP(hipGetLastError());
        scan_exclusive_i32to64(cnts, offs, 3 * nf, d_tot + 3, al, s);
        k_list_totals<<<1, 64, 0, s>>>(offs, nf, d_tot);
        FMM_HIP(hipGetLastError());
        int64_t tot[3];
        FMM_HIP(hipMemcpyAsync(tot, d_tot, sizeof(int64_t) * 3, hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        uint64_t *cx = tot[0] ? static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * tot[0])) : nullptr;
        uint64_t *pp = tot[1] ? static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * tot[1])) : nullptr;
        int2 *nx = tot[2] ? static_cast<int2 *>(al.alloc(sizeof(int2) * tot[2])) : nullptr;
        k_expand_write<<<grid1(nf, 256), 256, 0, s>>>(T, F, nf, offs, offs + nf, offs + 2 * nf, cx, pp, nx, cbits,
                                                      d_err);
        FMM_HIP(hipGetLastError());
        if (cx) cross_parts.push_back({cx, tot[0]});
        if (pp) p2p_parts.push_back({pp, tot[1]});
        ncross += tot[0];
        np2p += tot[1];
        al.free(offs);
        al.free(cnts);
        al.free(F);
        F = nx;
        nf = tot[2];
    }
    if (F) al.free(F);
    al.free(d_tot);
    al.free(tile_pos);

    // Row counts (the flags the batched M2L lists its entries by); with
    // m2l_sparse > 0 the same-level pairs of sparse rows join the cross-level
    // pairs.
    int64_t nsparse = 0;
    const int64_t nrow = tiles * (int64_t)P->K;
    int32_t *spc = nullptr;
    if (nrow > 0) {
        FMM_CHECK(P->TW == 64 || P->TW == 128, FMM_ERR_DEVICE, "traversal: tile width");
        // (the flag array holds one byte per row: a count of at most 128 fits)
        // (with the rotation kernel every row moves: a threshold above the tile
        // width; the automatic threshold moves rows only in plans with at least
        // 1024 tiles)
        const int thr = P->m2l_rotation ? 65 : (P->m2l_sparse >= 0 ? P->m2l_sparse : (tiles >= 1024 ? 24 : 0));
        if (thr > 0) spc = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nrow));
        k_sparse_count<<<grid_fill(nrow * (P->TW / 4)), 256, 0, s>>>(reinterpret_cast<const int4 *>(P->slots),
                                                                      P->tile_kflag, nrow, P->TW, thr, spc);
        FMM_HIP(hipGetLastError());
    }
    if (spc) {
        int64_t *off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * nrow));
        int64_t *d_tot = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
        scan_exclusive_i32to64(spc, off, nrow, d_tot, al, s);
        FMM_HIP(hipMemcpyAsync(&nsparse, d_tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        if (nsparse > 0) {
            uint64_t *sp = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * nsparse));
            const dim3 gm = grid_fill((nrow + 63) / 64 * 64);
            if (P->TW == 64)
                k_sparse_move<1><<<gm, 256, 0, s>>>(P->slots, P->tile_kflag, P->tile_tgt, spc, off, nrow, P->K, cbits,
                                                    sp);
            else
                k_sparse_move<2><<<gm, 256, 0, s>>>(P->slots, P->tile_kflag, P->tile_tgt, spc, off, nrow, P->K, cbits,
                                                    sp);
            FMM_HIP(hipGetLastError());
            cross_parts.push_back({sp, nsparse});
        }
        al.free(d_tot);
        al.free(off);
        al.free(spc);
    }

    int h_err = 0;
    unsigned long long h_cnt[2];
    FMM_HIP(hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipMemcpyAsync(h_cnt, d_cnt, sizeof(h_cnt), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    FMM_CHECK(h_err == 0, FMM_ERR_DEVICE, "traversal: same-level pair outside its stencil");
    P->n_m2l_same = (int64_t)h_cnt[0];
    P->n_m2l_cross = ncross;
    P->n_m2l_sparse = nsparse;
    P->n_m2lx = ncross + nsparse;
    P->n_p2p = np2p;

    // Concatenate (unless one generation produced the whole list), sort and
    // convert to CSR.
    auto concat = [&](std::vector<std::pair<uint64_t *, int64_t>> &parts, int64_t tot) {
        if (parts.size() == 1) {
            uint64_t *only = parts[0].first;
            parts.clear();  // the caller frees it as the whole list
            return only;
        }
        uint64_t *all = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * std::max<int64_t>(1, tot)));
        int64_t o = 0;
        for (auto &pr : parts) {
            FMM_HIP(hipMemcpyAsync(all + o, pr.first, sizeof(uint64_t) * pr.second, hipMemcpyDeviceToDevice, s));
            o += pr.second;
        }
        return all;
    };
    uint64_t *p2p_all = concat(p2p_parts, np2p);
    uint64_t *cross_all = concat(cross_parts, ncross + nsparse);
    sort_to_csr(P, p2p_all, np2p, cbits, 1, &P->p2p_off, &P->p2p_src, &P->p2p_near, nullptr, s);
    sort_to_csr(P, cross_all, ncross + nsparse, cbits, 0, &P->m2lx_off, &P->m2lx_src, nullptr, nullptr, s);
    P->p2p_body_pairs = -1;  // counted on demand by p2p_body_pairs()
    for (auto &pr : p2p_parts) al.free(pr.first);
    for (auto &pr : cross_parts) al.free(pr.first);
    al.free(p2p_all);
    al.free(cross_all);
    al.free(d_err);
    al.free(d_cnt);
}

}  // namespace fmm
