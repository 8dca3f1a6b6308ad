// tree.hip -- local octree on gfx950 (Section II.B and II.C of the paper).
//
// The tree is built from the rank's own bounding box: root cube anchored at
// the per-axis minima with side S = largest extent; 21-bit lattice
// coordinates per axis interleaved into a 64-bit Morton key (three bits per
// level, x the high bit of each triple); stable radix sort; then, level by
// level, every cell holding more than ncrit bodies (and above level 21) is
// split into its non-empty octants.  Cells are stored in (level, key) order.
// Everything here is integer work or float64 arithmetic in a fixed order, so
// the result is bit-identical to any other implementation of the same rules.
#include "internal.hpp"

#include <cmath>

namespace fmm {

namespace {

struct BoxPart {
    double lo[3], hi[3];
    int bad;
};

template <class T>
__global__ __launch_bounds__(256) void k_bbox_partial(const T *x, int64_t n, BoxPart *parts)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = (double)x[3 * i + d];
            if (!isfinite(v)) bad = 1;
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
    }
    __shared__ double s_lo[3][256], s_hi[3][256];
    __shared__ int s_bad[256];
    for (int d = 0; d < 3; ++d) { s_lo[d][threadIdx.x] = lo[d]; s_hi[d][threadIdx.x] = hi[d]; }
    s_bad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            for (int d = 0; d < 3; ++d) {
                s_lo[d][threadIdx.x] = fmin(s_lo[d][threadIdx.x], s_lo[d][threadIdx.x + o]);
                s_hi[d][threadIdx.x] = fmax(s_hi[d][threadIdx.x], s_hi[d][threadIdx.x + o]);
            }
            s_bad[threadIdx.x] |= s_bad[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        BoxPart b;
        for (int d = 0; d < 3; ++d) { b.lo[d] = s_lo[d][0]; b.hi[d] = s_hi[d][0]; }
        b.bad = s_bad[0];
        parts[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(256) void k_bbox_final(BoxPart *parts, int nparts)
{
    __shared__ double s_lo[3][256], s_hi[3][256];
    __shared__ int s_bad[256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], parts[k].lo[d]);
            hi[d] = fmax(hi[d], parts[k].hi[d]);
        }
        bad |= parts[k].bad;
    }
    for (int d = 0; d < 3; ++d) { s_lo[d][threadIdx.x] = lo[d]; s_hi[d][threadIdx.x] = hi[d]; }
    s_bad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            for (int d = 0; d < 3; ++d) {
                s_lo[d][threadIdx.x] = fmin(s_lo[d][threadIdx.x], s_lo[d][threadIdx.x + o]);
                s_hi[d][threadIdx.x] = fmax(s_hi[d][threadIdx.x], s_hi[d][threadIdx.x + o]);
            }
            s_bad[threadIdx.x] |= s_bad[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        BoxPart b;
        for (int d = 0; d < 3; ++d) { b.lo[d] = s_lo[d][0]; b.hi[d] = s_hi[d][0]; }
        b.bad = s_bad[0];
        parts[0] = b;
    }
}

// Spread the low 21 bits of v so that bit b lands at bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Inverse of spread3.
__device__ __forceinline__ uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

// Lattice coordinate: min(2^21 - 1, floor((x - lo) * scale)); the
// subtraction and the product round once each (contraction is off).
__device__ __forceinline__ uint64_t lattice(double x, double lo, double scale)
{
#pragma clang fp contract(off)
    double s = (x - lo) * scale;
    double f = floor(s);
    uint64_t v = f <= 0.0 ? 0ull : (uint64_t)f;
    const uint64_t top = (1ull << kLevels) - 1;
    return v > top ? top : v;
}

template <class T>
__global__ __launch_bounds__(256) void k_keys(const T *x, int64_t n, double lx, double ly, double lz, double scale,
                                              uint64_t *keys, int32_t *idx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t cx = lattice((double)x[3 * i], lx, scale);
    uint64_t cy = lattice((double)x[3 * i + 1], ly, scale);
    uint64_t cz = lattice((double)x[3 * i + 2], lz, scale);
    keys[i] = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
    idx[i] = (int32_t)i;
}

// First index in [b, e) whose octant digit (at the child level) is >= d.
__device__ __forceinline__ int32_t lower_digit(const uint64_t *keys, int32_t b, int32_t e, int shift, int d)
{
    while (b < e) {
        int32_t m = b + ((e - b) >> 1);
        if ((int)((keys[m] >> shift) & 7u) < d) b = m + 1;
        else e = m;
    }
    return b;
}

// Children of the cells of one level, one thread per (cell, octant digit d):
// the thread finds where digit d starts inside the cell's body range (digits
// are non-decreasing there, the keys being sorted), so child d holds
// [bnd[8c+d], bnd[8c+d+1]) with bnd[8c+8] = end.  The eight lanes of a cell
// are neighbours in one wave; a ballot over them gives the child count.
__device__ __forceinline__ bool child_bounds(const uint64_t *keys, const int32_t *beg, const int32_t *end,
                                             int64_t cnt, int level, int ncrit, int64_t c, int d, int32_t &lo,
                                             int32_t &hi)
{
    const bool valid = c < cnt;
    int32_t b = 0, e = 0;
    if (valid) {
        b = beg[c];
        e = end[c];
    }
    const bool split = valid && e - b > ncrit && level < kLevels;
    lo = e;
    if (split) lo = d == 0 ? b : lower_digit(keys, b, e, 3 * (kLevels - level - 1), d);
    const int lane = threadIdx.x & 63;
    hi = __shfl(lo, (lane & 7) == 7 ? lane : lane + 1, 64);
    if (d == 7) hi = e;
    return split && hi > lo;
}

__global__ __launch_bounds__(256) void k_count_children(const uint64_t *keys, const int32_t *beg, const int32_t *end,
                                                        int64_t cnt, int level, int ncrit, int32_t *nch,
                                                        int32_t *bnd)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = t >> 3;
    const int d = (int)(t & 7);
    int32_t lo, hi;
    const bool ne = child_bounds(keys, beg, end, cnt, level, ncrit, c, d, lo, hi);
    const uint64_t m = __ballot(ne);
    if (c < cnt) {
        bnd[t] = lo;
        if (d == 0) nch[c] = __popcll((m >> (threadIdx.x & 56)) & 0xffull);
    }
}

__global__ __launch_bounds__(256) void k_write_children(const int32_t *end, const uint64_t *ckey, int64_t cnt,
                                                        int64_t cstart, const int64_t *off, int64_t nstart,
                                                        const int32_t *nch, const int32_t *bnd, int32_t *cbeg,
                                                        int32_t *nbeg, int32_t *nend, int32_t *npar,
                                                        uint64_t *nkey)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = t >> 3;
    const int d = (int)(t & 7);
    if (c >= cnt) return;
    const int32_t lo = bnd[t], hi = d == 7 ? end[c] : bnd[t + 1];
    const bool split = nch[c] > 0;
    if (d == 0) cbeg[c] = split ? (int32_t)(nstart + off[c]) : -1;
    if (!split || hi <= lo) return;
    // children before this one: the non-empty octants below d
    int before = 0;
    for (int k = 0; k < d; ++k) {
        const int32_t a = bnd[8 * c + k], z = bnd[8 * c + k + 1];
        before += z > a;
    }
    const int64_t o = off[c] + before;
    nbeg[o] = lo;
    nend[o] = hi;
    npar[o] = (int32_t)(cstart + c);
    nkey[o] = (ckey[c] << 3) | (uint64_t)d;
}

// Lattice coordinates and centers c_d = lo_d + (i_d + 1/2) h_l, h_l = S 2^-l.
__global__ __launch_bounds__(256) void k_geometry(const uint64_t *ckey, const int32_t *lvl, int64_t ncell, double lx,
                                                  double ly, double lz, double S, int32_t *ix, double *ctr)
{
#pragma clang fp contract(off)
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    uint64_t k = ckey[c];
    int l = lvl[c];
    uint32_t v[3] = {compact3(k >> 2), compact3(k >> 1), compact3(k)};
    double h = ldexp(S, -l);
    double lo[3] = {lx, ly, lz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ix[3 * c + d] = (int32_t)v[d];
        const double off = ((double)v[d] + 0.5) * h;  // rounds once (no fused multiply-add)
        ctr[3 * c + d] = lo[d] + off;
    }
}

// Per-level cell arrays of the level loop and where each level starts in
// the (level, key)-ordered arrays.
struct LevelSrc {
    const int32_t *beg, *end, *par, *nch, *cbeg;
    const uint64_t *key;
    int64_t start;
};

// Cell c of the final order: its level is the last one starting at or before
// c (levels are few; a linear scan over them).
__global__ __launch_bounds__(256) void k_gather_levels(const LevelSrc *src, int nlev, int64_t nc, int32_t *lvl,
                                                       int32_t *beg, int32_t *end, int32_t *par, int32_t *nch,
                                                       int32_t *cbeg, uint64_t *key)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int l = 0;
    while (l + 1 < nlev && src[l + 1].start <= c) ++l;
    const LevelSrc &b = src[l];
    const int64_t i = c - b.start;
    lvl[c] = l;
    beg[c] = b.beg[i];
    end[c] = b.end[i];
    par[c] = b.par[i];
    nch[c] = b.nch[i];
    cbeg[c] = b.cbeg[i];
    key[c] = b.key[i];
}

__global__ void k_root_cell(int32_t *beg, int32_t *end, int32_t *par, uint64_t *key, int32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        beg[0] = 0;
        end[0] = n;
        par[0] = -1;
        key[0] = 0;
    }
}

__global__ __launch_bounds__(256) void k_leaf_flags(const int32_t *nch, int64_t ncell, int32_t *flag)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) flag[c] = nch[c] == 0 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_leaf_list(const int32_t *nch, const int32_t *beg, const int32_t *end,
                                                   const int64_t *pos, int64_t ncell, int32_t *leaves,
                                                   int32_t *leaf_of)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell || nch[c] != 0) return;
    leaves[pos[c]] = (int32_t)c;
    for (int32_t i = beg[c]; i < end[c]; ++i) leaf_of[i] = (int32_t)c;
}

// Offsets of the bodies from their leaf centers, in the compute type; with
// ul given (float32), also what the rounding left out, so that u + ul carries
// the float64 offset to about 48 bits.
template <class TX, class V4>
__global__ __launch_bounds__(256) void k_body_offsets(const TX *x, const int32_t *perm, const int32_t *leaf_of,
                                                      const double *ctr, int64_t n, V4 *ub, V4 *ul)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t o = perm[i];
    int64_t c = leaf_of[i];
    const double dx = (double)x[3 * o] - ctr[3 * c], dy = (double)x[3 * o + 1] - ctr[3 * c + 1],
                 dz = (double)x[3 * o + 2] - ctr[3 * c + 2];
    V4 u;
    u.x = (decltype(u.x))dx;
    u.y = (decltype(u.y))dy;
    u.z = (decltype(u.z))dz;
    u.w = 0;
    ub[i] = u;
    if (ul) {
        V4 r;
        r.x = (decltype(r.x))(dx - (double)u.x);
        r.y = (decltype(r.y))(dy - (double)u.y);
        r.z = (decltype(r.z))(dz - (double)u.z);
        r.w = 0;
        ul[i] = r;
    }
}

template <class T>
void launch_bbox(const void *x, int64_t n, BoxPart *parts, int nparts, hipStream_t s)
{
    k_bbox_partial<T><<<nparts, 256, 0, s>>>(static_cast<const T *>(x), n, parts);
    FMM_HIP(hipGetLastError());
    k_bbox_final<<<1, 256, 0, s>>>(parts, nparts);
    FMM_HIP(hipGetLastError());
}

}  // namespace

void tree_build(fmm_plan *P, const void *x, hipStream_t s)
{
    const int64_t n = P->n;
    Allocator &al = P->al;

    // T1: bounding box and non-finite check.
    const int nparts = (int)std::min<int64_t>(1024, (n + 255) / 256);
    BoxPart *parts = static_cast<BoxPart *>(al.alloc(sizeof(BoxPart) * nparts));
    if (P->dtype == FMM_F64) launch_bbox<double>(x, n, parts, nparts, s);
    else launch_bbox<float>(x, n, parts, nparts, s);
    BoxPart hb;
    FMM_HIP(hipMemcpyAsync(&hb, parts, sizeof(BoxPart), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    al.free(parts);
    FMM_CHECK(!hb.bad, FMM_ERR_NONFINITE, "fmm_build: non-finite coordinate");
    double S = 0.0;
    for (int d = 0; d < 3; ++d) {
        P->lo[d] = hb.lo[d];
        S = std::max(S, hb.hi[d] - hb.lo[d]);
    }
    if (S == 0.0) S = 1.0;
    P->S = S;
    P->scale = std::ldexp(1.0, kLevels) / S;

    // T2 + T3: keys and stable sort.
    P->keys = static_cast<uint64_t *>(plan_alloc(P, sizeof(uint64_t) * n));
    P->perm = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * n));
    if (P->dtype == FMM_F64)
        k_keys<double><<<grid1(n, 256), 256, 0, s>>>(static_cast<const double *>(x), n, P->lo[0], P->lo[1], P->lo[2],
                                                      P->scale, P->keys, P->perm);
    else
        k_keys<float><<<grid1(n, 256), 256, 0, s>>>(static_cast<const float *>(x), n, P->lo[0], P->lo[1], P->lo[2],
                                                     P->scale, P->keys, P->perm);
    FMM_HIP(hipGetLastError());
    radix_sort_u64(P->keys, P->perm, n, 3 * kLevels, al, s);

    // T4: cells, level by level (per-level arrays, then one copy).
    struct LvlBufs {
        int32_t *beg, *end, *par, *nch, *cbeg;
        uint64_t *key;
        int64_t cnt;
    };
    std::vector<LvlBufs> L;
    {
        LvlBufs r{};
        r.cnt = 1;
        r.beg = static_cast<int32_t *>(al.alloc(sizeof(int32_t)));
        r.end = static_cast<int32_t *>(al.alloc(sizeof(int32_t)));
        r.par = static_cast<int32_t *>(al.alloc(sizeof(int32_t)));
        r.key = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t)));
        k_root_cell<<<1, 64, 0, s>>>(r.beg, r.end, r.par, r.key, (int32_t)n);
        FMM_HIP(hipGetLastError());
        L.push_back(r);
    }
    int64_t *d_total = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
    int64_t start = 0;
    for (int level = 0;; ++level) {
        LvlBufs &cur = L[level];
        cur.nch = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * cur.cnt));
        cur.cbeg = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * cur.cnt));
        int32_t *bnd = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * 8 * cur.cnt));
        k_count_children<<<grid1(8 * cur.cnt, 256), 256, 0, s>>>(P->keys, cur.beg, cur.end, cur.cnt, level,
                                                                  P->ncrit, cur.nch, bnd);
        FMM_HIP(hipGetLastError());
        int64_t *off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * cur.cnt));
        scan_exclusive_i32to64(cur.nch, off, cur.cnt, d_total, al, s);
        int64_t total = 0;
        FMM_HIP(hipMemcpyAsync(&total, d_total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        const int64_t nstart = start + cur.cnt;
        LvlBufs nx{};
        nx.cnt = total;
        if (total > 0) {
            nx.beg = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * total));
            nx.end = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * total));
            nx.par = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * total));
            nx.key = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * total));
        }
        k_write_children<<<grid1(8 * cur.cnt, 256), 256, 0, s>>>(cur.end, cur.key, cur.cnt, start, off, nstart,
                                                                  cur.nch, bnd, cur.cbeg, nx.beg, nx.end, nx.par,
                                                                  nx.key);
        FMM_HIP(hipGetLastError());
        al.free(off);
        al.free(bnd);
        start = nstart;
        if (total == 0) break;
        L.push_back(nx);
    }
    al.free(d_total);

    P->depth = (int)L.size() - 1;
    P->ncell = start;
    const int64_t nc = P->ncell;
    P->c_lvl = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nc));
    P->c_beg = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nc));
    P->c_end = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nc));
    P->c_par = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nc));
    P->c_cbeg = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nc));
    P->c_nch = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nc));
    P->c_key = static_cast<uint64_t *>(plan_alloc(P, sizeof(uint64_t) * nc));
    P->lv.assign(P->depth + 1, Level{});
    // one gather of the per-level arrays into the (level, key)-ordered SoA
    std::vector<LevelSrc> hsrc(P->depth + 1);
    int64_t o = 0;
    for (int l = 0; l <= P->depth; ++l) {
        const LvlBufs &b = L[l];
        P->lv[l].start = o;
        P->lv[l].count = b.cnt;
        hsrc[l] = LevelSrc{b.beg, b.end, b.par, b.nch, b.cbeg, b.key, o};
        o += b.cnt;
    }
    LevelSrc *dsrc = static_cast<LevelSrc *>(al.alloc(sizeof(LevelSrc) * hsrc.size()));
    FMM_HIP(hipMemcpyAsync(dsrc, hsrc.data(), sizeof(LevelSrc) * hsrc.size(), hipMemcpyHostToDevice, s));
    k_gather_levels<<<grid1(nc, 256), 256, 0, s>>>(dsrc, P->depth + 1, nc, P->c_lvl, P->c_beg, P->c_end, P->c_par,
                                                   P->c_nch, P->c_cbeg, P->c_key);
    FMM_HIP(hipGetLastError());
    FMM_HIP(hipStreamSynchronize(s));  // hsrc is host memory; per-level buffers are freed below
    al.free(dsrc);
    for (auto &b : L) {
        al.free(b.beg); al.free(b.end); al.free(b.par); al.free(b.key);
        al.free(b.nch); al.free(b.cbeg);
    }

    // T5: geometry.
    P->c_ix = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * 3 * nc));
    P->c_ctr = static_cast<double *>(plan_alloc(P, sizeof(double) * 3 * nc));
    k_geometry<<<grid1(nc, 256), 256, 0, s>>>(P->c_key, P->c_lvl, nc, P->lo[0], P->lo[1], P->lo[2], P->S, P->c_ix,
                                              P->c_ctr);
    FMM_HIP(hipGetLastError());

    // Leaves, body -> leaf map, body offsets from leaf centers.
    int32_t *flag = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nc));
    int64_t *pos = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * nc));
    int64_t *d_nl = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
    k_leaf_flags<<<grid1(nc, 256), 256, 0, s>>>(P->c_nch, nc, flag);
    FMM_HIP(hipGetLastError());
    scan_exclusive_i32to64(flag, pos, nc, d_nl, al, s);
    FMM_HIP(hipMemcpyAsync(&P->nleaf, d_nl, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    P->leaves = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, P->nleaf)));
    P->leaf_of = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * n));
    k_leaf_list<<<grid1(nc, 256), 256, 0, s>>>(P->c_nch, P->c_beg, P->c_end, pos, nc, P->leaves, P->leaf_of);
    FMM_HIP(hipGetLastError());
    al.free(d_nl);
    al.free(pos);
    al.free(flag);

    if (P->precision == FMM_PREC_FP64) {
        P->ubody = plan_alloc(P, sizeof(double4) * n);
        if (P->dtype == FMM_F64)
            k_body_offsets<double, double4><<<grid1(n, 256), 256, 0, s>>>(
                static_cast<const double *>(x), P->perm, P->leaf_of, P->c_ctr, n, static_cast<double4 *>(P->ubody),
                nullptr);
        else
            k_body_offsets<float, double4><<<grid1(n, 256), 256, 0, s>>>(
                static_cast<const float *>(x), P->perm, P->leaf_of, P->c_ctr, n, static_cast<double4 *>(P->ubody),
                nullptr);
    } else {
        P->ubody = plan_alloc(P, sizeof(float4) * n);
        P->ulo = plan_alloc(P, sizeof(float4) * n);
        if (P->dtype == FMM_F64)
            k_body_offsets<double, float4><<<grid1(n, 256), 256, 0, s>>>(
                static_cast<const double *>(x), P->perm, P->leaf_of, P->c_ctr, n, static_cast<float4 *>(P->ubody),
                static_cast<float4 *>(P->ulo));
        else
            k_body_offsets<float, float4><<<grid1(n, 256), 256, 0, s>>>(
                static_cast<const float *>(x), P->perm, P->leaf_of, P->c_ctr, n, static_cast<float4 *>(P->ubody),
                static_cast<float4 *>(P->ulo));
    }
    FMM_HIP(hipGetLastError());

    // Coarse prefix for mixed precision: cells of levels < cfl.
    const int cfl = P->precision == FMM_PREC_FP64 ? P->depth + 1 : std::min(P->cfl, P->depth + 1);
    P->ncoarse = cfl > P->depth ? nc : P->lv[cfl].start;
}

}  // namespace fmm
