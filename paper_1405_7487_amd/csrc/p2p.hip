// p2p.hip -- particle-to-particle near field on gfx950 (Section II.A: P2P
// between the leaves that the dual traversal did not accept for M2L).
//
// One wave per target leaf.  Source bodies of the leaf's P2P list are
// gathered into LDS in batches of up to 256 bodies drawn from as many list
// entries as fill a batch, shifted into the target leaf's frame
// (offsets from leaf centers keep float32 differences accurate to ~1e-7 of
// the leaf size at any depth).  When the leaf holds few bodies, G lanes share
// a target and split each batch (G close to 64 / bodies, not only powers of
// two); a fixed-order tree of wave shuffles sums them.
// Batches are padded with zero-charge bodies far away so that every lane runs
// the same unrolled loop with compile-time LDS offsets.  Only the leaf's own
// bodies can coincide with a target, so only that batch tests r^2 > 0.  In
// the mixed path the leaf's own bodies and the leaves that touch it (which
// lead each list) use compensated offsets, so that nearly coincident bodies
// keep their separation's precision wherever a leaf face falls between them.
// Batch partial sums enter the running totals through a compensated (Kahan)
// add.
#include "internal.hpp"

namespace fmm {

namespace {

constexpr int kStage = 256;
constexpr int64_t kItemEntries = 4096;  // list entries per P2P work item of a cut leaf
constexpr int kUnroll = 4;

template <class T> __device__ __forceinline__ T rsqrt_t(T x);
template <> __device__ __forceinline__ float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

template <class T>
__device__ __forceinline__ void kahan_add(T &sum, T &comp, T v)
{
    const T y = v - comp;
    const T t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

template <class T> struct Acc {
    T p, x, y, z;
};

// Interaction of one target (ux, uy, uz) with staged sources sub, sub+G, ...
// of a batch padded to a multiple of G * kUnroll.
template <class T, class V4, int G, bool MASK>
__device__ __forceinline__ void batch(const V4 *sb, int npad, int sub, T ux, T uy, T uz, Acc<T> &a)
{
    const V4 *p = sb + sub;
    for (int it = 0; it < npad; it += G * kUnroll, p += G * kUnroll) {
        V4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = p[u * G];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const T dx = ux - v[u].x, dy = uy - v[u].y, dz = uz - v[u].z;
            const T r2 = dx * dx + dy * dy + dz * dz;
            T ri = rsqrt_t<T>(r2);
            if (MASK) ri = r2 > (T)0 ? ri : (T)0;
            const T qri = v[u].w * ri;
            const T qr3 = qri * (ri * ri);
            a.p += qri;
            a.x += qr3 * dx;
            a.y += qr3 * dy;
            a.z += qr3 * dz;
        }
    }
}

// The same with compensated coordinates, for a leaf's own bodies: offsets
// u + l (u rounded, l its residual), differences formed as (u_i - u_j) +
// (l_i - l_j).  For close bodies the first difference is exact, so the pair's
// separation keeps its own relative precision instead of the leaf size's;
// coincident bodies still give exactly zero and are skipped.
template <class T, class V4, int G, int UNR = kUnroll>
__device__ __forceinline__ void batch_own(const V4 *sb, const V4 *sl, int npad, int sub, T ux, T uy, T uz, T lx,
                                          T ly, T lz, Acc<T> &a)
{
    const V4 *p = sb + sub, *r = sl + sub;
    for (int it = 0; it < npad; it += G * UNR, p += G * UNR, r += G * UNR) {
        V4 v[UNR], w[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            v[u] = p[u * G];
            w[u] = r[u * G];
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const T dx = (ux - v[u].x) + (lx - w[u].x), dy = (uy - v[u].y) + (ly - w[u].y),
                    dz = (uz - v[u].z) + (lz - w[u].z);
            const T r2 = dx * dx + dy * dy + dz * dz;
            T ri = rsqrt_t<T>(r2);
            ri = r2 > (T)0 ? ri : (T)0;
            const T qri = v[u].w * ri;
            const T qr3 = qri * (ri * ri);
            a.p += qri;
            a.x += qr3 * dx;
            a.y += qr3 * dy;
            a.z += qr3 * dz;
        }
    }
}

template <class T, class V4>
__device__ __forceinline__ V4 far_dummy()
{
    V4 v;
    v.x = (T)1e15;
    v.y = (T)1e15;
    v.z = (T)1e15;
    v.w = (T)0;
    return v;
}

// LDS of the cooperative gather: per list entry of a batch, its body-count
// prefix sums, first body and center shift.  Declared once per kernel so that
// the instantiations for each G share it.
template <class T> struct GatherLds {
    int32_t excl[64], incl[64], base[64];
    T sh[64][3], sl[64][3];  // center shift and its rounding residual
};

template <class T, bool KAHAN>
__device__ __forceinline__ void fold_into(Acc<T> &s, Acc<T> &c, const Acc<T> &pa)
{
    if (KAHAN) {
        kahan_add(s.p, c.p, pa.p);
        kahan_add(s.x, c.x, pa.x);
        kahan_add(s.y, c.y, pa.y);
        kahan_add(s.z, c.z, pa.z);
    } else {
        s.p += pa.p; s.x += pa.x; s.y += pa.y; s.z += pa.z;
    }
}

// Sources of list entries [k, k1) of target leaf A for the lanes' targets u
// (and residuals ut).  A batch is gathered from the next (up to) 64 list
// entries at once: lane l takes entry k + l, a wave prefix sum of the leaf
// sizes places the bodies, and every LDS slot finds its leaf by a branchless
// binary search of that sum.  The loads of batch i+1 are in flight while
// batch i is multiplied (two LDS buffers); slots past the batch hold
// zero-charge dummies, which also pad the batch for the unrolled loop.
//
// COMP (leaves that touch A): every source is staged as a float32 offset hi
// from A's center plus the residual lo of that rounding, the center shift's
// own residual and the body's residual included (the shift rounded to float32
// carries an error of order 1e-7 of the leaf size, which is the whole
// separation of nearly coincident bodies on either side of a face); a pair's
// difference is then (u_t - hi) + (l_t - lo), and half a stage holds the
// residuals.
template <class T, class V4, bool KAHAN, int G, bool COMP>
__device__ void list_pass(V4 *sb, GatherLds<T> *gs, int A, int64_t k, int64_t k1, const int32_t *beg,
                          const int32_t *end, const int32_t *src, const double *ctr, const V4 *ub, const V4 *ul,
                          const V4 &u, const V4 &ut, int sub, Acc<T> &s, Acc<T> &c)
{
    constexpr int STG = COMP ? kStage / 2 : kStage;  // sources per LDS buffer
    constexpr int SMAX = (STG / (G * kUnroll)) * (G * kUnroll);
    constexpr int R = STG / 64;
    const int lane = threadIdx.x;
    const double cax = ctr[3 * A], cay = ctr[3 * A + 1], caz = ctr[3 * A + 2];
    int32_t *s_excl = gs->excl, *s_incl = gs->incl, *s_base = gs->base;
    T(*s_sh)[3] = gs->sh;
    T(*s_sl)[3] = gs->sl;
    int32_t o = 0;  // bodies of entry k already consumed
    V4 regs[R], rlo[COMP ? R : 1];
    int st_next = 0;
    auto gather = [&]() {
        const int64_t kk = k + lane;
        const int b = kk < k1 ? src[kk] : A;
        const int32_t skip = lane == 0 ? o : 0;
        const int32_t sz = (kk < k1 && b != A) ? end[b] - beg[b] - skip : 0;
        int32_t pre = sz;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t v = __shfl_up(pre, d, 64);
            if (lane >= d) pre += v;
        }
        const int staged = min(__shfl(pre, 63, 64), SMAX);
        s_incl[lane] = pre;
        s_excl[lane] = pre - sz;
        s_base[lane] = beg[b] + skip;
        const double shx = ctr[3 * b] - cax, shy = ctr[3 * b + 1] - cay, shz = ctr[3 * b + 2] - caz;
        s_sh[lane][0] = (T)shx;
        s_sh[lane][1] = (T)shy;
        s_sh[lane][2] = (T)shz;
        if (COMP) {
            s_sl[lane][0] = (T)(shx - (double)(T)shx);
            s_sl[lane][1] = (T)(shy - (double)(T)shy);
            s_sl[lane][2] = (T)(shz - (double)(T)shz);
        }
        __syncthreads();
        int lo[R];
#pragma unroll
        for (int r = 0; r < R; ++r) lo[r] = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (s_incl[lo[r] + step - 1] <= lane + 64 * r) lo[r] += step;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = lane + 64 * r;
            if (t < staged) {
                const int64_t j = s_base[lo[r]] + (t - s_excl[lo[r]]);
                V4 v = ub[j];
                if (COMP) {
                    // hi = fl(u + shift), with the exact rounding error of
                    // that sum (two-sum) carried into lo
                    const V4 w = ul[j];
                    V4 e;
                    const T hx = v.x + s_sh[lo[r]][0], hy = v.y + s_sh[lo[r]][1], hz = v.z + s_sh[lo[r]][2];
                    const T bx = hx - v.x, by = hy - v.y, bz = hz - v.z;
                    e.x = ((v.x - (hx - bx)) + (s_sh[lo[r]][0] - bx)) + (w.x + s_sl[lo[r]][0]);
                    e.y = ((v.y - (hy - by)) + (s_sh[lo[r]][1] - by)) + (w.y + s_sl[lo[r]][1]);
                    e.z = ((v.z - (hz - bz)) + (s_sh[lo[r]][2] - bz)) + (w.z + s_sl[lo[r]][2]);
                    e.w = (T)0;
                    v.x = hx;
                    v.y = hy;
                    v.z = hz;
                    rlo[r] = e;
                } else {
                    v.x += s_sh[lo[r]][0];
                    v.y += s_sh[lo[r]][1];
                    v.z += s_sh[lo[r]][2];
                }
                regs[r] = v;
            } else {
                regs[r] = far_dummy<T, V4>();
                if (COMP) rlo[r] = V4{};
            }
        }
        // advance the cursor past the consumed entries
        const int nf = __popcll(__ballot(pre <= staged));
        if (nf == 64) {
            k += 64;
            o = 0;
        } else {
            const int32_t consumed = staged - __shfl(pre - sz, nf, 64);
            o = (nf == 0 ? o : 0) + consumed;
            k += nf;
        }
        st_next = staged;
    };
    if (k < k1) gather();
    int buf = 0;
    while (st_next > 0 || k < k1) {
        V4 *cur = sb + buf * kStage;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cur[lane + 64 * r] = regs[r];
            if (COMP) cur[STG + lane + 64 * r] = rlo[r];
        }
        const int st_cur = st_next;
        __syncthreads();
        if constexpr (COMP) {
            // the compensated products hold twice the source registers, so
            // the next batch is loaded only after them, two sources per lane
            // and step (this pass covers the few touching leaves)
            if (st_cur > 0) {
                const int npad = (st_cur + G * kUnroll - 1) / (G * kUnroll) * (G * kUnroll);
                Acc<T> pa{0, 0, 0, 0};
                batch_own<T, V4, G, 2>(cur, cur + STG, npad, sub, u.x, u.y, u.z, ut.x, ut.y, ut.z, pa);
                fold_into<T, KAHAN>(s, c, pa);
            }
            if (k < k1) gather();
            else st_next = 0;
        } else {
            if (k < k1) gather();
            else st_next = 0;
            if (st_cur > 0) {
                const int npad = (st_cur + G * kUnroll - 1) / (G * kUnroll) * (G * kUnroll);
                Acc<T> pa{0, 0, 0, 0};
                batch<T, V4, G, false>(cur, npad, sub, u.x, u.y, u.z, pa);
                fold_into<T, KAHAN>(s, c, pa);
            }
        }
        buf ^= 1;
    }
    __syncthreads();
}

// Targets [base, base + cnt) of leaf A against list entries [k0, k1) (and
// the leaf's own bodies when own is set); sums go to op[oi], oE[3 oi + d]
// with oi = o0 + target.  Entries [k0, kn) are leaves that touch A: with
// residuals (mixed path) they run with compensated offsets.
template <class T, class V4, bool KAHAN, int G>
__device__ void leaf_chunk(V4 *sb, GatherLds<T> *gs, int A, int32_t tb, int base, int cnt, bool own,
                           const int32_t *beg, const int32_t *end, int64_t k0, int64_t kn, int64_t k1,
                           const int32_t *src, const double *ctr, const V4 *ub, const V4 *ul, T *op, T *oE, int64_t o0)
{
    // sources per batch: a multiple of G kUnroll, so a padded batch never
    // runs past its kStage slots
    constexpr int SMAX = (kStage / (G * kUnroll)) * (G * kUnroll);
    const int lane = threadIdx.x;
    const int ti = lane / G, sub = lane % G;
    const bool active = ti < cnt;
    const V4 u = ub[tb + base + (active ? ti : 0)];
    Acc<T> s{0, 0, 0, 0}, c{0, 0, 0, 0};
    const int32_t ab = beg[A], ae = own ? end[A] : beg[A];
    // 1) the leaf's own bodies (may coincide with the target): masked, with
    //    the residuals (when given) staged in the second buffer
    const V4 ut = ul ? ul[tb + base + (active ? ti : 0)] : V4{};
    for (int32_t o = ab; o < ae; o += SMAX) {
        const int take = min(SMAX, ae - o);
        const int npad = (take + G * kUnroll - 1) / (G * kUnroll) * (G * kUnroll);
        for (int l = lane; l < npad; l += 64) sb[l] = l < take ? ub[o + l] : far_dummy<T, V4>();
        if (ul)
            for (int l = lane; l < npad; l += 64) sb[kStage + l] = l < take ? ul[o + l] : V4{};
        __syncthreads();
        Acc<T> pa{0, 0, 0, 0};
        if (ul) batch_own<T, V4, G>(sb, sb + kStage, npad, sub, u.x, u.y, u.z, ut.x, ut.y, ut.z, pa);
        else batch<T, V4, G, true>(sb, npad, sub, u.x, u.y, u.z, pa);
        fold_into<T, KAHAN>(s, c, pa);
        __syncthreads();
    }
    // 2) the other leaves of the list: touching ones first (compensated when
    //    residuals exist), then the rest
    if (ul && kn > k0) {
        list_pass<T, V4, KAHAN, G, true>(sb, gs, A, k0, kn, beg, end, src, ctr, ub, ul, u, ut, sub, s, c);
        k0 = kn;
    }
    if (k1 > k0) list_pass<T, V4, KAHAN, G, false>(sb, gs, A, k0, k1, beg, end, src, ctr, ub, ul, u, ut, sub, s, c);
    if (KAHAN) {
        s.p -= c.p; s.x -= c.x; s.y -= c.y; s.z -= c.z;
    }
    // sum over the G lanes of a target (lanes ti G + [0, G)): a tree in a
    // fixed order, sub 0 ends with the total
#pragma unroll
    for (int w = 1; w < G; w <<= 1) {
        const T rp = __shfl_down(s.p, w, 64), rx = __shfl_down(s.x, w, 64);
        const T ry = __shfl_down(s.y, w, 64), rz = __shfl_down(s.z, w, 64);
        if (sub % (2 * w) == 0 && sub + w < G) {
            s.p += rp;
            s.x += rx;
            s.y += ry;
            s.z += rz;
        }
    }
    if (active && sub == 0) {
        const int64_t i = o0 + base + ti;
        op[i] = s.p;
        oE[3 * i] = s.x;
        oE[3 * i + 1] = s.y;
        oE[3 * i + 2] = s.z;
    }
}

// One wave per work item: a target leaf and a range of its list.  Leaves
// whose list is longer than kItemEntries are cut into consecutive items (only
// the first also runs the leaf's own bodies); their partial sums go to a
// buffer and k_p2p_reduce adds them in item order.  Without the cut, a coarse leaf
// whose list reaches every body of the tree keeps one wave busy long after
// the rest of the chip has finished.
template <class T, class V4, bool KAHAN>
__global__ __launch_bounds__(64) void k_p2p(const int32_t *it_leaf, const int64_t *it_k0, const int64_t *it_k1,
                                            const int64_t *it_out, const int32_t *beg, const int32_t *end,
                                            const int32_t *src, const int64_t *near, const double *ctr,
                                            const V4 *ub, const V4 *ul, T *phi_s, T *E_s, T *part_p, T *part_E)
{
    __shared__ V4 sb[2 * kStage];
    __shared__ GatherLds<T> gs;
    const int64_t item = blockIdx.x;
    const int A = it_leaf[item];
    const int32_t tb = beg[A], te = end[A];
    const int nt = te - tb;
    const int64_t k0 = it_k0[item], k1 = it_k1[item], ov = it_out[item];
    const int64_t kn = min(k1, max(k0, near[A]));  // [k0, kn): leaves touching A
    // ov >= 0: write to phi_s / E_s at body ov + t; ov < 0: partial sums at -ov - 1 + t
    const bool direct = ov >= 0;
    T *op = direct ? phi_s : part_p;
    T *oE = direct ? E_s : part_E;
    const int64_t o0 = direct ? ov : -ov - 1;
    const bool first = direct || item == 0 || it_leaf[item - 1] != A;  // the leaf's first item
    // chunks of at most 64 targets; a leaf of 33-55 bodies runs as 32 (two
    // lanes each) plus the rest, which keeps more lanes busy than 64-wide
    // chunks with most lanes idle, at the price of a second pass over the list
    for (int base = 0, cnt = 0; base < nt; base += cnt) {
        const int rem = nt - base;
        cnt = (rem > 32 && rem < 56) ? 32 : min(64, rem);
        // lanes per target: G close to 64 / cnt (at most 16), so few lanes idle
#define P2P_CHUNK(GG) leaf_chunk<T, V4, KAHAN, GG>(sb, &gs, A, tb, base, cnt, first, beg, end, k0, kn, k1, src, ctr, ub, ul, op, oE, o0)
        if (cnt <= 4) P2P_CHUNK(16);
        else if (cnt <= 5) P2P_CHUNK(12);
        else if (cnt <= 8) P2P_CHUNK(8);
        else if (cnt <= 10) P2P_CHUNK(6);
        else if (cnt <= 12) P2P_CHUNK(5);
        else if (cnt <= 16) P2P_CHUNK(4);
        else if (cnt <= 21) P2P_CHUNK(3);
        else if (cnt <= 32) P2P_CHUNK(2);
        else P2P_CHUNK(1);
#undef P2P_CHUNK
    }
}

// phi / E of the bodies of a cut leaf: the items' partial sums in item order,
// added in float64.  One block per cut leaf.
template <class T>
__global__ __launch_bounds__(64) void k_p2p_reduce(const int32_t *cl_leaf, const int64_t *cl_part, const int32_t *cl_n,
                                                   const int32_t *beg, const int32_t *end, const T *part_p,
                                                   const T *part_E, T *phi_s, T *E_s)
{
    const int64_t l = blockIdx.x;
    const int A = cl_leaf[l];
    const int32_t tb = beg[A], nt = end[A] - beg[A];
    const int64_t p0 = cl_part[l];
    const int nch = cl_n[l];
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        double p = 0, x = 0, y = 0, z = 0;
        for (int c = 0; c < nch; ++c) {
            const int64_t i = p0 + (int64_t)c * nt + t;
            p += (double)part_p[i];
            x += (double)part_E[3 * i];
            y += (double)part_E[3 * i + 1];
            z += (double)part_E[3 * i + 2];
        }
        const int64_t o = tb + t;
        phi_s[o] = (T)p;
        E_s[3 * o] = (T)x;
        E_s[3 * o + 1] = (T)y;
        E_s[3 * o + 2] = (T)z;
    }
}

__device__ __forceinline__ int64_t item_count(int64_t entries) { return max((int64_t)1, (entries + kItemEntries - 1) / kItemEntries); }

// per leaf (index i < nl): items, partial slots (cut leaves) and cut flag; 0 at i = nl
__global__ __launch_bounds__(256) void k_items_count(const int32_t *leaves, int64_t nl, const int64_t *off,
                                                     const int32_t *beg, const int32_t *end, int32_t *ni,
                                                     int32_t *np, int32_t *nc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nl) return;
    if (i == nl) {
        ni[i] = np[i] = nc[i] = 0;
        return;
    }
    const int A = leaves[i];
    const int64_t nch = item_count(off[A + 1] - off[A]);
    ni[i] = (int32_t)nch;
    np[i] = nch > 1 ? (int32_t)(nch * (end[A] - beg[A])) : 0;
    nc[i] = nch > 1 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_items_fill(const int32_t *leaves, int64_t nl, const int64_t *off,
                                                    const int32_t *beg, const int32_t *end, const int64_t *si,
                                                    const int64_t *sp, const int64_t *scut, int32_t *it_leaf,
                                                    int64_t *it_k0, int64_t *it_k1, int64_t *it_out,
                                                    int32_t *cl_leaf, int64_t *cl_part, int32_t *cl_n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int A = leaves[i];
    const int64_t k0 = off[A], k1 = off[A + 1], nch = item_count(k1 - k0);
    // one scan covers the three count arrays back to back
    const int64_t o = si[i] - si[0];
    if (nch == 1) {
        it_leaf[o] = A;
        it_k0[o] = k0;
        it_k1[o] = k1;
        it_out[o] = beg[A];
        return;
    }
    const int nt = end[A] - beg[A];
    const int64_t part = sp[i] - sp[0], c0 = scut[i] - scut[0];
    cl_leaf[c0] = A;
    cl_part[c0] = part;
    cl_n[c0] = (int32_t)nch;
    for (int64_t c = 0; c < nch; ++c) {
        it_leaf[o + c] = A;
        it_k0[o + c] = k0 + c * kItemEntries;
        it_k1[o + c] = min(k1, k0 + (c + 1) * kItemEntries);
        it_out[o + c] = -(part + c * nt) - 1;
    }
}

// Totals of the three item arrays from the scan over their concatenated
// counts (m entries each).
__global__ void k_items_totals(const int64_t *sc, int64_t m, int64_t *tot)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t all = tot[3];
        tot[0] = sc[m];
        tot[1] = sc[2 * m] - sc[m];
        tot[2] = all - sc[2 * m];
    }
}

// ---------------------------------------------------------------- mutual P2P
// Mutual interactions (listed among the features in Section II.C): each
// unordered pair of different leaves (A, B), A < B, is evaluated once and both
// leaves gain their sums; a leaf's own pairs stay one-sided (k_p2p with an
// empty list).  One wave per work item (a leaf A and a run of its upper
// entries, the list entries with source B > A).  The sources of the run are
// staged 64 at a time as four chunks of 16; the wave's four rows of 16 lanes
// each pair up to 16 of A's bodies (one per lane, kept in registers) with one
// chunk.  In 16 steps lane i meets every source of its chunk once: the
// source-side sums travel one lane along the row per step (a DPP rotation
// within the row), so after the 16 steps every source's sum is back on the
// lane it started from, complete over the row's targets, with no atomics and
// no reduction across lanes.  Rows that hold different target chunks of A
// against the same source chunk add their sums in a fixed order (a lane
// exchange across rows).  The source-side sums of every (upper entry, target
// chunk of 64, source body) go to their own slot, the target-side sums of
// every item to theirs, and k_mu_reduce adds them per body in a fixed order:
// the leaf's items in order, then its lower entries ordered by their upper
// twin, then the leaf's own pairs.
constexpr int kMuBatch = 64;  // sources staged per batch: four chunks of 16

// Rotation of a value by n lanes within each row of 16 (DPP row_ror).
template <int N> __device__ __forceinline__ int row_ror_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x120 + N, 0xf, 0xf, false); }
template <int N> __device__ __forceinline__ float row_ror(float v)
{
    return __builtin_bit_cast(float, row_ror_i<N>(__builtin_bit_cast(int, v)));
}
template <int N> __device__ __forceinline__ double row_ror(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)row_ror_i<N>((int)(unsigned)u), hi = (unsigned)row_ror_i<N>((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int N, class T> __device__ __forceinline__ void row_ror_acc(Acc<T> &b)
{
    b.p = row_ror<N>(b.p);
    b.x = row_ror<N>(b.x);
    b.y = row_ror<N>(b.y);
    b.z = row_ror<N>(b.z);
}

template <class T, class V4>
__device__ __forceinline__ V4 near_dummy()
{
    V4 v;
    v.x = (T)-1e15;
    v.y = (T)-1e15;
    v.z = (T)-1e15;
    v.w = (T)0;
    return v;
}

// Stages the next (up to) kMuBatch sources of upper entries [k, k1) of leaf
// A (entry k already consumed up to body o) into this lane's v (and w, the
// residual, with COMP), shifted into A's frame exactly as list_pass does,
// with the slot of its source-side sums for target chunk c in dst; advances
// (k, o) and returns the number staged.  Slots past it hold zero-charge
// dummies.  The slots of upper entry u for target chunk c are
// pb[u] + c |B| + (body - beg[B]).
template <class T, class V4, bool COMP>
__device__ int mu_gather(GatherLds<T> *gs, int64_t *sdst, int A, int c, int64_t &k, int64_t k1, int32_t &o,
                         const int32_t *usrc, const int64_t *pb, const int32_t *beg, const int32_t *end,
                         const double *ctr, const V4 *ub, const V4 *ul, V4 &v, V4 &w, int64_t &dst)
{
    const int lane = threadIdx.x;
    const double cax = ctr[3 * A], cay = ctr[3 * A + 1], caz = ctr[3 * A + 2];
    const int64_t kk = k + lane;
    const bool in = kk < k1;
    const int b = in ? usrc[kk] : A;
    const int32_t skip = lane == 0 ? o : 0;
    const int32_t full = end[b] - beg[b];
    const int32_t sz = in ? full - skip : 0;
    int32_t pre = sz;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(pre, d, 64);
        if (lane >= d) pre += t;
    }
    const int staged = min(__shfl(pre, 63, 64), kMuBatch);
    gs->incl[lane] = pre;
    gs->excl[lane] = pre - sz;
    gs->base[lane] = beg[b] + skip;
    sdst[lane] = in ? pb[kk] + (int64_t)c * full + skip : 0;
    const double shx = ctr[3 * b] - cax, shy = ctr[3 * b + 1] - cay, shz = ctr[3 * b + 2] - caz;
    gs->sh[lane][0] = (T)shx;
    gs->sh[lane][1] = (T)shy;
    gs->sh[lane][2] = (T)shz;
    if (COMP) {
        gs->sl[lane][0] = (T)(shx - (double)(T)shx);
        gs->sl[lane][1] = (T)(shy - (double)(T)shy);
        gs->sl[lane][2] = (T)(shz - (double)(T)shz);
    }
    __syncthreads();
    int e = 0;  // the entry of slot `lane`: the first whose inclusive prefix exceeds it
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1)
        if (gs->incl[e + step - 1] <= lane) e += step;
    dst = 0;
    if (lane < staged) {
        const int32_t r = lane - gs->excl[e];
        const int64_t j = gs->base[e] + r;
        dst = sdst[e] + r;
        v = ub[j];
        if (COMP) {
            const V4 q = ul[j];
            const T hx = v.x + gs->sh[e][0], hy = v.y + gs->sh[e][1], hz = v.z + gs->sh[e][2];
            const T bx = hx - v.x, by = hy - v.y, bz = hz - v.z;
            w.x = ((v.x - (hx - bx)) + (gs->sh[e][0] - bx)) + (q.x + gs->sl[e][0]);
            w.y = ((v.y - (hy - by)) + (gs->sh[e][1] - by)) + (q.y + gs->sl[e][1]);
            w.z = ((v.z - (hz - bz)) + (gs->sh[e][2] - bz)) + (q.z + gs->sl[e][2]);
            w.w = (T)0;
            v.x = hx;
            v.y = hy;
            v.z = hz;
        } else {
            v.x += gs->sh[e][0];
            v.y += gs->sh[e][1];
            v.z += gs->sh[e][2];
        }
    } else {
        v = far_dummy<T, V4>();
        w = V4{};
    }
    const int nf = __popcll(__ballot(pre <= staged));
    if (nf == 64) {
        k += 64;
        o = 0;
    } else {
        const int32_t consumed = staged - __shfl(pre - sz, nf, 64);
        o = (nf == 0 ? o : 0) + consumed;
        k += nf;
    }
    return staged;
}

// One staged batch against this lane's target u (residual ut with COMP).
// nac target chunks of 16 (1, 2 or 4) share the four rows: row r holds target
// chunk r % nac and, in round rd, source chunk rd (4 / nac) + r / nac.  With
// a chunk of at most g = 8 or 4 targets (nac = 1) the row holds each target
// on 16 / g lanes, which together meet the 16 sources in g steps; the sums
// then turn the remaining 16 - g lanes in one rotation, back to their
// sources' lanes.  dsl: the source-side slot of every staged source.
template <class T, class V4, bool COMP>
__device__ __forceinline__ void mu_batch(const V4 *cur, const V4 *curw, const int64_t *dsl, int staged, int nac,
                                         int g, int row, int i, int delta, const V4 &u, const V4 &ut, Acc<T> &pa,
                                         V4 *bufB)
{
    const int spr = 4 / nac;
    for (int rd = 0; rd < nac; ++rd) {
        const int sc = rd * spr + row / nac;
        const V4 *cs = cur + sc * 16;
        const V4 *cw = curw + sc * 16;
        Acc<T> b{0, 0, 0, 0};
#pragma unroll 4
        for (int t = 0; t < g; ++t) {
            const int j = (i + t * delta) & 15;  // the source whose sum this lane holds now
            const V4 v = cs[j];
            T dx = u.x - v.x, dy = u.y - v.y, dz = u.z - v.z;
            if (COMP) {
                const V4 w = cw[j];
                dx += ut.x - w.x;
                dy += ut.y - w.y;
                dz += ut.z - w.z;
            }
            const T r2 = dx * dx + dy * dy + dz * dz;
            T ri = rsqrt_t<T>(r2);
            if (COMP) ri = r2 > (T)0 ? ri : (T)0;
            const T ri2 = ri * ri;
            const T qs = v.w * ri, qt = u.w * ri;
            const T fs = qs * ri2, ft = qt * ri2;
            pa.p += qs;
            pa.x += fs * dx;
            pa.y += fs * dy;
            pa.z += fs * dz;
            b.p += qt;
            b.x -= ft * dx;
            b.y -= ft * dy;
            b.z -= ft * dz;
            row_ror_acc<1>(b);
        }
        if (g == 8) row_ror_acc<8>(b);
        else if (g == 4) row_ror_acc<12>(b);
        if (nac >= 2) {
            b.p += __shfl_xor(b.p, 16, 64);
            b.x += __shfl_xor(b.x, 16, 64);
            b.y += __shfl_xor(b.y, 16, 64);
            b.z += __shfl_xor(b.z, 16, 64);
        }
        if (nac == 4) {
            b.p += __shfl_xor(b.p, 32, 64);
            b.x += __shfl_xor(b.x, 32, 64);
            b.y += __shfl_xor(b.y, 32, 64);
            b.z += __shfl_xor(b.z, 32, 64);
        }
        const int slot = sc * 16 + i;
        if (row % nac == 0 && slot < staged) {
            V4 o;
            o.x = b.p;
            o.y = b.x;
            o.z = b.y;
            o.w = b.z;
            bufB[dsl[slot]] = o;
        }
    }
}

// Upper entries [k, k1) of leaf A as one stream, batch by batch (the loads of
// batch i + 1 in flight while batch i is multiplied), against target chunk c.
template <class T, class V4, bool KAHAN, bool COMP>
__device__ void mu_pass(V4 *sb, int64_t *sd, GatherLds<T> *gs, int64_t *sdst, int A, int c, int64_t k, int64_t k1,
                        const int32_t *usrc, const int64_t *pb, const int32_t *beg, const int32_t *end,
                        const double *ctr, const V4 *ub, const V4 *ul, int nac, int g, int row, int i, int delta,
                        const V4 &u, const V4 &ut, Acc<T> &s, Acc<T> &cc, V4 *bufB)
{
    const int lane = threadIdx.x;
    int32_t o = 0;
    V4 v, w;
    int64_t dst = 0;
    int st_next = k < k1 ? mu_gather<T, V4, COMP>(gs, sdst, A, c, k, k1, o, usrc, pb, beg, end, ctr, ub, ul, v, w, dst)
                         : 0;
    int buf = 0;
    while (st_next > 0) {
        V4 *cur = sb + buf * 2 * kMuBatch;
        int64_t *cd = sd + buf * kMuBatch;
        cur[lane] = v;
        if (COMP) cur[kMuBatch + lane] = w;
        cd[lane] = dst;
        const int st_cur = st_next;
        __syncthreads();
        st_next = k < k1 ? mu_gather<T, V4, COMP>(gs, sdst, A, c, k, k1, o, usrc, pb, beg, end, ctr, ub, ul, v, w, dst)
                         : 0;
        Acc<T> pa{0, 0, 0, 0};
        mu_batch<T, V4, COMP>(cur, cur + kMuBatch, cd, st_cur, nac, g, row, i, delta, u, ut, pa, bufB);
        fold_into<T, KAHAN>(s, cc, pa);
        buf ^= 1;
    }
    __syncthreads();
}

// it_u: [4 nitem] = first upper entry, end of its touching run, end, first
// target-side slot.  Block b runs item order[b]: the items with the most
// pair work first, so that the short ones fill the end of the launch (a
// leaf's share of upper entries runs from none to its whole list).
template <class T, class V4, bool KAHAN>
__global__ __launch_bounds__(64) void k_p2p_mutual(const int32_t *order, const int32_t *it_leaf, const int64_t *it_u,
                                                   int64_t nitem, const int32_t *usrc, const int64_t *pb,
                                                   const int32_t *beg, const int32_t *end, const double *ctr,
                                                   const V4 *ub, const V4 *ul, V4 *bufA, V4 *bufB)
{
    __shared__ V4 sb[4 * kMuBatch];
    __shared__ int64_t sd[2 * kMuBatch];
    __shared__ int64_t sdst[64];
    __shared__ GatherLds<T> gs;
    const int64_t item = order[blockIdx.x];
    const int A = it_leaf[item];
    const int64_t u0 = it_u[item], un = it_u[nitem + item], u1 = it_u[2 * nitem + item], a0 = it_u[3 * nitem + item];
    const int lane = threadIdx.x, row = lane >> 4, i = lane & 15;
    // direction of the row rotation: after one step lane i holds the sum that
    // was on lane i + delta (mod 16)
    const int delta = (row_ror_i<1>(i) - i) & 15;
    const int32_t tb = beg[A], nt = end[A] - tb;
    for (int base = 0; base < nt; base += 64) {
        const int cnt = min(64, nt - base);
        const int nac = cnt <= 16 ? 1 : (cnt <= 32 ? 2 : 4);
        const int g = cnt <= 4 ? 4 : (cnt <= 8 ? 8 : 16);
        const int ti = (row % nac) * 16 + (i & (g - 1));
        const bool valid = ti < cnt;
        const V4 u = valid ? ub[tb + base + ti] : near_dummy<T, V4>();
        const V4 ut = (ul && valid) ? ul[tb + base + ti] : V4{};
        Acc<T> s{0, 0, 0, 0}, c{0, 0, 0, 0};
        int64_t k0 = u0;
        if (ul && un > u0) {
            mu_pass<T, V4, KAHAN, true>(sb, sd, &gs, sdst, A, base / 64, u0, un, usrc, pb, beg, end, ctr, ub, ul, nac,
                                        g, row, i, delta, u, ut, s, c, bufB);
            k0 = un;
        }
        if (u1 > k0)
            mu_pass<T, V4, KAHAN, false>(sb, sd, &gs, sdst, A, base / 64, k0, u1, usrc, pb, beg, end, ctr, ub, ul, nac,
                                         g, row, i, delta, u, ut, s, c, bufB);
        if (KAHAN) {
            s.p -= c.p; s.x -= c.x; s.y -= c.y; s.z -= c.z;
        }
        // lanes that hold the same target: a fixed-order sum, within the row
        // (copies of a short chunk), then across rows
        for (int w = g; w < 16; w <<= 1) {
            s.p += __shfl_xor(s.p, w, 64);
            s.x += __shfl_xor(s.x, w, 64);
            s.y += __shfl_xor(s.y, w, 64);
            s.z += __shfl_xor(s.z, w, 64);
        }
        if (nac == 1) {
            s.p += __shfl_xor(s.p, 16, 64);
            s.x += __shfl_xor(s.x, 16, 64);
            s.y += __shfl_xor(s.y, 16, 64);
            s.z += __shfl_xor(s.z, 16, 64);
        }
        if (nac <= 2) {
            s.p += __shfl_xor(s.p, 32, 64);
            s.x += __shfl_xor(s.x, 32, 64);
            s.y += __shfl_xor(s.y, 32, 64);
            s.z += __shfl_xor(s.z, 32, 64);
        }
        if (row < nac && i < g && valid) {
            V4 oa;
            oa.x = s.p;
            oa.y = s.x;
            oa.z = s.y;
            oa.w = s.z;
            bufA[a0 + base + ti] = oa;
        }
    }
}

// Per leaf: its own pairs (already in phi_s / E_s from k_p2p), then the
// target-side sums of its items in order, then the source-side sums of the
// upper entries that name it (ordered by entry, each over the target chunks
// of the entry's leaf in order); added in float64.  G groups of lanes take
// every G-th term, eight loads in flight, and their sums are added in group
// order.
template <class T, class V4>
__global__ __launch_bounds__(64) void k_mu_reduce(const int32_t *leaves, const int64_t *li, const int64_t *it_u,
                                                  int64_t nitem, const uint64_t *tkey, const int32_t *tval,
                                                  int64_t nup, const int64_t *pb, const int32_t *beg,
                                                  const int32_t *end, const V4 *bufA, const V4 *bufB, T *phi_s, T *E_s)
{
    __shared__ double red[64][4];
    const int64_t l = blockIdx.x;
    const int A = leaves[l];
    const int32_t tb = beg[A], nt = end[A] - tb;
    // [lo, hi): the entries whose source is A
    int64_t lo = 0, hi = nup;
    while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (tkey[m] < (uint64_t)A) lo = m + 1;
        else hi = m;
    }
    int64_t hi2 = nup, lo2 = lo;
    while (lo2 < hi2) {
        const int64_t m = (lo2 + hi2) >> 1;
        if (tkey[m] <= (uint64_t)A) lo2 = m + 1;
        else hi2 = m;
    }
    const int64_t i0 = li[l], i1 = li[l + 1];
    // groups: G = the largest power of two with G nt <= 64 (1 above 64 bodies)
    int G = 1;
    while (2 * G * nt <= 64) G *= 2;
    const int span = nt < 64 ? nt : 64;
    const int grp = threadIdx.x / span, tl = threadIdx.x % span;
    for (int t0 = 0; t0 < nt; t0 += span) {
        const int t = t0 + tl;
        const bool act = grp < G && t < nt;
        double p = 0, x = 0, y = 0, z = 0;
        if (act) {
            for (int64_t it = i0 + grp; it < i1; it += G) {
                const V4 a = bufA[it_u[3 * nitem + it] + t];
                p += (double)a.x;
                x += (double)a.y;
                y += (double)a.z;
                z += (double)a.w;
            }
            constexpr int D = 8;
            for (int64_t q = lo + grp; q < lo2; q += (int64_t)G * D) {
                V4 vals[D];
                int nv = 0;
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    const int64_t qq = q + (int64_t)r * G;
                    vals[r] = V4{};
                    if (qq < lo2) {
                        const int64_t e = tval[qq];
                        vals[r] = bufB[pb[e] + t];
                        nv = r + 1;
                    }
                }
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    if (r < nv) {
                        const int64_t qq = q + (int64_t)r * G;
                        const int64_t e = tval[qq];
                        const int64_t nch = (pb[e + 1] - pb[e]) / nt;
                        p += (double)vals[r].x;
                        x += (double)vals[r].y;
                        y += (double)vals[r].z;
                        z += (double)vals[r].w;
                        for (int64_t cc = 1; cc < nch; ++cc) {
                            const V4 b = bufB[pb[e] + cc * nt + t];
                            p += (double)b.x;
                            x += (double)b.y;
                            y += (double)b.z;
                            z += (double)b.w;
                        }
                    }
                }
            }
        }
        if (G > 1) {
            red[threadIdx.x][0] = p;
            red[threadIdx.x][1] = x;
            red[threadIdx.x][2] = y;
            red[threadIdx.x][3] = z;
            __syncthreads();
            if (grp == 0 && act) {
                for (int gg = 1; gg < G; ++gg) {
                    p += red[gg * span + tl][0];
                    x += red[gg * span + tl][1];
                    y += red[gg * span + tl][2];
                    z += red[gg * span + tl][3];
                }
            }
            __syncthreads();
        }
        if (grp == 0 && act) {
            const int64_t o = tb + t;
            phi_s[o] = (T)((double)phi_s[o] + p);
            E_s[3 * o] = (T)((double)E_s[3 * o] + x);
            E_s[3 * o + 1] = (T)((double)E_s[3 * o + 1] + y);
            E_s[3 * o + 2] = (T)((double)E_s[3 * o + 2] + z);
        }
    }
}

// One wave per leaf (i < nl): upper entries, those in the touching run, items
// and target-side slots; zeros at i = nl.
__global__ __launch_bounds__(256) void k_mu_count(const int32_t *leaves, int64_t nl, const int64_t *off,
                                                  const int64_t *near, const int32_t *src, const int32_t *beg,
                                                  const int32_t *end, int32_t *cu, int32_t *ct, int32_t *ci,
                                                  int32_t *ca)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i > nl) return;
    if (i == nl) {
        if (lane == 0) cu[i] = ct[i] = ci[i] = ca[i] = 0;
        return;
    }
    const int A = leaves[i];
    const int64_t k0 = off[A], kn = near[A], k1 = off[A + 1];
    int32_t nu = 0, nn = 0;
    for (int64_t k = k0 + lane; k - lane < k1; k += 64) {
        const bool up = k < k1 && src[k] > A;
        nu += __popcll(__ballot(up));
        nn += __popcll(__ballot(up && k < kn));
    }
    if (lane == 0) {
        const int32_t nit = (int32_t)((nu + kItemEntries - 1) / kItemEntries);
        cu[i] = nu;
        ct[i] = nn;
        ci[i] = nit;
        ca[i] = nit * (end[A] - beg[A]);
    }
}

// One wave per leaf: its upper entries in list order with their source-side
// slot counts (source bodies times A's target chunks), its items, and its
// first item.  su, si, sa: exclusive scans (first
// element at index 0 of each) of the upper-entry, item and target-slot counts.
__global__ __launch_bounds__(256) void k_mu_fill(const int32_t *leaves, int64_t nl, const int64_t *off,
                                                 const int32_t *src, const int32_t *beg, const int32_t *end,
                                                 const int32_t *ct, const int64_t *su, const int64_t *si,
                                                 const int64_t *sa, int32_t *usrc, int32_t *usz, int32_t *it_leaf,
                                                 int64_t *it_u, int64_t nitem, int64_t *li)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i > nl) return;
    if (lane == 0) li[i] = si[i] - si[0];
    if (i == nl) return;
    const int A = leaves[i];
    const int64_t k0 = off[A], k1 = off[A + 1];
    const int64_t ub0 = su[i] - su[0];
    const int32_t nch = (end[A] - beg[A] + 63) / 64;  // target chunks of A
    int64_t u = ub0;
    for (int64_t k = k0 + lane; k - lane < k1; k += 64) {
        const int32_t b = k < k1 ? src[k] : A;
        const bool up = b > A;
        const uint64_t m = __ballot(up);
        if (up) {
            const int64_t o = u + __popcll(m & ((1ull << lane) - 1));
            usrc[o] = b;
            usz[o] = (end[b] - beg[b]) * nch;
        }
        u += __popcll(m);
    }
    if (lane != 0) return;
    const int64_t ue = u, un = ub0 + ct[i];
    const int64_t it0 = si[i] - si[0], a_0 = sa[i] - sa[0];
    const int nt = end[A] - beg[A];
    for (int64_t c = 0; ub0 + c * kItemEntries < ue; ++c) {
        const int64_t it = it0 + c;
        const int64_t a = ub0 + c * kItemEntries, e = min(ue, a + kItemEntries);
        it_leaf[it] = A;
        it_u[it] = a;
        it_u[nitem + it] = min(e, max(a, un));
        it_u[2 * nitem + it] = e;
        it_u[3 * nitem + it] = a_0 + c * nt;
    }
}

// Sort key of every item: its pair work (source-side slots, i.e. source
// bodies times target chunks, times the target bodies of one chunk)
// subtracted from 2^40, so that an ascending stable sort puts the most work
// first.
__global__ __launch_bounds__(256) void k_mu_work(const int32_t *it_leaf, const int64_t *it_u, int64_t nitem,
                                                 const int64_t *pb, const int32_t *beg, const int32_t *end,
                                                 uint64_t *key, int32_t *val)
{
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= nitem) return;
    const int A = it_leaf[it];
    const int64_t u0 = it_u[it], u1 = it_u[2 * nitem + it];
    const int64_t w = (pb[u1] - pb[u0]) * min(64, end[A] - beg[A]);
    key[it] = (1ull << 40) - (uint64_t)min(w, (int64_t)(1ll << 40) - 1);
    val[it] = (int32_t)it;
}

__global__ __launch_bounds__(256) void k_mu_keys(const int32_t *usrc, int64_t n, uint64_t *key, int32_t *val)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    key[u] = (uint64_t)usrc[u];
    val[u] = (int32_t)u;
}

// The one-sided items of the mutual mode: every leaf with an empty list, so
// k_p2p runs only its own bodies and writes them straight to the outputs.
__global__ __launch_bounds__(256) void k_own_items(const int32_t *leaves, int64_t nl, const int64_t *off,
                                                   const int32_t *beg, int32_t *it_leaf, int64_t *it_k0,
                                                   int64_t *it_k1, int64_t *it_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int A = leaves[i];
    it_leaf[i] = A;
    it_k0[i] = it_k1[i] = off[A];
    it_out[i] = beg[A];
}

template <class T, class V4, bool KAHAN>
void launch_items(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    FMM_CHECK(P->p2p_nitem * 64 < (1ll << 32), FMM_ERR_UNSUPPORTED, "p2p: too many work items");
    k_p2p<T, V4, KAHAN><<<(unsigned)P->p2p_nitem, 64, 0, s>>>(
        P->p2p_it_leaf, P->p2p_it_k0, P->p2p_it_k1, P->p2p_it_out, P->c_beg, P->c_end, P->p2p_src, P->p2p_near, P->c_ctr,
        static_cast<const V4 *>(ub), static_cast<const V4 *>(P->ulo), static_cast<T *>(phi_s), static_cast<T *>(E_s),
        static_cast<T *>(P->p2p_part), static_cast<T *>(P->p2p_part) + P->p2p_npart);
    FMM_HIP(hipGetLastError());
    if (P->mutual && P->mu_nitem > 0) {
        FMM_CHECK(P->mu_nitem < (1ll << 32), FMM_ERR_UNSUPPORTED, "p2p: too many mutual work items");
        k_p2p_mutual<T, V4, KAHAN><<<(unsigned)P->mu_nitem, 64, 0, s>>>(
            P->mu_order, P->mu_it_leaf, P->mu_it_u, P->mu_nitem, P->mu_src, P->mu_pb, P->c_beg, P->c_end, P->c_ctr,
            static_cast<const V4 *>(ub), static_cast<const V4 *>(P->ulo), static_cast<V4 *>(P->mu_bufA),
            static_cast<V4 *>(P->mu_bufB));
        FMM_HIP(hipGetLastError());
    }
    if (P->mutual) {
        k_mu_reduce<T, V4><<<(unsigned)P->nleaf, 64, 0, s>>>(
            P->leaves, P->mu_li, P->mu_it_u, P->mu_nitem, P->mu_tkey, P->mu_tval, P->mu_nup, P->mu_pb, P->c_beg,
            P->c_end, static_cast<const V4 *>(P->mu_bufA), static_cast<const V4 *>(P->mu_bufB),
            static_cast<T *>(phi_s), static_cast<T *>(E_s));
        FMM_HIP(hipGetLastError());
    }
    if (P->p2p_ncut > 0) {
        k_p2p_reduce<T><<<(unsigned)P->p2p_ncut, 64, 0, s>>>(
            P->p2p_cl_leaf, P->p2p_cl_part, P->p2p_cl_n, P->c_beg, P->c_end, static_cast<const T *>(P->p2p_part),
            static_cast<const T *>(P->p2p_part) + P->p2p_npart, static_cast<T *>(phi_s), static_cast<T *>(E_s));
        FMM_HIP(hipGetLastError());
    }
}

void launch_p2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    if (P->precision == FMM_PREC_FP64) launch_items<double, double4, false>(P, ub, phi_s, E_s, s);
    else if (P->kahan) launch_items<float, float4, true>(P, ub, phi_s, E_s, s);
    else launch_items<float, float4, false>(P, ub, phi_s, E_s, s);
}

}  // namespace

void p2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    if (P->nleaf == 0) return;
    launch_p2p(P, ub, phi_s, E_s, s);
}

// Mutual mode: one-sided items for the leaves' own bodies, the upper entries
// of every list with their source-side slots (a scan of the source sizes),
// the entries ordered by source (a stable radix sort) and the work items.
static void p2p_mutual_prepare(fmm_plan *P, hipStream_t s)
{
    const int64_t nl = P->nleaf;
    Allocator &al = P->al;
    P->p2p_nitem = nl;
    P->p2p_it_leaf = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nl));
    P->p2p_it_k0 = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * nl));
    P->p2p_it_k1 = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * nl));
    P->p2p_it_out = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * nl));
    k_own_items<<<grid1(nl, 256), 256, 0, s>>>(P->leaves, nl, P->p2p_off, P->c_beg, P->p2p_it_leaf, P->p2p_it_k0,
                                              P->p2p_it_k1, P->p2p_it_out);
    FMM_HIP(hipGetLastError());

    const int64_t m = nl + 1;
    int32_t *cnt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * 4 * m));
    int64_t *sc = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 4 * m));
    int64_t *tot = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
    k_mu_count<<<grid1(m, 4), 256, 0, s>>>(P->leaves, nl, P->p2p_off, P->p2p_near, P->p2p_src, P->c_beg, P->c_end,
                                             cnt, cnt + m, cnt + 2 * m, cnt + 3 * m);
    FMM_HIP(hipGetLastError());
    // one scan over [upper entries | touching (unused) | items | target slots]
    scan_exclusive_i32to64(cnt, sc, 4 * m, tot, al, s);
    int64_t h[4];
    FMM_HIP(hipMemcpyAsync(&h[0], sc + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipMemcpyAsync(&h[1], sc + 2 * m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipMemcpyAsync(&h[2], sc + 3 * m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipMemcpyAsync(&h[3], tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    // sc[0 .. m) scans the upper-entry counts (total h[0]); sc[2m .. 3m) the
    // item counts, from h[1]; sc[3m .. 4m) the target slots, from h[2]
    const int64_t nup = h[0];
    P->mu_nup = nup;
    P->mu_nitem = h[2] - h[1];
    P->mu_nabody = h[3] - h[2];
    FMM_CHECK(nup < (1ll << 31), FMM_ERR_UNSUPPORTED, "mutual P2P: more than 2^31 upper entries");
    P->mu_li = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * m));
    P->mu_src = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, nup)));
    P->mu_it_leaf = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, P->mu_nitem)));
    P->mu_it_u = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * 4 * std::max<int64_t>(1, P->mu_nitem)));
    int32_t *usz = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * std::max<int64_t>(1, nup)));
    k_mu_fill<<<grid1(m, 4), 256, 0, s>>>(P->leaves, nl, P->p2p_off, P->p2p_src, P->c_beg, P->c_end, cnt + m, sc,
                                            sc + 2 * m, sc + 3 * m, P->mu_src, usz, P->mu_it_leaf, P->mu_it_u,
                                            P->mu_nitem, P->mu_li);
    FMM_HIP(hipGetLastError());
    al.free(tot);
    al.free(sc);
    al.free(cnt);
    const size_t esz = P->precision == FMM_PREC_FP64 ? sizeof(double) : sizeof(float);
    P->mu_pb = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * (nup + 1)));
    P->mu_tkey = static_cast<uint64_t *>(plan_alloc(P, sizeof(uint64_t) * std::max<int64_t>(1, nup)));
    P->mu_tval = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, nup)));
    P->mu_nslot = 0;
    if (nup > 0) {
        int64_t *t2 = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
        scan_exclusive_i32to64(usz, P->mu_pb, nup, t2, al, s);
        FMM_HIP(hipMemcpyAsync(P->mu_pb + nup, t2, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        FMM_HIP(hipMemcpyAsync(&P->mu_nslot, t2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        k_mu_keys<<<grid1(nup, 256), 256, 0, s>>>(P->mu_src, nup, P->mu_tkey, P->mu_tval);
        FMM_HIP(hipGetLastError());
        int bits = 1;
        while ((1ll << bits) < P->ncell) ++bits;
        radix_sort_u64(P->mu_tkey, P->mu_tval, nup, bits, al, s);
        FMM_HIP(hipStreamSynchronize(s));
        al.free(t2);
    }
    al.free(usz);
    // launch order of the items, most work first
    P->mu_order = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, P->mu_nitem)));
    if (P->mu_nitem > 0) {
        FMM_CHECK(P->mu_nitem < (1ll << 31), FMM_ERR_UNSUPPORTED, "mutual P2P: too many work items");
        uint64_t *wk = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * P->mu_nitem));
        k_mu_work<<<grid1(P->mu_nitem, 256), 256, 0, s>>>(P->mu_it_leaf, P->mu_it_u, P->mu_nitem, P->mu_pb, P->c_beg,
                                                          P->c_end, wk, P->mu_order);
        FMM_HIP(hipGetLastError());
        radix_sort_u64(wk, P->mu_order, P->mu_nitem, 41, al, s);
        al.free(wk);
    }
    P->mu_bufA = plan_alloc(P, esz * 4 * std::max<int64_t>(1, P->mu_nabody));
    P->mu_bufB = plan_alloc(P, esz * 4 * std::max<int64_t>(1, P->mu_nslot));
}

// Work items of the P2P kernel: one per leaf, or one per kItemEntries list
// entries for leaves with longer lists, with their partial-sum slots; built
// on the device by two scans in leaf order.
void p2p_prepare(fmm_plan *P, hipStream_t s)
{
    const int64_t nl = P->nleaf;
    P->p2p_nitem = 0;
    P->p2p_ncut = 0;
    P->p2p_npart = 0;
    if (nl == 0) return;
    if (P->mutual) {
        p2p_mutual_prepare(P, s);
        return;
    }
    Allocator &al = P->al;
    int32_t *cnt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * 3 * (nl + 1)));
    int64_t *sc = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 3 * (nl + 1)));
    int64_t *tot = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 4));
    k_items_count<<<grid1(nl + 1, 256), 256, 0, s>>>(P->leaves, nl, P->p2p_off, P->c_beg, P->c_end, cnt,
                                                      cnt + (nl + 1), cnt + 2 * (nl + 1));
    FMM_HIP(hipGetLastError());
    scan_exclusive_i32to64(cnt, sc, 3 * (nl + 1), tot + 3, al, s);
    k_items_totals<<<1, 64, 0, s>>>(sc, nl + 1, tot);
    FMM_HIP(hipGetLastError());
    int64_t h[3];
    FMM_HIP(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    P->p2p_nitem = h[0];
    P->p2p_npart = h[1];
    P->p2p_ncut = h[2];
    P->p2p_it_leaf = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * h[0]));
    P->p2p_it_k0 = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * h[0]));
    P->p2p_it_k1 = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * h[0]));
    P->p2p_it_out = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * h[0]));
    if (h[2] > 0) {
        const size_t esz = P->precision == FMM_PREC_FP64 ? sizeof(double) : sizeof(float);
        P->p2p_part = plan_alloc(P, esz * 4 * h[1]);
        P->p2p_cl_leaf = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * h[2]));
        P->p2p_cl_part = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * h[2]));
        P->p2p_cl_n = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * h[2]));
    }
    k_items_fill<<<grid1(nl, 256), 256, 0, s>>>(P->leaves, nl, P->p2p_off, P->c_beg, P->c_end, sc, sc + (nl + 1),
                                               sc + 2 * (nl + 1), P->p2p_it_leaf, P->p2p_it_k0, P->p2p_it_k1,
                                               P->p2p_it_out, P->p2p_cl_leaf, P->p2p_cl_part, P->p2p_cl_n);
    FMM_HIP(hipGetLastError());
    al.free(tot);
    al.free(sc);
    al.free(cnt);
}

}  // namespace fmm
