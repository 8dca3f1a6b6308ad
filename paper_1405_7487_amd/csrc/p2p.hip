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
// bodies can coincide with a target, so only that batch tests r^2 > 0.
// Batch partial sums enter the running totals through a compensated (Kahan)
// add.
#include "internal.hpp"

namespace fmm {

namespace {

constexpr int kStage = 256;
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
    T sh[64][3];
};

template <class T, class V4, bool KAHAN, int G>
__device__ void leaf_chunk(V4 *sb, GatherLds<T> *gs, int A, int32_t tb, int base, int cnt, const int32_t *beg, const int32_t *end,
                           int64_t k0, int64_t k1, const int32_t *src, const double *ctr, const V4 *ub, T *phi_s,
                           T *E_s)
{
    // sources per batch: a multiple of G kUnroll, so a padded batch never
    // runs past its kStage slots
    constexpr int SMAX = (kStage / (G * kUnroll)) * (G * kUnroll);
    const int lane = threadIdx.x;
    const int ti = lane / G, sub = lane % G;
    const bool active = ti < cnt;
    const V4 u = ub[tb + base + (active ? ti : 0)];
    const double cax = ctr[3 * A], cay = ctr[3 * A + 1], caz = ctr[3 * A + 2];
    Acc<T> s{0, 0, 0, 0}, c{0, 0, 0, 0};
    auto fold = [&](const Acc<T> &pa) {
        if (KAHAN) {
            kahan_add(s.p, c.p, pa.p);
            kahan_add(s.x, c.x, pa.x);
            kahan_add(s.y, c.y, pa.y);
            kahan_add(s.z, c.z, pa.z);
        } else {
            s.p += pa.p; s.x += pa.x; s.y += pa.y; s.z += pa.z;
        }
    };
    const int32_t ab = beg[A], ae = end[A];
    // 1) the leaf's own bodies (may coincide with the target): masked
    for (int32_t o = ab; o < ae; o += SMAX) {
        const int take = min(SMAX, ae - o);
        const int npad = (take + G * kUnroll - 1) / (G * kUnroll) * (G * kUnroll);
        for (int l = lane; l < npad; l += 64) sb[l] = l < take ? ub[o + l] : far_dummy<T, V4>();
        __syncthreads();
        Acc<T> pa{0, 0, 0, 0};
        batch<T, V4, G, true>(sb, npad, sub, u.x, u.y, u.z, pa);
        fold(pa);
        __syncthreads();
    }
    {
        // 2) every other leaf of the list, batched, no test needed.  A batch is
        //    gathered from the next (up to) 64 list entries at once: lane l takes
        //    entry k + l, a wave prefix sum of the leaf sizes places the bodies,
        //    and every LDS slot finds its leaf by a branchless binary search of
        //    that sum.  The loads of batch i+1 are in flight while batch i is
        //    multiplied (two LDS buffers); slots past the batch hold zero-charge
        //    dummies, which also pad the batch for the unrolled loop.
        int32_t *s_excl = gs->excl, *s_incl = gs->incl, *s_base = gs->base;
        T(*s_sh)[3] = gs->sh;
        int64_t k = k0;
        int32_t o = 0;  // bodies of entry k already consumed
        V4 regs[kStage / 64];
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
            s_sh[lane][0] = (T)(ctr[3 * b] - cax);
            s_sh[lane][1] = (T)(ctr[3 * b + 1] - cay);
            s_sh[lane][2] = (T)(ctr[3 * b + 2] - caz);
            __syncthreads();
            int lo[kStage / 64];
#pragma unroll
            for (int r = 0; r < kStage / 64; ++r) lo[r] = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
#pragma unroll
                for (int r = 0; r < kStage / 64; ++r)
                    if (s_incl[lo[r] + step - 1] <= lane + 64 * r) lo[r] += step;
#pragma unroll
            for (int r = 0; r < kStage / 64; ++r) {
                const int t = lane + 64 * r;
                if (t < staged) {
                    V4 v = ub[s_base[lo[r]] + (t - s_excl[lo[r]])];
                    v.x += s_sh[lo[r]][0];
                    v.y += s_sh[lo[r]][1];
                    v.z += s_sh[lo[r]][2];
                    regs[r] = v;
                } else {
                    regs[r] = far_dummy<T, V4>();
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
            for (int r = 0; r < kStage / 64; ++r) cur[lane + 64 * r] = regs[r];
            const int st_cur = st_next;
            __syncthreads();
            if (k < k1) gather();
            else st_next = 0;
            if (st_cur > 0) {
                const int npad = (st_cur + G * kUnroll - 1) / (G * kUnroll) * (G * kUnroll);
                Acc<T> pa{0, 0, 0, 0};
                batch<T, V4, G, false>(cur, npad, sub, u.x, u.y, u.z, pa);
                fold(pa);
            }
            buf ^= 1;
        }
        __syncthreads();
    }
    if (KAHAN) {
        s.p -= c.p; s.x -= c.x; s.y -= c.y; s.z -= c.z;
    }
    // sum over the G lanes of a target (lanes ti G + [0, G)): a tree in a
    // fixed order, sub 0 ends with the total
#pragma unroll
    for (int w = 1; w < G; w <<= 1) {
        const T op = __shfl_down(s.p, w, 64), ox = __shfl_down(s.x, w, 64);
        const T oy = __shfl_down(s.y, w, 64), oz = __shfl_down(s.z, w, 64);
        if (sub % (2 * w) == 0 && sub + w < G) {
            s.p += op;
            s.x += ox;
            s.y += oy;
            s.z += oz;
        }
    }
    if (active && sub == 0) {
        const int64_t i = tb + base + ti;
        phi_s[i] = s.p;
        E_s[3 * i] = s.x;
        E_s[3 * i + 1] = s.y;
        E_s[3 * i + 2] = s.z;
    }
}

template <class T, class V4, bool KAHAN>
__global__ __launch_bounds__(64) void k_p2p(const int32_t *leaves, const int32_t *beg, const int32_t *end,
                                            const int64_t *off, const int32_t *src, const double *ctr, const V4 *ub,
                                            T *phi_s, T *E_s)
{
    __shared__ V4 sb[2 * kStage];
    __shared__ GatherLds<T> gs;
    const int A = leaves[blockIdx.x];
    const int32_t tb = beg[A], te = end[A];
    const int nt = te - tb;
    const int64_t k0 = off[A], k1 = off[A + 1];
    // chunks of at most 64 targets; a leaf of 33-55 bodies runs as 32 (two
    // lanes each) plus the rest, which keeps more lanes busy than 64-wide
    // chunks with most lanes idle, at the price of a second pass over the list
    for (int base = 0, cnt = 0; base < nt; base += cnt) {
        const int rem = nt - base;
        cnt = (rem > 32 && rem < 56) ? 32 : min(64, rem);
        // lanes per target: G close to 64 / cnt (at most 16), so few lanes idle
#define P2P_CHUNK(GG) leaf_chunk<T, V4, KAHAN, GG>(sb, &gs, A, tb, base, cnt, beg, end, k0, k1, src, ctr, ub, phi_s, E_s)
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

void launch_p2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    const unsigned nb = (unsigned)P->nleaf;
    if (P->precision == FMM_PREC_FP64)
        k_p2p<double, double4, false><<<nb, 64, 0, s>>>(P->leaves, P->c_beg, P->c_end, P->p2p_off,
                                                                P->p2p_src, P->c_ctr, static_cast<const double4 *>(ub),
                                                                static_cast<double *>(phi_s), static_cast<double *>(E_s));
    else if (P->kahan)
        k_p2p<float, float4, true><<<nb, 64, 0, s>>>(P->leaves, P->c_beg, P->c_end, P->p2p_off, P->p2p_src,
                                                             P->c_ctr, static_cast<const float4 *>(ub),
                                                             static_cast<float *>(phi_s), static_cast<float *>(E_s));
    else
        k_p2p<float, float4, false><<<nb, 64, 0, s>>>(P->leaves, P->c_beg, P->c_end, P->p2p_off, P->p2p_src,
                                                              P->c_ctr, static_cast<const float4 *>(ub),
                                                              static_cast<float *>(phi_s), static_cast<float *>(E_s));
    FMM_HIP(hipGetLastError());
}

}  // namespace

void p2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    if (P->nleaf == 0) return;
    launch_p2p(P, ub, phi_s, E_s, s);
}

}  // namespace fmm
