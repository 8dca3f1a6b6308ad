// m2l.hip -- multipole-to-local translations on gfx950 (Section II.A; the
// paper notes that M2L and P2P take more than 90% of the run time).
//
// Same-level pairs.  With level-scaled coefficients the M2L operator between
// two cells of one level depends only on their integer offset t, so the
// translation L(A) += T(t) M(A - t) is a dense p^2 x p^2 product.  A block
// owns a tile of 64 or 128 targets of one level and one octant class (so they
// share one stencil of offsets); for every stencil entry k it multiplies the
// common operator T(t_k) by the gathered source multipoles with MFMA
// (v_mfma_{f32,f64}_16x16x4), accumulating in registers; each target's sum is
// written once, without atomics, in a fixed order.
//
// Cross-level pairs (a leaf against a cell of another level) are keyed by
// level difference and lattice offset: keys with enough pairs get an operator
// of their own and run as shared-operator MFMA products, written per pair and
// summed per target in key order; the rest use a generic kernel that builds
// the operator of the actual offset on the fly.
#include "internal.hpp"

#include <cmath>
#include <type_traits>
#include <vector>

namespace fmm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
// Accumulator e of lane l holds row acc_row(l/16, e) of the 16x16 tile:
// 4 (l/16) + e for float32, l/16 + 4 e for float64.
template <> struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ int acc_row(int g, int e) { return 4 * g + e; }
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ int acc_row(int g, int e) { return g + 4 * e; }
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// The last row tile with at most 4 coefficient rows (float32): one 4x4x1
// MFMA, sixteen 4x4 blocks.  Block b = 4 g + j / 4 (lanes 4 b .. 4 b + 3)
// multiplies A rows i = lane % 4 (the operator stores row 16 (RT - 1) + i in
// fragment lane j) by the inputs of k-group g for columns 4 (j / 4) + jj; lane
// 4 b + jj accumulates rows e = 0..3 of column jj in slot e, a partial sum over
// k-group g that the four groups add at the end.
template <class T>
__device__ __forceinline__ typename Mfma<T>::acc_t mfma_tail(T a, T b, typename Mfma<T>::acc_t c)
{
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
    else return Mfma<T>::run(a, b, c);
}
// Sum of the four k-groups' partials of the tail tile (lanes j, j + 16,
// j + 32, j + 48), in a fixed order; every lane ends with its column's rows.
template <class A>
__device__ __forceinline__ A tail_sum(A v)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] += __shfl_xor(v[e], 16, 64);
        v[e] += __shfl_xor(v[e], 32, 64);
    }
    return v;
}

// Widest vector of T (16 bytes at most) whose length divides SCH.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f1v __attribute__((ext_vector_type(1)));
typedef double d1v __attribute__((ext_vector_type(1)));
template <class T, int SCH> struct BVec;
template <int SCH> struct BVec<float, SCH> {
    static constexpr int n = SCH % 4 == 0 ? 4 : (SCH % 2 == 0 ? 2 : 1);
    typedef typename std::conditional<n == 4, f4v, typename std::conditional<n == 2, f2v, f1v>::type>::type t;
};
template <int SCH> struct BVec<double, SCH> {
    static constexpr int n = SCH % 2 == 0 ? 2 : 1;
    typedef typename std::conditional<n == 2, d2v, d1v>::type t;
};

// Column groups of 16 targets per wave: more groups reuse each operator
// fragment more often but need more accumulator registers.


// Batched same-level M2L.  The stencil of each octant class is cut into
// chunks of E entries; one launch covers G consecutive chunks for every tile,
// and launches run chunk after chunk, so at any time the GPU works on a few
// chunks and their operators stay in L2.  Block b = (chunk c0 + b / ntpos,
// slot b % ntpos of the class-interleaved tile order): consecutive blocks
// alternate over the 8 octant classes, so with workgroups dealt round-robin
// to the 8 XCDs each XCD sees one class and caches only that class's
// operators.  Block = WV waves = one tile of TW = 16 CG WV targets; for every
// stencil entry k of its chunk that has a source in the tile, the block
// stages the common operator T(t_k) in LDS and each wave multiplies it by its
// 16 CG gathered source multipoles:
//     D[i][j] = sum_k A[i][k] B[k][j] (16x16x4 MFMA), A = operator fragment
//     (lane l: A[l%16][l/16]), B = multipoles (lane l: B[l/16][l%16]); lane l
//     accumulates D[acc_row(l/16, e)][l%16] in slot e.
// The loop body has no divergent branch and never edits loaded data: the
// next operator stage and the next entry's sources (slot indices two entries
// ahead) are fetched while the current stage is multiplied; a missing source
// reads the all-zero multipole row zero_row (= ncell).  With G = 1 a block
// adds its sums to L (launches are ordered, so the sum order is fixed); with
// G > 1 it writes partial sums that a reduction adds in chunk order.  The
// four k-groups of a stage sit 16 words apart in LDS bank order when RT is
// odd, so the operator reads of lanes 0-31 do not collide.
typedef __attribute__((address_space(1))) const void gmem_t;
typedef __attribute__((address_space(3))) void lmem_t;

// Copies one operator stage (4 GST elements, contiguous in the table) into an
// LDS buffer: each lane moves 16 bytes straight to LDS (lane l of a wave
// writes at its base + 16 l), ROUNDS rounds of WV KiB per block.
template <class T, int RT, int Q, int WV>
__device__ __forceinline__ void stage_copy(const T *src, T *dst, int wave, int lane)
{
    constexpr int WE = 1024 / (int)sizeof(T);  // elements per wave and round
    constexpr int ROUNDS = m2l_rounds(RT, Q, (int)sizeof(T), WV);
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u) {
        const int o = (u * WV + wave) * WE;
        __builtin_amdgcn_global_load_lds((gmem_t *)(src + o + lane * (16 / (int)sizeof(T))), (lmem_t *)(dst + o), 16,
                                         0, 0);
    }
}

template <class T, int RT, int Q, int CG, int WV, int TR>
__global__ __launch_bounds__(64 * WV) void k_m2l_batched(const int32_t *__restrict__ tile_order, int ntpos,
                                                     const int32_t *__restrict__ tile_cls,
                                                     const int32_t *__restrict__ slots,
                                                     const int32_t *__restrict__ tile_kl,
                                                     const int32_t *__restrict__ tile_nk,
                                                     const int32_t *__restrict__ st_op, int K, int E, int c0, int G,
                                                     const int32_t *__restrict__ slot_none, int zero_row,
                                                     const T *__restrict__ Tf, const T *__restrict__ M,
                                                     T *__restrict__ part, const int32_t *__restrict__ tile_tgt,
                                                     T *__restrict__ L, int64_t ntile)
{
    constexpr int ESZ = (int)sizeof(T);
    constexpr int P2pad = 16 * RT, TW = 16 * CG * WV;
    constexpr bool TAIL = TR > 0 && ESZ == 4;  // the last row tile on 4x4x1 blocks
    constexpr int SCH = m2l_sch(RT, Q, ESZ), NC = Q / SCH, GST = m2l_gst(RT, Q, ESZ);
    constexpr int64_t OPSZ = m2l_opsz(RT, Q, ESZ);
    constexpr int BUF = m2l_rounds(RT, Q, ESZ, WV) * 1024 * WV / ESZ;  // elements per LDS stage buffer
    constexpr int VB = BVec<T, SCH>::n;                   // vector width of the multipole loads
    typedef typename BVec<T, SCH>::t bvec_t;
    typedef typename Mfma<T>::acc_t acc_t;
    __shared__ __align__(16) T lds[2 * BUF];

    const int64_t b = blockIdx.x;
    const int gch = (int)(b / ntpos);
    const int tile = tile_order[b % ntpos];
    if (tile < 0) return;  // an empty slot of the class-interleaved order (whole block)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 15, g = lane >> 4;
    const int cls = tile_cls[tile];
    const int nk = tile_nk[tile];
    const int32_t *kl = tile_kl + (int64_t)tile * K;
    // the tile's listed entries with k in this chunk: [i0, i1) of its sorted list
    const int klo = (c0 + gch) * E, khi = min(K, klo + E);
    int lo = 0, hi = nk;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (kl[mid] < klo) lo = mid + 1;
        else hi = mid;
    }
    const int i0 = lo;
    hi = nk;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (kl[mid] < khi) lo = mid + 1;
        else hi = mid;
    }
    const int i1 = lo;
    if (G == 1 && i0 == i1) return;  // nothing to add (whole block)
    const int32_t *sl = slots + (int64_t)tile * K * TW + wave * CG * 16 + j;
    const int32_t *sl_none = slot_none + wave * CG * 16 + j;  // a row of -1
    const int32_t *opk = st_op + (int64_t)cls * K;

    acc_t acc[CG][RT];
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[cg][r] = acc_t{0, 0, 0, 0};

    if (i0 < i1) {
#define M2L_STAGE(KK, CC, BUFI)                                                                    \
    {                                                                                              \
        int op_ = opk[KK];                                                                         \
        op_ = op_ < 0 ? 0 : op_;                                                                   \
        stage_copy<T, RT, Q, WV>(Tf + (int64_t)op_ * OPSZ + (CC) * 4 * GST, lds + (BUFI) * BUF, wave, lane); \
    }
#define M2L_SLOTS(II, DST)                                                                         \
    {                                                                                              \
        const int32_t *sp_ = (II) < i1 ? sl + (int64_t)kl[II] * TW : sl_none;                      \
        _Pragma("unroll") for (int cg = 0; cg < CG; ++cg) DST[cg] = sp_[cg * 16];                  \
    }
        // multipole values of chunk CC for this lane's columns (rows g Q + CC SCH + [0, SCH))
#define M2L_LOAD_B(SRC, CC, DST)                                                                   \
    {                                                                                              \
        _Pragma("unroll") for (int cg = 0; cg < CG; ++cg)                                          \
        {                                                                                          \
            const int sv = SRC[cg];                                                                \
            const bvec_t *mp = reinterpret_cast<const bvec_t *>(M + (int64_t)(sv < 0 ? zero_row : sv) * P2pad + g * Q + (CC) * SCH); \
            _Pragma("unroll") for (int v = 0; v < SCH / VB; ++v)                                   \
            {                                                                                      \
                const bvec_t x = mp[v];                                                            \
                _Pragma("unroll") for (int w = 0; w < VB; ++w) DST[cg][v * VB + w] = x[w];         \
            }                                                                                      \
        }                                                                                          \
    }
        T bq[2][CG][SCH];
        int sX[CG], sY[CG];
        M2L_SLOTS(i0, sX);
        M2L_SLOTS(i0 + 1, sY);
        M2L_STAGE(kl[i0], 0, 0);
        M2L_LOAD_B(sX, 0, bq[0]);
        // One stencil entry, step by step (a step = one chunk of SCH input
        // rows).  At the top of a step every wave waits for its own copies and
        // loads of this step and meets the others at the barrier, after which
        // the other LDS buffer is free: the next step's operator rows are
        // copied into it and its multipole values loaded into bq[cur ^ 1]
        // while this step is multiplied.  After the last chunk the next
        // entry's first chunk follows (slot indices SN, loaded one entry
        // ahead).  PAR is the parity of chunk 0.  With NC odd the parity
        // alternates, so two entries run per trip (every register role fixed
        // at compile time) and an odd tail runs one entry whose sources are
        // all missing (exact zeros are added).
#define M2L_ENTRY(IT, SC, SN, PAR)                                                                 \
    {                                                                                              \
        const int k_ = kl[min(IT, i1 - 1)];                                                        \
        const int kn_ = kl[min((IT) + 1, i1 - 1)];                                                 \
        bool hv[CG]; /* a column group without any source adds nothing: skip its products */      \
        _Pragma("unroll") for (int cg = 0; cg < CG; ++cg) hv[cg] = __ballot(SC[cg] >= 0) != 0;     \
        _Pragma("unroll") for (int c = 0; c < NC; ++c)                                             \
        {                                                                                          \
            const int cur = ((PAR) + c) & 1;                                                       \
            __builtin_amdgcn_s_waitcnt(0);                                                         \
            __syncthreads();                                                                       \
            if (c + 1 < NC) {                                                                      \
                M2L_STAGE(k_, c + 1, cur ^ 1);                                                     \
                M2L_LOAD_B(SC, c + 1, bq[cur ^ 1]);                                                \
            } else {                                                                               \
                M2L_STAGE(kn_, 0, cur ^ 1);                                                        \
                M2L_LOAD_B(SN, 0, bq[cur ^ 1]);                                                    \
                M2L_SLOTS((IT) + 2, SC);                                                           \
            }                                                                                      \
            const T *sbuf = lds + cur * BUF + g * GST + j * RT;                                    \
            {                                                                                      \
                _Pragma("unroll") for (int ss = 0; ss < SCH; ++ss)                                 \
                {                                                                                  \
                    T a[RT];                                                                       \
                    _Pragma("unroll") for (int r = 0; r < RT; ++r) a[r] = sbuf[ss * P2pad + r];    \
                    _Pragma("unroll") for (int cg = 0; cg < CG; ++cg)                              \
                        if (CG == 1 || hv[cg]) /* (with one group, skipping costs more than it saves) */ \
                            _Pragma("unroll") for (int r = 0; r < RT; ++r)                         \
                                acc[cg][r] = (TAIL && r == RT - 1)                                 \
                                                 ? mfma_tail<T>(a[r], bq[cur][cg][ss], acc[cg][r]) \
                                                 : Mfma<T>::run(a[r], bq[cur][cg][ss], acc[cg][r]); \
                }                                                                                  \
            }                                                                                      \
        }                                                                                          \
    }
        if constexpr (NC % 2 == 0) {
            // every entry starts on buffer 0: one entry per trip, slot roles swapped by copies
            for (int it = i0; it < i1; ++it) {
                M2L_ENTRY(it, sX, sY, 0);
#pragma unroll
                for (int cg = 0; cg < CG; ++cg) {
                    const int t_ = sX[cg];
                    sX[cg] = sY[cg];
                    sY[cg] = t_;
                }
            }
        } else {
            for (int it = i0; it < i1; it += 2) {
                M2L_ENTRY(it, sX, sY, 0);
                M2L_ENTRY(it + 1, sY, sX, 1);
            }
        }
#undef M2L_ENTRY
#undef M2L_STAGE
#undef M2L_SLOTS
#undef M2L_LOAD_B
        // the last prefetch still writes LDS: let it land before the block ends
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
        const int col = wave * CG * 16 + cg * 16 + j;
        constexpr int RM = TAIL ? RT - 1 : RT;  // row tiles in the 16x16 layout
        acc_t tl = acc[cg][RT - 1];
        if (TAIL) tl = tail_sum(tl);  // rows 16 (RT - 1) + e of column col, in every group g
        if (G == 1) {
            const int tgt = tile_tgt[(int64_t)tile * TW + col];
            if (tgt < 0) continue;
            T *dst = L + (int64_t)tgt * P2pad;
#pragma unroll
            for (int r = 0; r < RM; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[16 * r + Mfma<T>::acc_row(g, e)] += acc[cg][r][e];
            if (TAIL && g == 0)
#pragma unroll
                for (int e = 0; e < TR; ++e) dst[16 * (RT - 1) + e] += tl[e];
        } else {
            T *dst = part + (((int64_t)gch * ntile + tile) * TW + col) * P2pad;
#pragma unroll
            for (int r = 0; r < RM; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[16 * r + Mfma<T>::acc_row(g, e)] = acc[cg][r][e];
            if (TAIL)
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[16 * (RT - 1) + 4 * g + e] = g == 0 ? tl[e] : (T)0;
        }
    }
}

__global__ void k_fill_none(int32_t *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = -1;
}

// Per tile, the stencil entries with at least one source (flags set by the
// traversal), in stencil order.
__global__ __launch_bounds__(256) void k_tile_klist(const uint8_t *kflag, int K, int32_t *kl, int32_t *nk)
{
    const int64_t tile = blockIdx.x;
    const uint8_t *fl = kflag + tile * (int64_t)K;
    __shared__ int32_t s_cnt[4];
    __shared__ int32_t s_base;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k0 = 0; k0 < K; k0 += 256) {
        const int k = k0 + threadIdx.x;
        const bool any = k < K && fl[k] != 0;
        const uint64_t m = __ballot(any);
        if (lane == 0) s_cnt[wave] = __popcll(m);
        __syncthreads();
        int off = s_base;
        for (int w = 0; w < wave; ++w) off += s_cnt[w];
        if (any) kl[tile * (int64_t)K + off + __popcll(m & ((1ull << lane) - 1))] = k;
        __syncthreads();
        if (threadIdx.x == 0) s_base += s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) nk[tile] = s_base;
}

// Sum of the tiles' entry counts (rows the batched kernel multiplies).
__global__ __launch_bounds__(1024) void k_sum_rows(const int32_t *nk, int64_t ntile, unsigned long long *out)
{
    __shared__ unsigned long long part[16];
    unsigned long long t = 0;
    for (int64_t i = threadIdx.x; i < ntile; i += blockDim.x) t += (unsigned long long)nk[i];
    for (int w = 32; w >= 1; w >>= 1) t += __shfl_xor(t, w, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += part[w];
        *out = a;
    }
}

// L += the G partial products of each target, in chunk order.
template <class T>
__global__ __launch_bounds__(256) void k_m2l_reduce(const T *part, int G, int64_t ncol, int P2pad,
                                                    const int32_t *tile_tgt, T *L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pos = t / P2pad;
    const int row = (int)(t % P2pad);
    if (pos >= ncol) return;
    const int tgt = tile_tgt[pos];
    if (tgt < 0) return;
    T s = L[(int64_t)tgt * P2pad + row];
    for (int k = 0; k < G; ++k) s += part[((int64_t)k * ncol + pos) * P2pad + row];
    L[(int64_t)tgt * P2pad + row] = s;
}

// ------------------------------------------------------- cross-level pairs
struct cd {
    double re, im;
};

__device__ __forceinline__ cd hget(const cd *H, int nmax, int n, int m)
{
    if (n < 0 || n >= nmax || m > n || m < -n) return {0.0, 0.0};
    if (m >= 0) return H[n * (n + 1) / 2 + m];
    cd v = H[n * (n + 1) / 2 - m];
    return (m & 1) ? cd{-v.re, v.im} : cd{v.re, -v.im};
}

__device__ __forceinline__ void rdecode(int r, int &n, int &m, int &im)
{
    n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    const int o = r - n * n;
    if (o == 0) { m = 0; im = 0; }
    else { m = (o + 1) / 2; im = (o & 1) ? 0 : 1; }
}

// Cross-level pairs left to the generic path, one 64-thread block (one wave)
// per chunk of at most kGChunk pairs of one target, float64 arithmetic in the
// complex form.  For a source of level l_B and a target of level l_A, with
// tau = (c_A - c_B)/h_A and rho = h_B/h_A:
//     Lt_j^s += (-1)^j sum_{n<p} rho^n sum_{m=-n..n} Mt_n^m I_{n+j}^{m+s}(tau),
// M^{-m} = (-1)^m conj(M^m), I^{-l} = (-1)^l conj(I^l).  Lane t owns the
// outputs (j, s >= 0) numbered t, t + 64 and t + 128 and sums over the
// chunk's pairs in list order; the chunk's sums go to part[chunk] (float64).
// The block's barriers are reached by the whole block.
constexpr int kGChunk = 16;
constexpr int kOutSlots = (kMaxP * (kMaxP + 1) / 2 + 63) / 64;

template <class TM>
__global__ __launch_bounds__(64) void k_m2l_cross(const int32_t *ch_tgt, const int64_t *ch_k0, const int64_t *off,
                                                  const int32_t *src, const int32_t *lvl, const double *ctr,
                                                  double S, int p, int P2pad, const TM *M, double *part)
{
    const int lane = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int c = ch_tgt[chunk];
    const int64_t k0 = ch_k0[chunk], k1 = min(k0 + (int64_t)kGChunk, off[c + 1]);
    __shared__ cd H[(2 * kMaxP) * (2 * kMaxP + 1) / 2];
    __shared__ cd Ms[kMaxP * (kMaxP + 1) / 2];
    const int nI = 2 * p - 1, P2 = p * p, NO = p * (p + 1) / 2;
    const double hA = ldexp(S, -lvl[c]);
    // output (j, s) of each of this lane's slots
    int oj[kOutSlots], os[kOutSlots];
    for (int q = 0; q < kOutSlots; ++q) {
        const int t = lane + 64 * q;
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= t) ++j;
        oj[q] = t < NO ? j : -1;
        os[q] = t - j * (j + 1) / 2;
    }
    double are[kOutSlots] = {}, aim[kOutSlots] = {};
    for (int64_t k = k0; k < k1; ++k) {
        const int b = src[k];
        const double tx = (ctr[3 * c] - ctr[3 * b]) / hA, ty = (ctr[3 * c + 1] - ctr[3 * b + 1]) / hA,
                     tz = (ctr[3 * c + 2] - ctr[3 * b + 2]) / hA;
        const int dl = lvl[c] - lvl[b];
        const double r2 = tx * tx + ty * ty + tz * tz, ir2 = 1.0 / r2;
        if (lane == 0) {
            cd mm = {1.0 / sqrt(r2), 0.0};
            for (int m = 0; m < nI; ++m) {
                if (m > 0) {
                    const double f = -(2.0 * m - 1.0) * ir2;
                    mm = cd{(mm.re * tx - mm.im * ty) * f, (mm.re * ty + mm.im * tx) * f};
                }
                H[m * (m + 1) / 2 + m] = mm;
            }
        }
        // source multipole as complex coefficients, scaled by rho^n
        const TM *mb = M + (int64_t)b * P2pad;
        for (int r = lane; r < P2; r += 64) {
            const int n = (int)sqrtf((float)r + 0.5f);
            const int o = r - n * n;
            const double sc = ldexp(1.0, n * dl);
            if (o == 0) Ms[n * (n + 1) / 2] = cd{sc * (double)mb[r], 0.0};
            else if (o & 1) {
                const int m = (o + 1) / 2;
                Ms[n * (n + 1) / 2 + m] = cd{sc * (double)mb[r], sc * (double)mb[r + 1]};
            }
        }
        __syncthreads();
        if (lane < nI) {
            const int m = lane;
            cd mm = H[m * (m + 1) / 2 + m], p2 = {0, 0}, p1 = mm;
            for (int n = m + 1; n < nI; ++n) {
                cd cur;
                if (n == m + 1) cur = cd{mm.re * (2.0 * m + 1.0) * tz * ir2, mm.im * (2.0 * m + 1.0) * tz * ir2};
                else {
                    const double a = (2.0 * n - 1.0) * tz, bb = -(double)((n + m - 1) * (n - m - 1));
                    cur = cd{(a * p1.re + bb * p2.re) * ir2, (a * p1.im + bb * p2.im) * ir2};
                }
                H[n * (n + 1) / 2 + m] = cur;
                p2 = p1;
                p1 = cur;
            }
        }
        __syncthreads();
        for (int q = 0; q < kOutSlots; ++q) {
            const int j = oj[q], sO = os[q];
            if (j < 0) continue;
            double sr = 0.0, si = 0.0;
            for (int n = 0; n < p; ++n) {
                const int kk = n + j;
                const cd *Hk = H + kk * (kk + 1) / 2;
                const cd *Mn = Ms + n * (n + 1) / 2;
                for (int m = -n; m <= n; ++m) {
                    cd mv = Mn[m < 0 ? -m : m];
                    if (m < 0) mv = (m & 1) ? cd{-mv.re, mv.im} : cd{mv.re, -mv.im};
                    const int l = m + sO;  // |l| <= kk always
                    cd iv = Hk[l < 0 ? -l : l];
                    if (l < 0) iv = (l & 1) ? cd{-iv.re, iv.im} : cd{iv.re, -iv.im};
                    sr += mv.re * iv.re - mv.im * iv.im;
                    si += mv.re * iv.im + mv.im * iv.re;
                }
            }
            are[q] += sr;
            aim[q] += si;
        }
        __syncthreads();
    }
    double *dp = part + chunk * P2pad;
    for (int q = 0; q < kOutSlots; ++q) {
        const int j = oj[q], sO = os[q];
        if (j < 0) continue;
        const double sg = (j & 1) ? -1.0 : 1.0;
        if (sO == 0) dp[j * j] = sg * are[q];
        else {
            const int r = j * j + 2 * sO - 1;
            dp[r] = sg * are[q];
            dp[r + 1] = sg * aim[q];
        }
    }
}


// L[c] += sum of the cell's generic-chunk sums, in chunk order.
template <class TM>
__global__ __launch_bounds__(256) void k_gx_reduce(int64_t nc, const int64_t *cofs, const double *part, int P2,
                                                   int P2pad, TM *L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = t / P2;
    const int r = (int)(t % P2);
    if (c >= nc) return;
    const int64_t a = cofs[c], b = cofs[c + 1];
    if (a == b) return;
    const double acc = strided_sum(part + a * P2pad + r, b - a, (int64_t)P2pad);
    TM *dst = L + c * P2pad + r;
    *dst = (TM)((double)*dst + acc);
}

__global__ __launch_bounds__(256) void k_gx_count(const int64_t *off, int64_t nc, int32_t *cnt)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc) return;
    cnt[c] = c < nc ? (int32_t)((off[c + 1] - off[c] + kGChunk - 1) / kGChunk) : 0;
}

__global__ __launch_bounds__(256) void k_gx_fill(const int64_t *off, const int64_t *cofs, int64_t nc,
                                                 int32_t *ch_tgt, int64_t *ch_k0)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    for (int64_t i = cofs[c]; i < cofs[c + 1]; ++i) {
        ch_tgt[i] = (int32_t)c;
        ch_k0[i] = off[c] + (i - cofs[c]) * kGChunk;
    }
}

// ------------------------------------------- batched cross-level pairs
//
// A cross-level pair joins a leaf A and a cell B of another level.  With
// lattice centers, the operator depends only on the key (dl, D): the level
// difference dl = l_B - l_A and the center offset D = C_A - C_B in half-units
// of the finer cell (tau = D 2^-max(dl,0) / 2 in units of h_A, rho = 2^-dl).
// Keys with |dl| <= kXMaxDl and enough pairs get an operator of their own and
// run as shared-operator MFMA products, tiles of TW pairs of one key; the
// products go to a per-pair buffer, chunk by chunk, and a reduction adds them
// to each target in (key) order, so the sums are deterministic.  All other
// cross pairs use k_m2l_cross.

constexpr int kXMaxDl = 2;
constexpr int kXMinPairs = 64;
constexpr int kXStripes = 8;

// Code of the key (dl, D), or -1 when the pair is left to the generic kernel.
struct XCodes {
    int maxdl = 0;
    int R[kXMaxDl + 1] = {0, 0, 0};
    int base[2 * kXMaxDl + 1] = {0, 0, 0, 0, 0};
    int64_t ncode = 0;
};

__global__ __launch_bounds__(256) void k_x_targets(const int64_t *off, int64_t nc, int32_t *tgt)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    for (int64_t k = off[c]; k < off[c + 1]; ++k) tgt[k] = (int32_t)c;
}

__global__ __launch_bounds__(256) void k_x_codes(const int32_t *tgt, const int32_t *src, int64_t nx,
                                                 const int32_t *lvl, const int32_t *ix, XCodes xc, int32_t *code,
                                                 int32_t *cnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nx) return;
    const int a = tgt[k], b = src[k];
    const int la = lvl[a], lb = lvl[b], dl = lb - la;
    const int adl = dl < 0 ? -dl : dl;
    int cd = -1;
    if (adl <= xc.maxdl && xc.R[adl] > 0) {
        const int f = la > lb ? la : lb, R = xc.R[adl], W = 2 * R + 1;
        int64_t D[3];
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            const int64_t ca = (2 * (int64_t)ix[3 * a + d] + 1) << (f - la);
            const int64_t cb = (2 * (int64_t)ix[3 * b + d] + 1) << (f - lb);
            D[d] = ca - cb;
            ok = ok && D[d] >= -R && D[d] <= R;
        }
        if (ok) {
            cd = xc.base[dl + kXMaxDl] + (int)(((D[0] + R) * W + (D[1] + R)) * W + (D[2] + R));
            // one of kXStripes copies of the histogram: popular keys take
            // millions of increments, which one counter would serialise
            atomicAdd(&cnt[(int64_t)(blockIdx.x % kXStripes) * xc.ncode + cd], 1);
        }
    }
    code[k] = cd;
}

// cnt[c] = the sum of the kXStripes histogram copies.
__global__ __launch_bounds__(256) void k_x_sum_stripes(int32_t *cnt, int64_t ncode)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncode) return;
    int32_t t = cnt[c];
    for (int k = 1; k < kXStripes; ++k) t += cnt[k * ncode + c];
    cnt[c] = t;
}

// The shared-operator tiles of key id: tile tile0[id] + j covers pairs
// pair0[id] + j TW onwards (at most TW of the key's count).
__global__ __launch_bounds__(256) void k_x_tiles(const int64_t *tile0, const int64_t *pair0, const int64_t *cnt,
                                                 int TW, int32_t *xt_op, int64_t *xt_first, int32_t *xt_cnt)
{
    const int id = blockIdx.x;
    const int64_t t0 = tile0[id], nt = tile0[id + 1] - t0;
    for (int64_t j = threadIdx.x; j < nt; j += blockDim.x) {
        xt_op[t0 + j] = id;
        xt_first[t0 + j] = pair0[id] + j * TW;
        xt_cnt[t0 + j] = (int32_t)min((int64_t)TW, cnt[id] - j * TW);
    }
}

// Sort key (key id, target) for batched pairs; generic pairs get id = nk and
// are counted per target.
__global__ __launch_bounds__(256) void k_x_key1(const int32_t *tgt, const int32_t *src, const int32_t *code,
                                                const int32_t *id_of, int nk, int64_t nx, uint64_t *k1, int32_t *v1,
                                                int32_t *gcnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nx) return;
    const int cd = code[k];
    const int id = cd >= 0 ? id_of[cd] : -1;
    const int32_t a = tgt[k];
    if (id < 0) atomicAdd(&gcnt[a], 1);
    k1[k] = ((uint64_t)(uint32_t)(id < 0 ? nk : id) << 32) | (uint32_t)a;
    v1[k] = src[k];
}

// Sort key (chunk, target, key id) of each batched pair; value = its position.
// (chunk, target, key) packed as chunk << cs | target << 21 | key
__global__ __launch_bounds__(256) void k_x_key2(const uint64_t *k1, int64_t nb, const int32_t *chunk_of, int cs,
                                                uint64_t *k2, int32_t *v2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const uint64_t id = k1[i] >> 32, a = k1[i] & 0xffffffffull;
    k2[i] = ((uint64_t)(uint32_t)chunk_of[id] << cs) | (a << 21) | id;
    v2[i] = (int32_t)i;
}

// inv[pos[i]] = i: the reduce-order position of each pair in key order
__global__ __launch_bounds__(256) void k_x_invert(const int32_t *pos, int64_t nb, int32_t *inv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) inv[pos[i]] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_x_segflag(const uint64_t *k2, int64_t nb, int32_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    flag[i] = (i == 0 || (k2[i] >> 21) != (k2[i - 1] >> 21)) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_x_segments(const uint64_t *k2, const int32_t *flag, const int64_t *sidx,
                                                    int64_t nb, int cs, int64_t *s_off, int32_t *s_tgt,
                                                    int64_t *chunk_seg0)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb || !flag[i]) return;
    const int64_t seg = sidx[i];
    s_off[seg] = i;
    s_tgt[seg] = (int32_t)((k2[i] >> 21) & ((1ull << (cs - 21)) - 1ull));
    const uint64_t ch = k2[i] >> cs;
    if (i == 0 || (k2[i - 1] >> cs) != ch) chunk_seg0[ch] = seg;
}

// One tile of TW pairs sharing one operator: out[rpos(pair)] = T(key) M[src(pair)],
// rpos = the pair's position in (chunk, target, key) order, so each target's
// products lie together for the reduction.
// Block = WV waves; the operator passes through two LDS stage buffers, the
// next stage copied while the current one is multiplied.
template <class T, int RT, int Q, int CG, int WV, int TR>
__global__ __launch_bounds__(64 * WV) void k_m2l_pairs(const int32_t *__restrict__ t_op,
                                                   const int64_t *__restrict__ t_first,
                                                   const int32_t *__restrict__ t_cnt, const int32_t *__restrict__ src,
                                                   const int32_t *__restrict__ rpos, int zero_row,
                                                   const T *__restrict__ Tf, const T *__restrict__ M,
                                                   T *__restrict__ out, int64_t pos0)
{
    constexpr int ESZ = (int)sizeof(T);
    constexpr int P2pad = 16 * RT;
    constexpr bool TAIL = TR > 0 && ESZ == 4;  // the last row tile on 4x4x1 blocks
    constexpr int SCH = m2l_sch(RT, Q, ESZ), NC = Q / SCH, GST = m2l_gst(RT, Q, ESZ);
    constexpr int BUF = m2l_rounds(RT, Q, ESZ, WV) * 1024 * WV / ESZ;
    constexpr int VN = BVec<T, Q>::n;
    typedef typename BVec<T, Q>::t vec_t;
    typedef typename Mfma<T>::acc_t acc_t;
    __shared__ __align__(16) T lds[2 * BUF];

    const int64_t tile = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 15, g = lane >> 4;
    const int cnt = t_cnt[tile];
    const int64_t first = t_first[tile];
    constexpr int64_t OPSZ = m2l_opsz(RT, Q, ESZ);
    const T *opb = Tf + (int64_t)t_op[tile] * OPSZ;

    stage_copy<T, RT, Q, WV>(opb, lds, wave, lane);
    T bq[CG][Q];
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
        const int col = wave * CG * 16 + cg * 16 + j;
        const int sv = col < cnt ? src[first + col] : zero_row;
        const vec_t *mp = reinterpret_cast<const vec_t *>(M + (int64_t)sv * P2pad + g * Q);
#pragma unroll
        for (int v = 0; v < Q / VN; ++v) {
            const vec_t x = mp[v];
#pragma unroll
            for (int w = 0; w < VN; ++w) bq[cg][v * VN + w] = x[w];
        }
    }
    acc_t acc[CG][RT];
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[cg][r] = acc_t{0, 0, 0, 0};

#pragma unroll
    for (int c = 0; c < NC; ++c) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (c + 1 < NC) stage_copy<T, RT, Q, WV>(opb + (c + 1) * 4 * GST, lds + ((c + 1) & 1) * BUF, wave, lane);
        const T *sbuf = lds + (c & 1) * BUF + g * GST + j * RT;
#pragma unroll
        for (int ss = 0; ss < SCH; ++ss) {
            T a[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) a[r] = sbuf[ss * P2pad + r];
#pragma unroll
            for (int cg = 0; cg < CG; ++cg)
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    acc[cg][r] = (TAIL && r == RT - 1) ? mfma_tail<T>(a[r], bq[cg][c * SCH + ss], acc[cg][r])
                                                       : Mfma<T>::run(a[r], bq[cg][c * SCH + ss], acc[cg][r]);
        }
    }
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
        const int col = wave * CG * 16 + cg * 16 + j;
        constexpr int RM = TAIL ? RT - 1 : RT;
        acc_t tl = acc[cg][RT - 1];
        if (TAIL) tl = tail_sum(tl);  // every lane takes part in the exchange
        if (col >= cnt) continue;
        T *dst = out + ((int64_t)rpos[first + col] - pos0) * P2pad;
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[16 * r + Mfma<T>::acc_row(g, e)] = acc[cg][r][e];
        if (TAIL)
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[16 * (RT - 1) + 4 * g + e] = g == 0 ? tl[e] : (T)0;
    }
}

// L[target] += sum of its pairs' products in this chunk, in key order (the
// sum in float64).  One thread per (segment, coefficient).
template <class T>
__global__ __launch_bounds__(256) void k_x_reduce(const int64_t *s_off, const int32_t *s_tgt, int64_t nseg,
                                                  int64_t pos0, const T *buf, int P2pad, T *L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t seg = t / P2pad;
    const int row = (int)(t % P2pad);
    if (seg >= nseg) return;
    const int64_t k0 = s_off[seg];
    const double acc = strided_sum(buf + (k0 - pos0) * P2pad + row, s_off[seg + 1] - k0, (int64_t)P2pad);
    T *dst = L + (int64_t)s_tgt[seg] * P2pad + row;
    *dst = (T)((double)*dst + acc);
}

__global__ void k_mfma_probe_f32(float *out)
{
    const int l = threadIdx.x;
    v4f acc = {0, 0, 0, 0};
    // A[i][k] = i + 1 + 100 k (lane i + 16 k); B[k][j] = 1 + 1000 j for k = 0, else 0
    // (lane j + 16 k); so D[i][j] = (i + 1)(1 + 1000 j)
    const float a = (float)((l & 15) + 1 + 100 * (l >> 4));
    const float b = (l >> 4) == 0 ? 1.0f + (float)(l & 15) * 1000.0f : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    for (int e = 0; e < 4; ++e) out[l * 4 + e] = acc[e];
}
__global__ void k_mfma_probe_f32_4x4(float *out)
{
    const int l = threadIdx.x;
    v4f acc = {0, 0, 0, 0};
    // block b = l / 4: A_b[i] = i + 1 + 16 b (lane 4 b + i), B_b[jj] = 1 + 1000 jj
    // (lane 4 b + jj); so D_b[i][jj] = (i + 1 + 16 b)(1 + 1000 jj)
    const float a = (float)((l & 3) + 1 + 16 * (l >> 2));
    const float b = 1.0f + (float)(l & 3) * 1000.0f;
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc, 0, 0, 0);
    for (int e = 0; e < 4; ++e) out[l * 4 + e] = acc[e];
}
__global__ void k_mfma_probe_f64(double *out)
{
    const int l = threadIdx.x;
    v4d acc = {0, 0, 0, 0};
    const double a = (double)((l & 15) + 1 + 100 * (l >> 4));
    const double b = (l >> 4) == 0 ? 1.0 + (double)(l & 15) * 1000.0 : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int e = 0; e < 4; ++e) out[l * 4 + e] = acc[e];
}

// Launches chunk after chunk (G chunks at a time) over every tile.
template <class T, int RT, int Q, int TR>
void launch_batched(fmm_plan *P, hipStream_t s)
{
    constexpr int CG = m2l_cg(RT, sizeof(T) == 8), WV = m2l_wv(RT, sizeof(T) == 8);
    FMM_CHECK(P->TW == 16 * CG * WV, FMM_ERR_DEVICE, "m2l: tile width mismatch");
    const int ntpos = 8 * P->TPC;
    for (int c0 = 0; c0 < P->NCH; c0 += P->G) {
        const int g = std::min(P->G, P->NCH - c0);
        const int64_t nb = (int64_t)g * ntpos;
        FMM_CHECK(nb * 64 * WV < (1ll << 32), FMM_ERR_UNSUPPORTED, "m2l: too many tiles");
        k_m2l_batched<T, RT, Q, CG, WV, TR><<<(unsigned)nb, 64 * WV, 0, s>>>(
            P->tile_order, ntpos, P->tile_cls, P->slots, P->tile_kl, P->tile_nk, P->st_op, P->K, P->E, c0, g,
            P->slot_none, (int)P->ncell, static_cast<const T *>(P->ops), static_cast<const T *>(P->Mc),
            static_cast<T *>(P->m2l_part), P->tile_tgt, static_cast<T *>(P->Lc), P->ntile);
        FMM_HIP(hipGetLastError());
        if (g > 1) {
            const int64_t ncol = P->ntile * P->TW;
            k_m2l_reduce<T><<<grid1(ncol * P->P2pad, 256), 256, 0, s>>>(static_cast<const T *>(P->m2l_part), g, ncol,
                                                                       P->P2pad, P->tile_tgt,
                                                                       static_cast<T *>(P->Lc));
            FMM_HIP(hipGetLastError());
        }
    }
}

// One instantiation per expansion order (row tiles and input steps follow from p).
#define M2L_FOR_EACH_P(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <class T>
void dispatch_tiles(fmm_plan *P, hipStream_t s)
{
    switch (P->p) {
#define M2L_CASE(pp)                                             \
    case pp: launch_batched<T, m2l_rt(pp), m2l_q(pp), m2l_tail_rows(pp)>(P, s); break;
        M2L_FOR_EACH_P(M2L_CASE)
#undef M2L_CASE
    default: throw Error(FMM_ERR_UNSUPPORTED, "m2l: unsupported expansion order");
    }
}

template <class T, int RT, int Q, int TR>
void launch_pairs(fmm_plan *P, const XChunk &ch, hipStream_t s)
{
    constexpr int CG = m2l_cg(RT, sizeof(T) == 8), WV = m2l_wv(RT, sizeof(T) == 8);
    FMM_CHECK(P->TW == 16 * CG * WV, FMM_ERR_DEVICE, "m2l: tile width mismatch");
    const int64_t nt = ch.t1 - ch.t0;
    FMM_CHECK(nt * 64 * WV < (1ll << 32), FMM_ERR_UNSUPPORTED, "m2l: too many cross tiles");
    if (nt > 0) {
        k_m2l_pairs<T, RT, Q, CG, WV, TR><<<(unsigned)nt, 64 * WV, 0, s>>>(
            P->xt_op + ch.t0, P->xt_first + ch.t0, P->xt_cnt + ch.t0, P->xp_src, P->xr_inv, (int)P->ncell,
            static_cast<const T *>(P->xops), static_cast<const T *>(P->Mc), static_cast<T *>(P->xbuf), ch.p0);
        FMM_HIP(hipGetLastError());
    }
    const int64_t ns = ch.s1 - ch.s0;
    if (ns > 0) {
        k_x_reduce<T><<<grid1(ns * P->P2pad, 256), 256, 0, s>>>(P->xs_off + ch.s0, P->xs_tgt + ch.s0, ns, ch.p0, static_cast<const T *>(P->xbuf), P->P2pad,
                                                               static_cast<T *>(P->Lc));
        FMM_HIP(hipGetLastError());
    }
}

template <class T>
void dispatch_pairs(fmm_plan *P, const XChunk &ch, hipStream_t s)
{
    switch (P->p) {
#define M2L_CASE(pp)                                                    \
    case pp: launch_pairs<T, m2l_rt(pp), m2l_q(pp), m2l_tail_rows(pp)>(P, ch, s); break;
        M2L_FOR_EACH_P(M2L_CASE)
#undef M2L_CASE
    default: throw Error(FMM_ERR_UNSUPPORTED, "m2l: unsupported expansion order");
    }
}

int bits_of(int64_t v)
{
    int b = 1;
    while ((1ll << b) <= v) ++b;
    return b;
}

}  // namespace

int m2l_tile_width(int p, bool f64)
{
    const int RT = p2pad_of(p) / 16;
    return 16 * m2l_cg(RT, f64) * m2l_wv(RT, f64);
}

// Chunking of the stencils and the class-interleaved tile order.  Chunks
// hold E entries whose operators fit comfortably in one XCD's L2 next to the
// gathered multipoles; G chunks share a launch when there are too few tiles
// to fill the chip, and with very few tiles the chunks are shortened so that
// the launch still has enough blocks.
void m2l_prepare(fmm_plan *P, hipStream_t s)
{
    P->NCH = 0;
    P->G = 1;
    if (P->ntile <= 0 || P->K <= 0) return;
    P->tile_kl = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->ntile * P->K));
    P->slot_none = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->TW));
    k_fill_none<<<1, 256, 0, s>>>(P->slot_none, P->TW);
    P->tile_nk = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->ntile));
    k_tile_klist<<<(unsigned)P->ntile, 256, 0, s>>>(P->tile_kflag, P->K, P->tile_kl, P->tile_nk);
    FMM_HIP(hipGetLastError());
    // (read by the host after the build's final synchronisation)
    P->d_m2l_rows = static_cast<unsigned long long *>(plan_alloc(P, sizeof(unsigned long long)));
    k_sum_rows<<<1, 1024, 0, s>>>(P->tile_nk, P->ntile, P->d_m2l_rows);
    FMM_HIP(hipGetLastError());

    const size_t esz = P->precision == FMM_PREC_FP64 ? sizeof(double) : sizeof(float);
    const double opbytes = (double)m2l_opsz(P->P2pad / 16, m2l_q(P->p), (int)esz) * esz;
    const bool many = P->ntile >= 1024;
    const double budget = many ? 2.5 * 1048576.0 : 2.0 * 1048576.0;
    // entries per chunk: what the operator budget allows, but short enough
    // that tiles x chunks gives about 4096 blocks when the tiles are few
    // (each block walks its entries one after another)
    const int64_t e_fill = ((int64_t)P->K * P->ntile + 4095) / 4096;
    P->E = (int)std::max<int64_t>(8, std::min<int64_t>({(int64_t)P->K, (int64_t)(budget / opbytes), e_fill}));
    P->NCH = (P->K + P->E - 1) / P->E;
    P->G = many ? 1 : (int)std::min<int64_t>(P->NCH, (8192 + P->ntile - 1) / P->ntile);
    if (P->G > 1)
        P->m2l_part = plan_alloc(P, esz * (size_t)P->G * P->ntile * P->TW * P->P2pad);

    // class-interleaved order: slot 8 i + c holds the i-th tile of class c
    const std::vector<int32_t> &cls = P->h_tile_cls;
    std::vector<std::vector<int32_t>> by(8);
    for (int64_t t = 0; t < P->ntile; ++t) by[cls[t] & 7].push_back((int32_t)t);
    size_t tpc = 0;
    for (auto &v : by) tpc = std::max(tpc, v.size());
    P->TPC = (int)tpc;
    std::vector<int32_t> &order = P->h_tile_order;  // kept: the copy's source
    order.assign(std::max<size_t>(1, 8 * tpc), -1);
    for (int c = 0; c < 8; ++c)
        for (size_t i = 0; i < by[c].size(); ++i) order[8 * i + c] = by[c][i];
    P->tile_order = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * order.size()));
    FMM_HIP(hipMemcpyAsync(P->tile_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice, s));
}

void m2l_same(fmm_plan *P, hipStream_t s)
{
    const bool f64 = P->precision == FMM_PREC_FP64;
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    // every local expansion starts from zero; the chunks add to it
    FMM_HIP(hipMemsetAsync(P->Lc, 0, esz * P->P2pad * P->ncell, s));
    if (P->ntile > 0 && P->K > 0 && P->m2l_rows > 0) {
        if (f64) dispatch_tiles<double>(P, s);
        else dispatch_tiles<float>(P, s);
    }
}

namespace {

// Groups the cross-level pairs by key, builds the operators of the frequent
// keys, the tiles, the chunks and the reduction segments, and the CSR of the
// pairs left to the generic kernel.
void x_batch_prepare(fmm_plan *P, hipStream_t s)
{
    const int64_t nx = P->n_m2lx, nc = P->ncell;
    Allocator &al = P->al;
    const bool f64 = P->precision == FMM_PREC_FP64;
    const size_t esz = f64 ? sizeof(double) : sizeof(float);

    // Key (dl, D): level difference dl = l_B - l_A and center offset D in
    // half sides of the finer cell.  Same-level pairs (dl = 0, from sparse
    // slot rows) have D = 2 t with t in the stencil, |t_d| <= R.
    XCodes xc;
    for (int maxdl = kXMaxDl; maxdl >= 1; --maxdl) {
        xc = XCodes();
        xc.maxdl = maxdl;
        int64_t base = 0;
        xc.R[0] = P->n_m2l_sparse > 0 ? 2 * P->R : 0;
        for (int adl = 1; adl <= maxdl; ++adl)
            xc.R[adl] = (int)std::ceil(std::sqrt(3.0) * ((std::ldexp(1.0, adl) + 2.0) / P->theta + 1.0));
        for (int dl = -maxdl; dl <= maxdl; ++dl) {
            if (xc.R[dl < 0 ? -dl : dl] == 0) continue;
            const int64_t W = 2 * xc.R[dl < 0 ? -dl : dl] + 1;
            xc.base[dl + kXMaxDl] = (int)base;
            base += W * W * W;
        }
        xc.ncode = base;
        if (base <= (1ll << 24)) break;
    }
    if (xc.ncode > (1ll << 24)) return;  // theta too small for a dense key table: all generic

    int32_t *tgt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nx));
    int32_t *code = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nx));
    int32_t *cnt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * kXStripes * xc.ncode));
    FMM_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * kXStripes * xc.ncode, s));
    k_x_targets<<<grid1(nc, 256), 256, 0, s>>>(P->m2lx_off, nc, tgt);
    k_x_codes<<<grid1(nx, 256), 256, 0, s>>>(tgt, P->m2lx_src, nx, P->c_lvl, P->c_ix, xc, code, cnt);
    FMM_HIP(hipGetLastError());
    k_x_sum_stripes<<<grid1(xc.ncode, 256), 256, 0, s>>>(cnt, xc.ncode);
    FMM_HIP(hipGetLastError());
    std::vector<int32_t> hc(xc.ncode);
    FMM_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * xc.ncode, hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));

    // keys with enough pairs, in code order; their operators' (tau, e)
    std::vector<int32_t> id_of(xc.ncode, -1), key_cnt;
    std::vector<double4> tr;
    for (int dl = -xc.maxdl; dl <= xc.maxdl; ++dl) {
        if (xc.R[dl < 0 ? -dl : dl] == 0) continue;
        const int R = xc.R[dl < 0 ? -dl : dl], W = 2 * R + 1, b0 = xc.base[dl + kXMaxDl];
        const double sc = std::ldexp(0.5, -std::max(dl, 0));
        for (int64_t o = 0; o < (int64_t)W * W * W; ++o) {
            const int64_t cd = b0 + o;
            if (hc[cd] < kXMinPairs) continue;
            id_of[cd] = (int32_t)key_cnt.size();
            key_cnt.push_back(hc[cd]);
            const int dx = (int)(o / ((int64_t)W * W)) - R, dy = (int)((o / W) % W) - R, dz = (int)(o % W) - R;
            tr.push_back(make_double4(dx * sc, dy * sc, dz * sc, (double)(-dl)));
        }
    }
    const int nk = (int)key_cnt.size();
    if (nk == 0) {
        al.free(cnt);
        al.free(code);
        al.free(tgt);
        return;
    }
    FMM_CHECK(nk < (1 << 21), FMM_ERR_UNSUPPORTED, "m2l: too many cross-level keys");

    // tiles of TW pairs per key; chunks of whole keys whose products fit the buffer
    const int TW = P->TW;
    // buffer of per-pair products: a quarter of all of them, within [2, 16] GiB
    // (each chunk's reduction reads and writes every target it touches once)
    int64_t allpairs = 0;
    for (int id = 0; id < nk; ++id) allpairs += key_cnt[id];
    const int64_t pbytes = (int64_t)P->P2pad * (int64_t)esz;
    // (a plan that may not allocate keeps it at 16 MiB: more chunks, same sums)
    const int64_t bbytes = P->noalloc ? (16ll << 20)
                                      : std::min<int64_t>(16ll << 30, std::max<int64_t>(2ll << 30, allpairs * pbytes / 4));
    const int64_t budget = std::max<int64_t>((int64_t)TW, bbytes / pbytes);
    // per key: first tile, first pair and pair count (the tiles themselves
    // are filled on the device)
    std::vector<int32_t> chunk_of(nk);
    std::vector<int64_t> kinfo(3 * (size_t)nk + 1);  // [tile0 (nk + 1) | pair0 (nk) | count (nk)]
    P->xchunks.clear();
    int64_t pos = 0, ntl = 0, maxchunk = 0;
    XChunk cur;
    for (int id = 0; id < nk; ++id) {
        if (pos > cur.p0 && pos - cur.p0 + key_cnt[id] > budget) {
            cur.p1 = pos;
            cur.t1 = ntl;
            maxchunk = std::max(maxchunk, cur.p1 - cur.p0);
            P->xchunks.push_back(cur);
            cur = XChunk();
            cur.p0 = pos;
            cur.t0 = ntl;
        }
        chunk_of[id] = (int32_t)P->xchunks.size();
        kinfo[id] = ntl;
        kinfo[nk + 1 + id] = pos;
        kinfo[2 * (size_t)nk + 1 + id] = key_cnt[id];
        ntl += (key_cnt[id] + TW - 1) / TW;
        pos += key_cnt[id];
    }
    kinfo[nk] = ntl;
    cur.p1 = pos;
    cur.t1 = ntl;
    maxchunk = std::max(maxchunk, cur.p1 - cur.p0);
    P->xchunks.push_back(cur);
    const int64_t nb = pos;
    const int nchunk = (int)P->xchunks.size();
    FMM_CHECK(nchunk < (1 << 11), FMM_ERR_UNSUPPORTED, "m2l: too many cross-level chunks");
    P->nxk = nk;
    P->nxb = nb;
    P->nxt = ntl;

    P->xt_op = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->nxt));
    P->xt_first = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * P->nxt));
    P->xt_cnt = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->nxt));
    int64_t *d_kinfo = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * kinfo.size()));
    FMM_HIP(hipMemcpyAsync(d_kinfo, kinfo.data(), sizeof(int64_t) * kinfo.size(), hipMemcpyHostToDevice, s));
    k_x_tiles<<<(unsigned)nk, 256, 0, s>>>(d_kinfo, d_kinfo + nk + 1, d_kinfo + 2 * (size_t)nk + 1, TW, P->xt_op,
                                           P->xt_first, P->xt_cnt);
    FMM_HIP(hipGetLastError());
    double4 *d_tr = static_cast<double4 *>(al.alloc(sizeof(double4) * nk));
    FMM_HIP(hipMemcpyAsync(d_tr, tr.data(), sizeof(double4) * nk, hipMemcpyHostToDevice, s));
    const int RTx = P->P2pad / 16;
    const int Qx = m2l_q(P->p);
    const size_t xn = (size_t)nk * m2l_opsz(RTx, Qx, (int)esz) + m2l_tail(RTx, Qx, (int)esz);
    P->xops = plan_alloc(P, esz * xn);
    FMM_HIP(hipMemsetAsync(P->xops, 0, esz * xn, s));
    make_m2l_ops(P, d_tr, nk, P->xops, s);
    int32_t *d_id_of = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * xc.ncode));
    int32_t *d_chunk_of = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nk));
    FMM_HIP(hipMemcpyAsync(d_id_of, id_of.data(), sizeof(int32_t) * xc.ncode, hipMemcpyHostToDevice, s));
    FMM_HIP(hipMemcpyAsync(d_chunk_of, chunk_of.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));

    // batched pairs in (key, target) order; the others, still in target order, at the end
    uint64_t *k1 = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * nx));
    int32_t *v1 = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nx));
    int32_t *gcnt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * (nc + 1)));
    FMM_HIP(hipMemsetAsync(gcnt, 0, sizeof(int32_t) * (nc + 1), s));
    k_x_key1<<<grid1(nx, 256), 256, 0, s>>>(tgt, P->m2lx_src, code, d_id_of, nk, nx, k1, v1, gcnt);
    FMM_HIP(hipGetLastError());
    // the pairs arrive in target order, so a stable sort on the key bits alone
    // gives (key, target) order
    radix_sort_u64(k1, v1, nx, 32 + bits_of(nk), al, s, 32);
    P->xp_src = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nb));
    FMM_HIP(hipMemcpyAsync(P->xp_src, v1, sizeof(int32_t) * nb, hipMemcpyDeviceToDevice, s));
    P->n_gx = nx - nb;
    P->gx_off = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * (nc + 1)));
    scan_exclusive_i32to64(gcnt, P->gx_off, nc + 1, nullptr, al, s);
    P->gx_src = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, P->n_gx)));
    if (P->n_gx > 0)
        FMM_HIP(hipMemcpyAsync(P->gx_src, v1 + nb, sizeof(int32_t) * P->n_gx, hipMemcpyDeviceToDevice, s));

    // reduction order: (chunk, target, key)
    uint64_t *k2 = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * nb));
    int32_t *v2 = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nb));
    const int csh = 21 + bits_of(nc);
    FMM_CHECK(csh + bits_of(nchunk) <= 64, FMM_ERR_UNSUPPORTED, "m2l: cross-level key too wide");
    k_x_key2<<<grid1(nb, 256), 256, 0, s>>>(k1, nb, d_chunk_of, csh, k2, v2);
    FMM_HIP(hipGetLastError());
    // the input is in (key, target) order, so sorting the chunk and target
    // bits stably leaves the keys of a target in order
    radix_sort_u64(k2, v2, nb, csh + bits_of(nchunk), al, s, 21);
    P->xr_inv = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nb));
    k_x_invert<<<grid1(nb, 256), 256, 0, s>>>(v2, nb, P->xr_inv);
    FMM_HIP(hipGetLastError());
    int32_t *flag = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nb));
    int64_t *sidx = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * nb));
    int64_t *d_nseg = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
    k_x_segflag<<<grid1(nb, 256), 256, 0, s>>>(k2, nb, flag);
    FMM_HIP(hipGetLastError());
    scan_exclusive_i32to64(flag, sidx, nb, d_nseg, al, s);
    int64_t nseg = 0;
    FMM_HIP(hipMemcpyAsync(&nseg, d_nseg, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    P->xs_off = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * (nseg + 1)));
    P->xs_tgt = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * std::max<int64_t>(1, nseg)));
    int64_t *d_cs = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * (nchunk + 1)));
    k_x_segments<<<grid1(nb, 256), 256, 0, s>>>(k2, flag, sidx, nb, csh, P->xs_off, P->xs_tgt, d_cs);
    FMM_HIP(hipGetLastError());
    FMM_HIP(hipMemcpyAsync(P->xs_off + nseg, &nb, sizeof(int64_t), hipMemcpyHostToDevice, s));
    std::vector<int64_t> cs(nchunk + 1);
    FMM_HIP(hipMemcpyAsync(cs.data(), d_cs, sizeof(int64_t) * nchunk, hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    cs[nchunk] = nseg;
    for (int c = 0; c < nchunk; ++c) {
        P->xchunks[c].s0 = cs[c];
        P->xchunks[c].s1 = cs[c + 1];
    }
    P->xbuf = plan_alloc(P, esz * (size_t)maxchunk * P->P2pad);

    al.free(d_cs);
    al.free(d_kinfo);
    al.free(d_nseg);
    al.free(sidx);
    al.free(flag);
    al.free(v2);
    al.free(k2);
    al.free(gcnt);
    al.free(v1);
    al.free(k1);
    al.free(d_chunk_of);
    al.free(d_id_of);
    al.free(d_tr);
    al.free(cnt);
    al.free(code);
    al.free(tgt);
}

// Chunks of at most kGChunk generic pairs of one target, and their buffer.
void x_generic_prepare(fmm_plan *P, hipStream_t s)
{
    const int64_t nc = P->ncell;
    P->n_gchunk = 0;
    if (P->n_gx == 0) return;
    Allocator &al = P->al;
    int32_t *cnt = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * (nc + 1)));
    int64_t *d_tot = static_cast<int64_t *>(al.alloc(sizeof(int64_t)));
    k_gx_count<<<grid1(nc + 1, 256), 256, 0, s>>>(P->gx_off, nc, cnt);
    FMM_HIP(hipGetLastError());
    P->gx_cofs = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * (nc + 1)));
    scan_exclusive_i32to64(cnt, P->gx_cofs, nc + 1, d_tot, al, s);
    int64_t nch = 0;
    FMM_HIP(hipMemcpyAsync(&nch, d_tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    P->n_gchunk = nch;
    P->gx_ctgt = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * nch));
    P->gx_ck0 = static_cast<int64_t *>(plan_alloc(P, sizeof(int64_t) * nch));
    k_gx_fill<<<grid1(nc, 256), 256, 0, s>>>(P->gx_off, P->gx_cofs, nc, P->gx_ctgt, P->gx_ck0);
    FMM_HIP(hipGetLastError());
    P->gx_part = static_cast<double *>(plan_alloc(P, sizeof(double) * nch * P->P2pad));
    FMM_HIP(hipStreamSynchronize(s));
    al.free(d_tot);
    al.free(cnt);
}

}  // namespace


void m2l_cross_prepare(fmm_plan *P, hipStream_t s)
{
    P->n_gx = P->n_m2lx;
    P->gx_off = P->m2lx_off;
    P->gx_src = P->m2lx_src;
    if (P->n_m2lx == 0) return;
    if (P->m2l_rotation) {  // every pair of the list runs the rotation kernel
        rotation_prepare(P, s);
        return;
    }
    x_batch_prepare(P, s);
    x_generic_prepare(P, s);
}

void m2l_cross(fmm_plan *P, hipStream_t s)
{
    const bool f64 = P->precision == FMM_PREC_FP64;
    if (P->m2l_rotation) {
        rotation_m2l(P, s);
        return;
    }
    for (const XChunk &ch : P->xchunks) {
        if (f64) dispatch_pairs<double>(P, ch, s);
        else dispatch_pairs<float>(P, ch, s);
    }
    if (P->n_gchunk > 0) {
        FMM_CHECK(P->n_gchunk * 64 < (1ll << 32), FMM_ERR_UNSUPPORTED, "m2l: too many cross-level chunks");
        const unsigned nb = (unsigned)P->n_gchunk;
        const dim3 gr = grid1(P->ncell * P->P2, 256);
        if (f64) {
            k_m2l_cross<double><<<nb, 64, 0, s>>>(P->gx_ctgt, P->gx_ck0, P->gx_off, P->gx_src, P->c_lvl, P->c_ctr,
                                                   P->S, P->p, P->P2pad, static_cast<const double *>(P->Mc),
                                                   P->gx_part);
            k_gx_reduce<double><<<gr, 256, 0, s>>>(P->ncell, P->gx_cofs, P->gx_part, P->P2, P->P2pad,
                                                    static_cast<double *>(P->Lc));
        } else {
            k_m2l_cross<float><<<nb, 64, 0, s>>>(P->gx_ctgt, P->gx_ck0, P->gx_off, P->gx_src, P->c_lvl, P->c_ctr,
                                                  P->S, P->p, P->P2pad, static_cast<const float *>(P->Mc),
                                                  P->gx_part);
            k_gx_reduce<float><<<gr, 256, 0, s>>>(P->ncell, P->gx_cofs, P->gx_part, P->P2, P->P2pad,
                                                   static_cast<float *>(P->Lc));
        }
        FMM_HIP(hipGetLastError());
    }
}

void mfma_probe(int f64, void *out_host)
{
    void *d = nullptr;
    FMM_HIP(hipMalloc(&d, 64 * 4 * sizeof(double)));
    if (f64 == 1) k_mfma_probe_f64<<<1, 64>>>(static_cast<double *>(d));
    else if (f64 == 2) k_mfma_probe_f32_4x4<<<1, 64>>>(static_cast<float *>(d));
    else k_mfma_probe_f32<<<1, 64>>>(static_cast<float *>(d));
    FMM_HIP(hipGetLastError());
    FMM_HIP(hipMemcpy(out_host, d, 64 * 4 * (f64 == 1 ? sizeof(double) : sizeof(float)), hipMemcpyDeviceToHost));
    FMM_HIP(hipFree(d));
}

}  // namespace fmm
