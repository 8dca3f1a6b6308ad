// m2l.hip -- multipole-to-local translations on gfx950 (Section II.A; the
// paper notes that M2L and P2P take more than 90% of the run time).
//
// Same-level pairs.  With level-scaled coefficients the M2L operator between
// two cells of one level depends only on their integer offset t, so the
// translation L(A) += T(t) M(A - t) is a dense p^2 x p^2 product.  A block
// owns a tile of 64 targets of one level and one octant class (so they share
// one stencil of offsets); for every stencil entry k it multiplies the common
// operator T(t_k) by the 64 gathered source multipoles with MFMA
// (v_mfma_{f32,f64}_16x16x4), accumulating in registers; each target's sum is
// written once, without atomics, in a fixed order.
//
// Cross-level pairs (a leaf against a finer cell) use a generic kernel that
// builds the operator of the actual offset on the fly.
#include "internal.hpp"

#include <cmath>

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

template <class T> struct Vec16;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <> struct Vec16<float> {
    typedef f4v t;
    static constexpr int n = 4;
};
template <> struct Vec16<double> {
    typedef d2v t;
    static constexpr int n = 2;
};

// Column groups of 16 targets per wave: more groups reuse each operator
// fragment more often but need more accumulator registers.
__host__ __device__ constexpr int m2l_cg(int RT, bool f64) { return f64 ? 1 : (RT <= 4 ? 2 : 1); }

// Input steps of the operator per LDS stage: the largest divisor of Q = 4 RT
// whose stage (4 groups x steps x P2pad values) fits in 32 KiB.
__host__ __device__ constexpr int m2l_sch(int RT, int bytes)
{
    int best = 1;
    for (int sc = 1; sc <= 4 * RT; ++sc)
        if ((4 * RT) % sc == 0 && 4 * sc * 16 * RT * bytes <= 32768) best = sc;
    return best;
}

// Batched same-level M2L.  Block = 4 waves = one tile of TW = 64 CG targets of
// one octant class, restricted to chunk ks = block mod KS of the tile's list
// of stencil entries that have at least one source (chunks, not tiles, vary
// fastest across blocks, so blocks resident on one XCD share operators in its
// L2).  For every listed entry k the block stages the common operator T(t_k)
// in LDS; each wave multiplies it by its 16 CG gathered source multipoles:
//     D[i][j] = sum_k A[i][k] B[k][j] (16x16x4 MFMA), A = operator fragment
//     (lane l: A[l%16][l/16]), B = multipoles (lane l: B[l/16][l%16]); lane l
//     accumulates D[acc_row(l/16, e)][l%16] in slot e.
// The loop body has no divergent branch and never edits loaded data: the
// next operator stage and the next entry's sources (slot indices two entries
// ahead) are fetched while the current stage is multiplied; a missing source
// reads the all-zero multipole row zero_row (= ncell).
template <class T, int RT, int CG, int SCH>
__global__ __launch_bounds__(256) void k_m2l_batched(const int32_t *__restrict__ tile_cls,
                                                     const int32_t *__restrict__ slots,
                                                     const int32_t *__restrict__ tile_kl,
                                                     const int32_t *__restrict__ tile_nk,
                                                     const int32_t *__restrict__ st_op, int K, int KS,
                                                     const int32_t *__restrict__ slot_none, int zero_row,
                                                     const T *__restrict__ Tf, const T *__restrict__ M,
                                                     T *__restrict__ part, const int32_t *__restrict__ tile_tgt,
                                                     T *__restrict__ L, int64_t ntile)
{
    constexpr int P2pad = 16 * RT, Q = 4 * RT, NC = Q / SCH, TW = 64 * CG;
    constexpr int STAGE = 4 * SCH * P2pad;
    constexpr int VN = Vec16<T>::n;
    constexpr int NV = STAGE / VN;
    constexpr int PV = (NV + 255) / 256;
    typedef typename Vec16<T>::t vec_t;
    typedef typename Mfma<T>::acc_t acc_t;
    __shared__ __align__(16) T lds[STAGE];

    const int64_t b = blockIdx.x;
    const int ks = (int)(b % KS);
    const int64_t tile = b / KS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 15, g = lane >> 4;
    const int cls = tile_cls[tile];
    const int nk = tile_nk[tile];
    const int Kc = (nk + KS - 1) / KS;
    const int i0 = ks * Kc, i1 = min(nk, i0 + Kc);
    const int32_t *kl = tile_kl + tile * (int64_t)K;
    const int32_t *sl = slots + tile * (int64_t)K * TW + wave * CG * 16 + j;
    const int32_t *sl_none = slot_none + wave * CG * 16 + j;  // a row of -1
    const int32_t *opk = st_op + (int64_t)cls * K;

    acc_t acc[CG][RT];
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[cg][r] = acc_t{0, 0, 0, 0};

    if (i0 < i1) {
        vec_t treg[PV];
        // operator stage (entry KK, chunk CC): rows s in [CC SCH, (CC+1) SCH) of the 4 groups
#define M2L_LOAD_STAGE(KK, CC)                                                                     \
    {                                                                                              \
        int op_ = opk[KK];                                                                         \
        op_ = op_ < 0 ? 0 : op_;                                                                   \
        _Pragma("unroll") for (int u = 0; u < PV; ++u)                                             \
        {                                                                                          \
            const int v = min(tid + 256 * u, NV - 1);                                              \
            const int e = v * VN, gg = e / (SCH * P2pad), rem = e - gg * (SCH * P2pad);            \
            treg[u] = *reinterpret_cast<const vec_t *>(Tf + ((int64_t)(op_ * 4 + gg) * Q + (CC) * SCH) * P2pad + rem); \
        }                                                                                          \
    }
#define M2L_STORE_STAGE()                                                                          \
    {                                                                                              \
        _Pragma("unroll") for (int u = 0; u < PV; ++u)                                             \
        {                                                                                          \
            const int v = tid + 256 * u;                                                           \
            if (NV % 256 == 0 || v < NV) *reinterpret_cast<vec_t *>(lds + v * VN) = treg[u];        \
        }                                                                                          \
    }
#define M2L_SLOTS(II, DST)                                                                         \
    {                                                                                              \
        const int32_t *sp_ = (II) < i1 ? sl + (int64_t)kl[II] * TW : sl_none;                      \
        _Pragma("unroll") for (int cg = 0; cg < CG; ++cg) DST[cg] = sp_[cg * 16];                  \
    }
#define M2L_LOAD_B(SRC, DST)                                                                       \
    {                                                                                              \
        _Pragma("unroll") for (int cg = 0; cg < CG; ++cg)                                          \
        {                                                                                          \
            const int sv = SRC[cg];                                                                \
            const vec_t *mp = reinterpret_cast<const vec_t *>(M + (int64_t)(sv < 0 ? zero_row : sv) * P2pad + g * Q); \
            _Pragma("unroll") for (int v = 0; v < Q / VN; ++v)                                     \
            {                                                                                      \
                const vec_t x = mp[v];                                                             \
                _Pragma("unroll") for (int w = 0; w < VN; ++w) DST[cg][v * VN + w] = x[w];         \
            }                                                                                      \
        }                                                                                          \
    }
        T bA[CG][Q], bB[CG][Q];
        int sA[CG], sB[CG];
        {
            int s0[CG];
            M2L_SLOTS(i0, s0);
            M2L_SLOTS(i0 + 1, sA);
            M2L_LOAD_STAGE(kl[i0], 0);
            M2L_LOAD_B(s0, bA);
            M2L_STORE_STAGE();
        }
        // One stencil entry: multiply with BCUR while the next entry's sources
        // (slot indices SREAD) go to BNEXT and the slot indices two entries
        // ahead go to SWRITE.  Two entries per trip with swapped roles, so no
        // loaded register is ever copied; an odd tail runs one entry whose
        // sources are all missing (it adds exact zeros).
#define M2L_ENTRY(IT, BCUR, BNEXT, SREAD, SWRITE)                                                  \
    {                                                                                              \
        const int k_ = kl[min(IT, i1 - 1)];                                                        \
        const int kn_ = kl[min((IT) + 1, i1 - 1)];                                                 \
        _Pragma("unroll") for (int c = 0; c < NC; ++c)                                             \
        {                                                                                          \
            if (c + 1 < NC) M2L_LOAD_STAGE(k_, c + 1)                                              \
            else M2L_LOAD_STAGE(kn_, 0)                                                            \
            if (c == 0) {                                                                          \
                M2L_SLOTS((IT) + 2, SWRITE);                                                       \
                M2L_LOAD_B(SREAD, BNEXT);                                                          \
            }                                                                                      \
            __syncthreads();                                                                       \
            _Pragma("unroll") for (int ss = 0; ss < SCH; ++ss)                                     \
            {                                                                                      \
                T a[RT];                                                                           \
                const T *ap = lds + g * (SCH * P2pad) + ss * P2pad + j * RT;                       \
                _Pragma("unroll") for (int r = 0; r < RT; ++r) a[r] = ap[r];                       \
                _Pragma("unroll") for (int cg = 0; cg < CG; ++cg)                                  \
                    _Pragma("unroll") for (int r = 0; r < RT; ++r)                                 \
                        acc[cg][r] = Mfma<T>::run(a[r], BCUR[cg][c * SCH + ss], acc[cg][r]);       \
            }                                                                                      \
            __syncthreads();                                                                       \
            M2L_STORE_STAGE();                                                                     \
        }                                                                                          \
    }
        for (int it = i0; it < i1; it += 2) {
            M2L_ENTRY(it, bA, bB, sA, sB);
            M2L_ENTRY(it + 1, bB, bA, sB, sA);
        }
#undef M2L_ENTRY
#undef M2L_LOAD_STAGE
#undef M2L_STORE_STAGE
#undef M2L_SLOTS
#undef M2L_LOAD_B
    }
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
        const int col = wave * CG * 16 + cg * 16 + j;
        T *dst;
        if (KS == 1) {
            const int tgt = tile_tgt[tile * TW + col];
            if (tgt < 0) continue;
            dst = L + (int64_t)tgt * P2pad;
        } else {
            dst = part + (((int64_t)ks * ntile + tile) * TW + col) * P2pad;
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[16 * r + Mfma<T>::acc_row(g, e)] = acc[cg][r][e];
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

// Sum of the KS partial products of each target, in chunk order.
template <class T>
__global__ __launch_bounds__(256) void k_m2l_reduce(const T *part, int KS, int64_t ncol, int P2pad,
                                                    const int32_t *tile_tgt, T *L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pos = t / P2pad;
    const int row = (int)(t % P2pad);
    if (pos >= ncol) return;
    const int tgt = tile_tgt[pos];
    if (tgt < 0) return;
    T s = 0;
    for (int k = 0; k < KS; ++k) s += part[((int64_t)k * ncol + pos) * P2pad + row];
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

// Cross-level pairs, one 64-thread block (one wave) per target cell, float64
// arithmetic in the complex form.  For a source of level l_B and a target of
// level l_A, with tau = (c_A - c_B)/h_A and rho = h_B/h_A:
//     Lt_j^s += (-1)^j sum_{n<p} rho^n sum_{m=-n..n} Mt_n^m I_{n+j}^{m+s}(tau),
// M^{-m} = (-1)^m conj(M^m), I^{-l} = (-1)^l conj(I^l).  Lane t owns the
// outputs (j, s >= 0) numbered t and t + 64 and sums over the target's pairs
// in list order; the block's barriers are reached by the whole block.
template <class TM>
__global__ __launch_bounds__(64) void k_m2l_cross(int64_t ncell, const int64_t *off, const int32_t *src,
                                                  const int32_t *lvl, const double *ctr, double S, int p, int P2pad,
                                                  const TM *M, TM *L)
{
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    if (c >= ncell) return;
    const int64_t k0 = off[c], k1 = off[c + 1];
    if (k0 == k1) return;
    __shared__ cd H[(2 * kMaxP) * (2 * kMaxP + 1) / 2];
    __shared__ cd Ms[kMaxP * (kMaxP + 1) / 2];
    const int nI = 2 * p - 1, P2 = p * p, NO = p * (p + 1) / 2;
    const double hA = ldexp(S, -lvl[c]);
    // output (j, s) of each of this lane's two slots
    int oj[2], os[2];
    for (int q = 0; q < 2; ++q) {
        const int t = lane + 64 * q;
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= t) ++j;
        oj[q] = t < NO ? j : -1;
        os[q] = t - j * (j + 1) / 2;
    }
    double are[2] = {0, 0}, aim[2] = {0, 0};
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
        for (int q = 0; q < 2; ++q) {
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
    TM *dl = L + c * P2pad;
    for (int q = 0; q < 2; ++q) {
        const int j = oj[q], sO = os[q];
        if (j < 0) continue;
        const double sg = (j & 1) ? -1.0 : 1.0;
        if (sO == 0) dl[j * j] = (TM)((double)dl[j * j] + sg * are[q]);
        else {
            const int r = j * j + 2 * sO - 1;
            dl[r] = (TM)((double)dl[r] + sg * are[q]);
            dl[r + 1] = (TM)((double)dl[r + 1] + sg * aim[q]);
        }
    }
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
__global__ void k_mfma_probe_f64(double *out)
{
    const int l = threadIdx.x;
    v4d acc = {0, 0, 0, 0};
    const double a = (double)((l & 15) + 1 + 100 * (l >> 4));
    const double b = (l >> 4) == 0 ? 1.0 + (double)(l & 15) * 1000.0 : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int e = 0; e < 4; ++e) out[l * 4 + e] = acc[e];
}

template <class T, int RT>
void launch_batched(fmm_plan *P, hipStream_t s)
{
    constexpr int CG = m2l_cg(RT, sizeof(T) == 8);
    constexpr int SCH = m2l_sch(RT, (int)sizeof(T));
    const int64_t nb = P->ntile * P->KS;
    FMM_CHECK(nb < (1ll << 31), FMM_ERR_UNSUPPORTED, "m2l: too many tiles");
    FMM_CHECK(P->TW == 64 * CG, FMM_ERR_DEVICE, "m2l: tile width mismatch");
    k_m2l_batched<T, RT, CG, SCH><<<(unsigned)nb, 256, 0, s>>>(
        P->tile_cls, P->slots, P->tile_kl, P->tile_nk, P->st_op, P->K, P->KS, P->slot_none, (int)P->ncell,
        static_cast<const T *>(P->ops),
        static_cast<const T *>(P->Mc), static_cast<T *>(P->m2l_part), P->tile_tgt, static_cast<T *>(P->Lc), P->ntile);
    FMM_HIP(hipGetLastError());
    if (P->KS > 1) {
        const int64_t ncol = P->ntile * P->TW;
        k_m2l_reduce<T><<<grid1(ncol * P->P2pad, 256), 256, 0, s>>>(static_cast<const T *>(P->m2l_part), P->KS, ncol,
                                                                   P->P2pad, P->tile_tgt, static_cast<T *>(P->Lc));
        FMM_HIP(hipGetLastError());
    }
}

template <class T>
void dispatch_tiles(fmm_plan *P, hipStream_t s)
{
    switch (P->P2pad / 16) {
    case 1: launch_batched<T, 1>(P, s); break;
    case 2: launch_batched<T, 2>(P, s); break;
    case 3: launch_batched<T, 3>(P, s); break;
    case 4: launch_batched<T, 4>(P, s); break;
    case 6: launch_batched<T, 6>(P, s); break;
    case 7: launch_batched<T, 7>(P, s); break;
    case 8: launch_batched<T, 8>(P, s); break;
    case 9: launch_batched<T, 9>(P, s); break;
    case 11: launch_batched<T, 11>(P, s); break;
    case 13: launch_batched<T, 13>(P, s); break;
    case 15: launch_batched<T, 15>(P, s); break;
    case 16: launch_batched<T, 16>(P, s); break;
    default: throw Error(FMM_ERR_UNSUPPORTED, "m2l: unsupported padded coefficient count");
    }
}

}  // namespace

int m2l_tile_width(int p, bool f64) { return 64 * m2l_cg(p2pad_of(p) / 16, f64); }

// Stencil split: enough blocks to fill the chip (about 8 per compute unit),
// but at least 8 stencil entries per chunk.
void m2l_prepare(fmm_plan *P, hipStream_t s)
{
    P->KS = 1;
    if (P->ntile <= 0 || P->K <= 0) return;
    P->tile_kl = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->ntile * P->K));
    P->slot_none = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->TW));
    k_fill_none<<<1, 256, 0, s>>>(P->slot_none, P->TW);
    P->tile_nk = static_cast<int32_t *>(plan_alloc(P, sizeof(int32_t) * P->ntile));
    k_tile_klist<<<(unsigned)P->ntile, 256, 0, s>>>(P->tile_kflag, P->K, P->tile_kl, P->tile_nk);
    FMM_HIP(hipGetLastError());
    // a power of two (a divisor or multiple of the 8 XCDs), at least 8 entries per chunk
    int64_t ks = 1;
    while (ks < 16 && P->ntile * ks < 2048 && P->K / (2 * ks) >= 8) ks *= 2;
    P->KS = (int)ks;
    if (P->KS > 1) {
        const size_t esz = P->precision == FMM_PREC_FP64 ? sizeof(double) : sizeof(float);
        P->m2l_part = plan_alloc(P, esz * (size_t)P->KS * P->ntile * P->TW * P->P2pad);
    }
}

void m2l_same(fmm_plan *P, hipStream_t s)
{
    const bool f64 = P->precision == FMM_PREC_FP64;
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    // root (and any cell outside the tiles) starts from zero
    FMM_HIP(hipMemsetAsync(P->Lc, 0, esz * P->P2pad, s));
    if (P->ntile > 0 && P->K > 0) {
        if (f64) dispatch_tiles<double>(P, s);
        else dispatch_tiles<float>(P, s);
    } else {
        FMM_HIP(hipMemsetAsync(P->Lc, 0, esz * P->P2pad * P->ncell, s));
    }
}

void m2l_cross(fmm_plan *P, hipStream_t s)
{
    const bool f64 = P->precision == FMM_PREC_FP64;
    if (P->n_m2l_cross > 0) {
        const unsigned nb = (unsigned)P->ncell;
        if (f64)
            k_m2l_cross<double><<<nb, 64, 0, s>>>(P->ncell, P->m2lx_off, P->m2lx_src, P->c_lvl, P->c_ctr, P->S, P->p,
                                                   P->P2pad, static_cast<const double *>(P->Mc),
                                                   static_cast<double *>(P->Lc));
        else
            k_m2l_cross<float><<<nb, 64, 0, s>>>(P->ncell, P->m2lx_off, P->m2lx_src, P->c_lvl, P->c_ctr, P->S, P->p,
                                                  P->P2pad, static_cast<const float *>(P->Mc),
                                                  static_cast<float *>(P->Lc));
        FMM_HIP(hipGetLastError());
    }
}

void mfma_probe(int f64, void *out_host)
{
    void *d = nullptr;
    FMM_HIP(hipMalloc(&d, 64 * 4 * sizeof(double)));
    if (f64) k_mfma_probe_f64<<<1, 64>>>(static_cast<double *>(d));
    else k_mfma_probe_f32<<<1, 64>>>(static_cast<float *>(d));
    FMM_HIP(hipGetLastError());
    FMM_HIP(hipMemcpy(out_host, d, 64 * 4 * (f64 ? sizeof(double) : sizeof(float)), hipMemcpyDeviceToHost));
    FMM_HIP(hipFree(d));
}

}  // namespace fmm
