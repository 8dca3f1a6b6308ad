// let.hip -- virtual ranks on one GPU (Section II.B: orthogonal recursive
// bisection weighted by the work of Eq. (1); Section II.C: local trees from
// local bounding boxes, the local essential tree (LET) each rank sends, and
// the receiver's traversal against the grafted remote root, Fig. `tree').
//
// Every rank is a plan of its own (its tree built from its own bounding
// box, Morton keys of its own cube), evaluated by the same kernels as a
// single-rank evaluation.  Between ranks:
//   * the sender s selects, for receiver r, the cells of its tree that r's
//     traversal can reach: top-down, a cell that meets the acceptance
//     criterion against r's whole root cube (R_B < theta d, d the distance
//     from the cell's center to the cube) is sent with its multipole only; a
//     leaf that does not is sent with its bodies; any other cell is sent and
//     opened;
//   * the receiver walks its tree against that grafted tree: accepted pairs
//     (R_A + R_B < theta |c_A - c_B|, decided in float64 with a fixed
//     operation order, the same as the oracle's) are M2L; a leaf against a
//     sent leaf is P2P (bodies sent) or M2P (multipole only, evaluated at the
//     leaf's bodies, all inside r's cube where the series converges); else a
//     sent leaf splits A, a leaf A splits B, and otherwise the larger cube
//     is split (both when equal).
// Remote M2L adds into the receiver's local expansions before its downward
// pass; remote P2P and M2P add to its bodies' sums afterwards.  The remote
// work runs in float64.
#include "internal.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>

namespace fmm {

namespace {

constexpr int kLetMaxP = kMaxP;

// double -> 64-bit key that orders like the value (-0 taken as +0)
__device__ __forceinline__ uint64_t order_bits(double v)
{
    if (v == 0.0) v = 0.0;
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

// ---------------------------------------------------------------- partition
// Per-block min/max of the segment's coordinates, then one block reduces.
__global__ __launch_bounds__(256) void k_seg_box(const double *x, const int32_t *idx, int64_t cnt, double *part)
{
    __shared__ double sm[6][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[j];
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], x[3 * i + d]);
            hi[d] = fmax(hi[d], x[3 * i + d]);
        }
    }
    for (int d = 0; d < 3; ++d) {
        sm[d][threadIdx.x] = lo[d];
        sm[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int d = 0; d < 3; ++d) {
                sm[d][threadIdx.x] = fmin(sm[d][threadIdx.x], sm[d][threadIdx.x + w]);
                sm[3 + d][threadIdx.x] = fmax(sm[3 + d][threadIdx.x], sm[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void k_box_final(const double *part, int nb, double *out)
{
    if (threadIdx.x >= 6) return;
    const int d = threadIdx.x;
    double v = part[d];
    for (int b = 1; b < nb; ++b) v = d < 3 ? fmin(v, part[b * 6 + d]) : fmax(v, part[b * 6 + d]);
    out[d] = v;
}

__global__ __launch_bounds__(256) void k_orb_keys(const double *x, const int32_t *idx, int64_t cnt, int axis,
                                                  uint64_t *key, int32_t *val)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    const int32_t i = idx[j];
    key[j] = order_bits(x[3 * (int64_t)i + axis]);
    val[j] = i;
}

__global__ __launch_bounds__(256) void k_orb_weights(const int64_t *w, const int32_t *val, int64_t cnt, int64_t *wt)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cnt) wt[j] = w ? w[val[j]] : 1;
}

// The split: the smallest k with P(k) m >= W mL (P(k) the weight of the
// first k bodies in coordinate order; unit weights when the box weighs
// nothing), at least one body on each side when there are two or more.
__global__ void k_orb_find(const int64_t *pre, const int64_t *tot, int64_t cnt, int m, int mL, int64_t *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const __int128 W0 = *tot;
    const bool unit = W0 == 0;
    const __int128 W = unit ? (__int128)cnt : W0;
    const __int128 goal = W * mL;
    int64_t lo = 0, hi = cnt;  // P(hi) m >= goal always (P(cnt) = W, mL < m)
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const __int128 P = unit ? (__int128)mid : (mid < cnt ? (__int128)pre[mid] : W);
        if (P * m >= goal) hi = mid;
        else lo = mid + 1;
    }
    int64_t k = lo;
    if (cnt >= 2) k = k < 1 ? 1 : (k > cnt - 1 ? cnt - 1 : k);
    *out = k;
}

__global__ __launch_bounds__(256) void k_check_weights(const int64_t *w, int64_t n, int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (w[i] < 0 || w[i] >= (1ll << 40))) atomicOr(bad, 1);
}

__global__ __launch_bounds__(256) void k_idx_keys(const int32_t *val, int64_t cnt, uint64_t *key)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cnt) key[j] = (uint64_t)(uint32_t)val[j];
}

__global__ __launch_bounds__(256) void k_keys_to_idx(const uint64_t *key, int64_t cnt, int32_t *idx)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cnt) idx[j] = (int32_t)key[j];
}

__global__ __launch_bounds__(256) void k_set_rank(const int32_t *idx, int64_t cnt, int32_t r, int32_t *rank)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cnt) rank[idx[j]] = r;
}

// coordinates (widened) and charges of a rank's members, in member order
template <class T>
__global__ __launch_bounds__(256) void k_gather_rank(const T *x, const T *q, const int32_t *mem, int64_t cnt, double *xr,
                                                     double *qr)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    const int64_t i = mem[j];
    xr[3 * j] = (double)x[3 * i];
    xr[3 * j + 1] = (double)x[3 * i + 1];
    xr[3 * j + 2] = (double)x[3 * i + 2];
    if (q) qr[j] = (double)q[i];
}

// ---------------------------------------------------------------- the LET
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct TreeRef {
    const int32_t *lvl, *par, *nch, *cbeg, *beg, *end;
    const double *ctr;
    double S;
    int64_t ncell;
};

TreeRef tree_ref(const fmm_plan *P)
{
    return TreeRef{P->c_lvl, P->c_par, P->c_nch, P->c_cbeg, P->c_beg, P->c_end, P->c_ctr, P->S, P->ncell};
}

__device__ __forceinline__ double side(const TreeRef &T, int c) { return ldexp(T.S, -T.lvl[c]); }

// 3 h^2 < t4 d^2 with d the distance from the cell's center to the cube
// [lo, lo + S]^3 of the receiver (the oracle's operation order)
__device__ __forceinline__ bool let_far(const TreeRef &T, int c, double lx, double ly, double lz, double S, double t4)
{
#pragma clang fp contract(off)
    const double lo[3] = {lx, ly, lz};
    double d[3];
    for (int k = 0; k < 3; ++k) {
        const double v = T.ctr[3 * c + k], a = lo[k], b = lo[k] + S;
        d[k] = v < a ? a - v : (v > b ? v - b : 0.0);
    }
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double h = side(T, c);
    return 3.0 * h * h < t4 * d2;
}

// kind of each of the sender's cells for one receiver: 0 not sent, 1 sent and
// opened, 2 multipole only, 3 leaf with bodies; counts and the LET digest
__global__ __launch_bounds__(256) void k_let_kind(TreeRef T, double lx, double ly, double lz, double S, double t4,
                                                  uint8_t *kind, unsigned long long *acc)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= T.ncell) return;
    for (int a = T.par[c]; a >= 0; a = T.par[a])
        if (let_far(T, a, lx, ly, lz, S, t4)) {
            kind[c] = 0;
            return;
        }
    uint8_t k;
    if (let_far(T, (int)c, lx, ly, lz, S, t4)) k = 2;
    else if (T.nch[c] == 0) k = 3;
    else k = 1;
    kind[c] = k;
    atomicAdd(&acc[0], 1ull);
    if (k == 2) atomicAdd(&acc[1], 1ull);
    if (k == 3) {
        atomicAdd(&acc[2], 1ull);
        atomicAdd(&acc[3], (unsigned long long)(T.end[c] - T.beg[c]));
    }
    atomicAdd(&acc[4], (unsigned long long)mix64(((uint64_t)c << 8) | k));
}

// ----------------------------------------------------- remote traversal
// 0 = M2L, 1 = P2P, 2 = M2P, 3 = split (sa, sb set)
__device__ __forceinline__ int lx_classify(const TreeRef &A, int a, const TreeRef &B, int b, const uint8_t *kind,
                                           double t4, bool &sa, bool &sb)
{
#pragma clang fp contract(off)
    const double dx = A.ctr[3 * a] - B.ctr[3 * b], dy = A.ctr[3 * a + 1] - B.ctr[3 * b + 1],
                 dz = A.ctr[3 * a + 2] - B.ctr[3 * b + 2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double ha = side(A, a), hb = side(B, b), sh = ha + hb;
    if (3.0 * sh * sh < t4 * d2) return 0;
    const bool aleaf = A.nch[a] == 0;
    const int bk = kind[b];
    const bool bleaf = bk == 2 || bk == 3;
    if (aleaf && bleaf) return bk == 3 ? 1 : 2;
    if (bleaf) { sa = true; sb = false; }
    else if (aleaf) { sa = false; sb = true; }
    else { sa = ha >= hb; sb = hb >= ha; }
    return 3;
}

__global__ __launch_bounds__(256) void k_lx_count(TreeRef A, TreeRef B, const uint8_t *kind, double t4, const int2 *F,
                                                  int64_t nf, int32_t *cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int a = F[i].x, b = F[i].y;
    bool sa = false, sb = false;
    const int k = lx_classify(A, a, B, b, kind, t4, sa, sb);
    int c[4] = {0, 0, 0, 0};
    if (k < 3) c[k] = 1;
    else c[3] = (sa ? A.nch[a] : 1) * (sb ? B.nch[b] : 1);
    for (int t = 0; t < 4; ++t) cnt[t * nf + i] = c[t];
}

__global__ __launch_bounds__(256) void k_lx_write(TreeRef A, TreeRef B, const uint8_t *kind, double t4, const int2 *F,
                                                  int64_t nf, const int64_t *off, uint64_t *m2l, uint64_t *p2p,
                                                  uint64_t *m2p, int2 *next)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int a = F[i].x, b = F[i].y;
    bool sa = false, sb = false;
    const int k = lx_classify(A, a, B, b, kind, t4, sa, sb);
    const uint64_t pr = ((uint64_t)a << 32) | (uint32_t)b;
    if (k == 0) m2l[off[i] - off[0]] = pr;
    else if (k == 1) p2p[off[nf + i] - off[nf]] = pr;
    else if (k == 2) m2p[off[2 * nf + i] - off[2 * nf]] = pr;
    else {
        int64_t o = off[3 * nf + i] - off[3 * nf];
        const int na = sa ? A.nch[a] : 1, nb = sb ? B.nch[b] : 1;
        for (int u = 0; u < na; ++u)
            for (int v = 0; v < nb; ++v) next[o++] = make_int2(sa ? A.cbeg[a] + u : a, sb ? B.cbeg[b] + v : b);
    }
}

__global__ void k_lx_totals(const int64_t *off, int64_t nf, int64_t *tot)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t all = tot[4];
        for (int t = 0; t < 3; ++t) tot[t] = off[(t + 1) * nf] - off[t * nf];
        tot[3] = all - off[3 * nf];
    }
}

// CSR over the receiver's cells of pairs sorted by (target, source)
__global__ __launch_bounds__(256) void k_pair_offsets(const uint64_t *keys, int64_t np, int64_t nc, int64_t *off)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc) return;
    const uint64_t want = (uint64_t)c << 32;
    int64_t lo = 0, hi = np;
    while (lo < hi) {
        const int64_t m = lo + ((hi - lo) >> 1);
        if (keys[m] < want) lo = m + 1;
        else hi = m;
    }
    off[c] = lo;
}

__global__ __launch_bounds__(256) void k_pair_sources(const uint64_t *keys, int64_t np, int32_t *src,
                                                      unsigned long long *dig)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    src[k] = (int32_t)(keys[k] & 0xffffffffu);
    atomicAdd(dig, (unsigned long long)mix64(keys[k]));
}

// ----------------------------------------------------- remote operators
struct cdd {
    double re, im;
};

// Irregular solid harmonics I_n^m(t) (n < nI, 0 <= m <= n) into H[n(n+1)/2 + m]
// by the recurrences in m and n (lane m computes column m).
__device__ void irregular_cols(double tx, double ty, double tz, int nI, cdd *H)
{
    const int lane = threadIdx.x & 63;
    const double r2 = tx * tx + ty * ty + tz * tz, ir2 = 1.0 / r2;
    if (lane == 0) {
        cdd mm = {1.0 / sqrt(r2), 0.0};
        for (int m = 0; m < nI; ++m) {
            if (m > 0) {
                const double f = -(2.0 * m - 1.0) * ir2;
                mm = cdd{(mm.re * tx - mm.im * ty) * f, (mm.re * ty + mm.im * tx) * f};
            }
            H[m * (m + 1) / 2 + m] = mm;
        }
    }
    __syncthreads();
    if (lane < nI) {
        const int m = lane;
        cdd p1 = H[m * (m + 1) / 2 + m], p2 = {0, 0};
        for (int n = m + 1; n < nI; ++n) {
            cdd cur;
            if (n == m + 1) cur = cdd{p1.re * (2.0 * m + 1.0) * tz * ir2, p1.im * (2.0 * m + 1.0) * tz * ir2};
            else {
                const double a = (2.0 * n - 1.0) * tz, bb = -(double)((n + m - 1) * (n - m - 1));
                cur = cdd{(a * p1.re + bb * p2.re) * ir2, (a * p1.im + bb * p2.im) * ir2};
            }
            H[n * (n + 1) / 2 + m] = cur;
            p2 = p1;
            p1 = cur;
        }
    }
    __syncthreads();
}

constexpr int kOutSlots = (kMaxP * (kMaxP + 1) / 2 + 63) / 64;

// Remote M2L: one wave per work item, a run of at most kRChunk pairs of one
// target cell A of the receiver with sources of one sender; the sources'
// multipoles (scaled by h_B^-n) translated to A's local expansion (scaled by
// h_A^{n+1}) in float64,
//   L_j^s = (-1)^j sum_{n,m} rho^n M_n^m I_{n+j}^{m+s}(tau),
// tau = (c_A - c_B) / h_A, rho = h_B / h_A, into the item's row of part.
constexpr int kRChunk = 16;

template <class TM>
__global__ __launch_bounds__(64) void k_m2l_remote(TreeRef A, TreeRef B, const int32_t *it_tgt, const int64_t *it_k0,
                                                   const int64_t *it_k1, const int32_t *src, int p, int P2pad,
                                                   const TM *MB, double *part)
{
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int c = it_tgt[item];
    __shared__ cdd H[(2 * kLetMaxP) * (2 * kLetMaxP + 1) / 2];
    __shared__ cdd Ms[kLetMaxP * (kLetMaxP + 1) / 2];
    const int nI = 2 * p - 1, P2 = p * p, NO = p * (p + 1) / 2;
    const double hA = side(A, c);
    int oj[kOutSlots], os[kOutSlots];
    for (int q = 0; q < kOutSlots; ++q) {
        const int t = lane + 64 * q;
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= t) ++j;
        oj[q] = t < NO ? j : -1;
        os[q] = t - j * (j + 1) / 2;
    }
    double are[kOutSlots] = {}, aim[kOutSlots] = {};
    for (int64_t k = it_k0[item]; k < it_k1[item]; ++k) {
        const int b = src[k];
        const double tx = (A.ctr[3 * c] - B.ctr[3 * b]) / hA, ty = (A.ctr[3 * c + 1] - B.ctr[3 * b + 1]) / hA,
                     tz = (A.ctr[3 * c + 2] - B.ctr[3 * b + 2]) / hA;
        const double rho = side(B, b) / hA;
        irregular_cols(tx, ty, tz, nI, H);
        const TM *mb = MB + (int64_t)b * P2pad;
        for (int r = lane; r < P2; r += 64) {
            const int n = (int)sqrtf((float)r + 0.5f);
            const int o = r - n * n;
            double sc = 1.0;
            for (int e = 0; e < n; ++e) sc *= rho;
            if (o == 0) Ms[n * (n + 1) / 2] = cdd{sc * (double)mb[r], 0.0};
            else if (o & 1) {
                const int m = (o + 1) / 2;
                Ms[n * (n + 1) / 2 + m] = cdd{sc * (double)mb[r], sc * (double)mb[r + 1]};
            }
        }
        __syncthreads();
        for (int q = 0; q < kOutSlots; ++q) {
            const int j = oj[q], sO = os[q];
            if (j < 0) continue;
            double sr = 0.0, si = 0.0;
            for (int n = 0; n < p; ++n) {
                const int kk = n + j;
                const cdd *Hk = H + kk * (kk + 1) / 2;
                const cdd *Mn = Ms + n * (n + 1) / 2;
                for (int m = -n; m <= n; ++m) {
                    cdd mv = Mn[m < 0 ? -m : m];
                    if (m < 0) mv = (m & 1) ? cdd{-mv.re, mv.im} : cdd{mv.re, -mv.im};
                    const int l = m + sO;
                    cdd iv = Hk[l < 0 ? -l : l];
                    if (l < 0) iv = (l & 1) ? cdd{-iv.re, iv.im} : cdd{iv.re, -iv.im};
                    sr += mv.re * iv.re - mv.im * iv.im;
                    si += mv.re * iv.im + mv.im * iv.re;
                }
            }
            are[q] += sr;
            aim[q] += si;
        }
        __syncthreads();
    }
    double *dst = part + item * P2pad;
    for (int q = 0; q < kOutSlots; ++q) {
        const int j = oj[q], sO = os[q];
        if (j < 0) continue;
        const double sg = (j & 1) ? -1.0 : 1.0;
        if (sO == 0) dst[j * j] = sg * are[q];
        else {
            const int r = j * j + 2 * sO - 1;
            dst[r] = sg * are[q];
            dst[r + 1] = sg * aim[q];
        }
    }
}

// L[c] += the sum of the cell's item rows, in item order (one thread per
// (target, coefficient)).
template <class TM>
__global__ __launch_bounds__(256) void k_m2l_remote_reduce(const int32_t *tg, const int64_t *tg_i, int64_t ntg,
                                                           const double *part, int P2, int P2pad, TM *LA)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = t / P2;
    const int r = (int)(t % P2);
    if (k >= ntg) return;
    const double acc = strided_sum(part + tg_i[k] * P2pad + r, tg_i[k + 1] - tg_i[k], (int64_t)P2pad);
    TM *dst = LA + (int64_t)tg[k] * P2pad + r;
    *dst = (TM)((double)*dst + acc);
}

// Remote P2P and M2P: one wave per work item, a run of list entries of one
// target leaf A; G lanes share a body of A (G a power of two, about 64 / |A|)
// and split the item's sources, a fixed-order tree of shuffles sums them, and
// the item's sums per body go to its rows of part (4 doubles per body).
//   P2P: the bodies of the sent leaves, direct sum skipping r = 0 pairs
//        (absolute float64 positions xa, xb in sorted order; FAST takes the
//        reciprocal square root at float32 precision, for the mixed path);
//   M2P: the multipole series of each multipole-only cell at the body, with
//        t = (x - c_B) / h_B:  phi += Re L_0^0 / h_B,
//        E += (Re L_1^1, Im L_1^1, -Re L_1^0) / h_B^2,
//        L_j^s = (-1)^j sum_{n<p, m} M_n^m I_{n+j}^{m+s}(t)
//   (the local expansion of the series about the body itself, whose value
//   and gradient there are the series' own).
__device__ __forceinline__ int lanes_per_body(int cnt)
{
    int G = 1;
    while (G < 16 && 2 * G * cnt <= 64) G *= 2;
    return G;
}

template <bool FAST>
__device__ __forceinline__ double rsqrt_d(double r2)
{
    if (FAST) return (double)__builtin_amdgcn_rsqf((float)r2);
    return 1.0 / sqrt(r2);
}

// the M2P series of one multipole row (real layout, scaled) at t, accumulated
template <class TM>
__device__ __forceinline__ void m2p_series(const TM *Mr, int p, double tx, double ty, double tz, double &l00,
                                           double &l10, double &l11r, double &l11i)
{
    const double r2 = tx * tx + ty * ty + tz * tz, ir2 = 1.0 / r2;
    cdd mm = {1.0 / sqrt(r2), 0.0};  // I_m^m
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const double f = -(2.0 * m - 1.0) * ir2;
            mm = cdd{(mm.re * tx - mm.im * ty) * f, (mm.re * ty + mm.im * tx) * f};
        }
        cdd i1 = mm, i2 = {0.0, 0.0};
        for (int n = m; n <= p; ++n) {
            if (n > m) {
                cdd cur;
                if (n == m + 1) cur = cdd{i1.re * (2.0 * m + 1.0) * tz * ir2, i1.im * (2.0 * m + 1.0) * tz * ir2};
                else {
                    const double a = (2.0 * n - 1.0) * tz, bb = -(double)((n + m - 1) * (n - m - 1));
                    cur = cdd{(a * i1.re + bb * i2.re) * ir2, (a * i1.im + bb * i2.im) * ir2};
                }
                i2 = i1;
                i1 = cur;
            }
            const cdd I = i1;  // I_n^m(t)
            const double w = m == 0 ? 1.0 : 2.0;
            if (n < p) {  // phi: M_n^m I_n^m, both signs of m
                const double Mre = (double)Mr[m == 0 ? n * n : n * n + 2 * m - 1];
                const double Mim = m == 0 ? 0.0 : (double)Mr[n * n + 2 * m];
                l00 += w * (Mre * I.re - Mim * I.im);
            }
            if (n >= 1 && n - 1 >= m) {  // L_1^0 = -sum M_{n-1}^m I_n^m, both signs of m
                const int d = n - 1;
                const double Mre = (double)Mr[m == 0 ? d * d : d * d + 2 * m - 1];
                const double Mim = m == 0 ? 0.0 : (double)Mr[d * d + 2 * m];
                l10 -= w * (Mre * I.re - Mim * I.im);
            }
            // L_1^1 = -sum_{m'>=0} M_{n-1}^{m'} I_n^{m'+1} + sum_{k>=1} conj(M_{n-1}^k I_n^{k-1})
            if (n >= 1 && m >= 1) {  // m' = m - 1
                const int d = n - 1, mp = m - 1;
                const double Mre = (double)Mr[mp == 0 ? d * d : d * d + 2 * mp - 1];
                const double Mim = mp == 0 ? 0.0 : (double)Mr[d * d + 2 * mp];
                l11r -= Mre * I.re - Mim * I.im;
                l11i -= Mre * I.im + Mim * I.re;
            }
            if (n >= 1 && m + 1 <= n - 1) {  // k = m + 1
                const int d = n - 1, kk = m + 1;
                const double Mre = (double)Mr[d * d + 2 * kk - 1], Mim = (double)Mr[d * d + 2 * kk];
                l11r += Mre * I.re - Mim * I.im;
                l11i -= Mre * I.im + Mim * I.re;
            }
        }
    }
}

template <class TM, bool FAST>
__global__ __launch_bounds__(64) void k_leaf_remote(TreeRef A, TreeRef B, const int32_t *it_leaf, const int64_t *it_k0,
                                                    const int64_t *it_k1, const int64_t *it_base, int kind,
                                                    const int32_t *src, const double4 *xa, const double4 *xb, int p,
                                                    int P2pad, const TM *MB, double4 *part)
{
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int c = it_leaf[item];
    const int32_t b0 = A.beg[c], cnt = A.end[c] - b0;
    const int G = lanes_per_body(cnt);
    const int sub = lane % G, per = 64 / G;
    const int64_t k0 = it_k0[item], k1 = it_k1[item];
    for (int32_t base = 0; base < cnt; base += per) {
        const int t = base + lane / G;
        const bool act = t < cnt;
        const double4 X = xa[b0 + (act ? t : 0)];
        double ph = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        if (kind == 0) {
            // P2P: the item's source bodies, dealt to the G lanes in turn
            int rot = 0;
            for (int64_t k = k0; k < k1; ++k) {
                const int b = src[k];
                const int32_t j0 = B.beg[b], nb = B.end[b] - j0;
                for (int32_t jj = (sub - rot + G) % G; jj < nb; jj += G) {
                    const double4 Y = xb[j0 + jj];
                    const double dx = X.x - Y.x, dy = X.y - Y.y, dz = X.z - Y.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;
                    const double ri = rsqrt_d<FAST>(r2);
                    const double qr = Y.w * ri, qr3 = qr * ri * ri;
                    ph += qr;
                    ex += qr3 * dx;
                    ey += qr3 * dy;
                    ez += qr3 * dz;
                }
                rot = (rot + nb) % G;
            }
        } else {
            // M2P: the item's cells dealt to the G lanes
            for (int64_t k = k0 + sub; k < k1; k += G) {
                const int b = src[k];
                const double ih = 1.0 / side(B, b);
                const double tx = (X.x - B.ctr[3 * b]) * ih, ty = (X.y - B.ctr[3 * b + 1]) * ih,
                             tz = (X.z - B.ctr[3 * b + 2]) * ih;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                m2p_series<TM>(MB + (int64_t)b * P2pad, p, tx, ty, tz, a0, a1, a2, a3);
                ph += a0 * ih;
                ex += a2 * ih * ih;
                ey += a3 * ih * ih;
                ez += -a1 * ih * ih;
            }
        }
        // the G lanes of a body, in a fixed order
        for (int w = 1; w < G; w <<= 1) {
            const double rp = __shfl_down(ph, w, 64), rx = __shfl_down(ex, w, 64);
            const double ry = __shfl_down(ey, w, 64), rz = __shfl_down(ez, w, 64);
            if (sub % (2 * w) == 0 && sub + w < G) {
                ph += rp;
                ex += rx;
                ey += ry;
                ez += rz;
            }
        }
        if (act && sub == 0) part[it_base[item] + t] = make_double4(ph, ex, ey, ez);
    }
}

// Each body of a leaf: its items' sums in item order (P2P items, then M2P
// items), added to the body's potential and field.
template <class TS>
__global__ __launch_bounds__(256) void k_leaf_reduce(TreeRef A, const int32_t *lf, const int64_t *lf_i,
                                                     const int64_t *it_base, int64_t nlf, const double4 *part,
                                                     TS *phi_s, TS *E_s)
{
    const int64_t k = blockIdx.x;
    if (k >= nlf) return;
    const int c = lf[k];
    const int32_t b0 = A.beg[c], cnt = A.end[c] - b0;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
        double ph = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int64_t it = lf_i[k]; it < lf_i[k + 1]; ++it) {
            const double4 v = part[it_base[it] + t];
            ph += v.x;
            ex += v.y;
            ey += v.z;
            ez += v.w;
        }
        const int64_t i = b0 + t;
        phi_s[i] = (TS)((double)phi_s[i] + ph);
        E_s[3 * i] = (TS)((double)E_s[3 * i] + ex);
        E_s[3 * i + 1] = (TS)((double)E_s[3 * i + 1] + ey);
        E_s[3 * i + 2] = (TS)((double)E_s[3 * i + 2] + ez);
    }
}

// sorted absolute positions and charges of a rank (x, q in member order)
__global__ __launch_bounds__(256) void k_sorted_bodies(const double *xr, const double *qr, const int32_t *perm,
                                                       int64_t n, double4 *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    out[i] = make_double4(xr[3 * o], xr[3 * o + 1], xr[3 * o + 2], qr[o]);
}

template <class TC, class TO>
__global__ __launch_bounds__(256) void k_let_out(const TC *phi_s, const TC *E_s, const int32_t *perm,
                                                 const int32_t *mem, int64_t n, TO *phi, TO *field)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = mem[perm[i]];
    phi[o] = (TO)phi_s[i];
    if (field) {
        field[3 * o] = (TO)E_s[3 * i];
        field[3 * o + 1] = (TO)E_s[3 * i + 1];
        field[3 * o + 2] = (TO)E_s[3 * i + 2];
    }
}

// ------------------------------------------------------------ work counts
// per cell: entries of its M2L lists (same-level slots, cross-level CSR) and,
// for leaves, the bodies of its P2P list
__global__ __launch_bounds__(256) void k_slot_counts(const int32_t *slots, const int32_t *tile_tgt, int64_t ntile,
                                                     int K, int TW, int64_t *own)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile * TW) return;
    const int64_t tile = t / TW;
    const int lane = (int)(t % TW);
    const int32_t c = tile_tgt[t];
    if (c < 0) return;
    int64_t cnt = 0;
    for (int k = 0; k < K; ++k) cnt += slots[(tile * K + k) * TW + lane] >= 0;
    own[c] += cnt;
}

__global__ __launch_bounds__(256) void k_csr_counts(const int64_t *off, const int32_t *src, const int32_t *beg,
                                                    const int32_t *end, int64_t nc, int bodies, int64_t *own)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc || !off) return;
    int64_t s = 0;
    if (bodies)
        for (int64_t k = off[c]; k < off[c + 1]; ++k) s += end[src[k]] - beg[src[k]];
    else s = off[c + 1] - off[c];
    own[c] += s;
}

__global__ __launch_bounds__(256) void k_down_counts(int64_t start, int64_t cnt, const int32_t *par, int64_t *own)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    const int64_t c = start + j;
    own[c] += own[par[c]];
}

__global__ __launch_bounds__(256) void k_work_out(const int32_t *leaf_of, const int32_t *perm, const int32_t *mem,
                                                  int64_t n, const int64_t *own, int64_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[mem[perm[i]]] = own[leaf_of[i]];
}

// ------------------------------------------------------------------ host
struct RemoteLists {
    int64_t n[3] = {0, 0, 0};                 // M2L, P2P, M2P pairs
    uint64_t dig[3] = {0, 0, 0};
    int64_t *off[3] = {nullptr, nullptr, nullptr};
    int32_t *src[3] = {nullptr, nullptr, nullptr};
    // work items: M2L runs of one target (and each target's first item);
    // P2P and M2P runs of one leaf (rows of their sums; each leaf's items)
    int64_t nmi = 0, nmt = 0, npi = 0, nqi = 0, nlf = 0, nrow = 0;
    int32_t *mi_tgt = nullptr, *mt_tgt = nullptr, *pi_leaf = nullptr, *qi_leaf = nullptr, *lf = nullptr;
    int64_t *mi_k0 = nullptr, *mi_k1 = nullptr, *mt_i = nullptr, *pi_k0 = nullptr, *pi_k1 = nullptr;
    int64_t *qi_k0 = nullptr, *qi_k1 = nullptr, *it_base = nullptr, *lf_i = nullptr;
    int64_t *pb = nullptr, *qb = nullptr;  // row base of each P2P / M2P item
    int64_t let[5] = {0, 0, 0, 0, 0};         // cells, multipole-only, body leaves, bodies, digest
};

void *dalloc(Allocator &al, size_t bytes) { return al.alloc(std::max<size_t>(bytes, 8)); }

int bits_of(int64_t v)
{
    int b = 1;
    while ((1ll << b) <= v) ++b;
    return b;
}

// Host copy of a CSR offset array.
std::vector<int64_t> host_offsets(const int64_t *d, int64_t nc, hipStream_t s)
{
    std::vector<int64_t> h(nc + 1);
    FMM_HIP(hipMemcpyAsync(h.data(), d, sizeof(int64_t) * (nc + 1), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    return h;
}

}  // namespace

// The whole virtual-rank evaluation (see fmm_let_evaluate in fmm.h).
void let_evaluate(const void *x, const void *q, fmm_dtype dtype, int64_t n, int R, const int64_t *w,
                  const fmm_params &prm, const fmm_allocator *ualloc, void *phi, void *field, int32_t *rank_out,
                  int64_t *work_l, int64_t *work_r, int64_t *pair_stats, fmm_let_stats *stats, hipStream_t s)
{
    using clock = std::chrono::steady_clock;
    auto ms_since = [](clock::time_point a) {
        return std::chrono::duration<double, std::milli>(clock::now() - a).count();
    };
    const auto t0 = clock::now();
    Allocator al;
    al.stream = s;
    if (ualloc) {
        al.user = *ualloc;
        al.has_user = true;
    }
    std::vector<void *> held;  // freed at the end (also on error)
    std::vector<fmm_plan *> plans(R, nullptr);
    auto hold = [&](size_t bytes) {
        void *p = dalloc(al, bytes);
        held.push_back(p);
        return p;
    };
    try {
        // ---- coordinates in float64 and the ORB partition
        double *X = static_cast<double *>(hold(sizeof(double) * 3 * n));
        double *Q = static_cast<double *>(hold(sizeof(double) * n));
        int32_t *ident = static_cast<int32_t *>(hold(sizeof(int32_t) * n));
        {
            std::vector<int32_t> h(n);
            for (int64_t i = 0; i < n; ++i) h[i] = (int32_t)i;
            FMM_HIP(hipMemcpyAsync(ident, h.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
            if (dtype == FMM_F64)
                k_gather_rank<double><<<grid1(n, 256), 256, 0, s>>>(static_cast<const double *>(x),
                                                                    static_cast<const double *>(q), ident, n, X, Q);
            else
                k_gather_rank<float><<<grid1(n, 256), 256, 0, s>>>(static_cast<const float *>(x),
                                                                   static_cast<const float *>(q), ident, n, X, Q);
            FMM_HIP(hipGetLastError());
            FMM_HIP(hipStreamSynchronize(s));
        }
        if (w) {
            int *bad = static_cast<int *>(hold(sizeof(int)));
            FMM_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
            k_check_weights<<<grid1(n, 256), 256, 0, s>>>(w, n, bad);
            FMM_HIP(hipGetLastError());
            int hb = 0;
            FMM_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
            FMM_HIP(hipStreamSynchronize(s));
            FMM_CHECK(hb == 0, FMM_ERR_INVALID, "weights must be in [0, 2^40)");
        }
        int32_t *idx = ident;  // members, split in place segment by segment
        int32_t *rank = static_cast<int32_t *>(hold(sizeof(int32_t) * n));
        std::vector<int64_t> rstart(R, 0), rcount(R, 0);
        {
            struct Seg { int64_t off, cnt; int m, r0; };
            std::vector<Seg> st{{0, n, R, 0}};
            uint64_t *key = static_cast<uint64_t *>(hold(sizeof(uint64_t) * n));
            int32_t *val = static_cast<int32_t *>(hold(sizeof(int32_t) * n));
            int64_t *wt = static_cast<int64_t *>(hold(sizeof(int64_t) * n));
            int64_t *pre = static_cast<int64_t *>(hold(sizeof(int64_t) * n));
            int64_t *aux = static_cast<int64_t *>(hold(sizeof(int64_t) * 2));
            double *part = static_cast<double *>(hold(sizeof(double) * 6 * 1025));
            while (!st.empty()) {
                const Seg g = st.back();
                st.pop_back();
                if (g.cnt == 0) continue;
                if (g.m <= 1) {
                    rstart[g.r0] = g.off;
                    rcount[g.r0] = g.cnt;
                    k_set_rank<<<grid1(g.cnt, 256), 256, 0, s>>>(idx + g.off, g.cnt, g.r0, rank);
                    FMM_HIP(hipGetLastError());
                    continue;
                }
                const int nb = (int)std::min<int64_t>(1024, (g.cnt + 255) / 256);
                k_seg_box<<<nb, 256, 0, s>>>(X, idx + g.off, g.cnt, part);
                k_box_final<<<1, 64, 0, s>>>(part, nb, part + 6 * 1024);
                FMM_HIP(hipGetLastError());
                double box[6];
                FMM_HIP(hipMemcpyAsync(box, part + 6 * 1024, sizeof(box), hipMemcpyDeviceToHost, s));
                FMM_HIP(hipStreamSynchronize(s));
                int axis = 0;
                for (int d = 1; d < 3; ++d)
                    if (box[3 + d] - box[d] > box[3 + axis] - box[axis]) axis = d;
                k_orb_keys<<<grid1(g.cnt, 256), 256, 0, s>>>(X, idx + g.off, g.cnt, axis, key, val);
                FMM_HIP(hipGetLastError());
                radix_sort_u64(key, val, g.cnt, 64, al, s);  // stable: ties keep ascending index
                k_orb_weights<<<grid1(g.cnt, 256), 256, 0, s>>>(w, val, g.cnt, wt);
                FMM_HIP(hipGetLastError());
                scan_exclusive_i64(wt, pre, g.cnt, aux, al, s);
                const int mL = g.m / 2;
                k_orb_find<<<1, 64, 0, s>>>(pre, aux, g.cnt, g.m, mL, aux + 1);
                FMM_HIP(hipGetLastError());
                int64_t k = 0;
                FMM_HIP(hipMemcpyAsync(&k, aux + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
                FMM_HIP(hipStreamSynchronize(s));
                // each side back in ascending index order
                for (int side_ = 0; side_ < 2; ++side_) {
                    const int64_t o = side_ ? k : 0, c = side_ ? g.cnt - k : k;
                    if (c == 0) continue;
                    k_idx_keys<<<grid1(c, 256), 256, 0, s>>>(val + o, c, key);
                    FMM_HIP(hipGetLastError());
                    radix_sort_u64(key, nullptr, c, 31, al, s);
                    k_keys_to_idx<<<grid1(c, 256), 256, 0, s>>>(key, c, idx + g.off + o);
                    FMM_HIP(hipGetLastError());
                }
                st.push_back({g.off + k, g.cnt - k, g.m - mL, g.r0 + mL});
                st.push_back({g.off, k, mL, g.r0});
            }
            FMM_HIP(hipStreamSynchronize(s));
        }
        if (rank_out) FMM_HIP(hipMemcpyAsync(rank_out, rank, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        const double ms_part = ms_since(t0);

        // ---- local trees: one plan per rank, from its own bodies
        const auto t1 = clock::now();
        std::vector<double *> xr(R, nullptr), qr(R, nullptr);
        for (int r = 0; r < R; ++r) {
            if (rcount[r] == 0) continue;
            xr[r] = static_cast<double *>(hold(sizeof(double) * 3 * rcount[r]));
            qr[r] = static_cast<double *>(hold(sizeof(double) * rcount[r]));
            k_gather_rank<double><<<grid1(rcount[r], 256), 256, 0, s>>>(X, Q, idx + rstart[r], rcount[r], xr[r], qr[r]);
            FMM_HIP(hipGetLastError());
            fmm_params pr = prm;
            fmm_plan *P = nullptr;
            const fmm_status st = fmm_build(xr[r], FMM_F64, rcount[r], &pr, ualloc, s, &P);
            if (st != FMM_OK) throw Error(st, std::string("rank ") + std::to_string(r) + ": " + fmm_last_error());
            plans[r] = P;
        }
        const double ms_build = ms_since(t1);

        // ---- LETs and the remote traversals (geometry only)
        const auto t2 = clock::now();
        const int64_t RR = (int64_t)R * R;
        std::vector<RemoteLists> RL(RR);
        unsigned long long *acc = static_cast<unsigned long long *>(hold(sizeof(unsigned long long) * 8));
        for (int r = 0; r < R; ++r) {
            if (!plans[r]) continue;
            fmm_plan *PA = plans[r];
            const TreeRef A = tree_ref(PA);
            for (int sdr = 0; sdr < R; ++sdr) {
                if (sdr == r || !plans[sdr]) continue;
                fmm_plan *PB = plans[sdr];
                const TreeRef B = tree_ref(PB);
                RemoteLists &L = RL[(int64_t)r * R + sdr];
                uint8_t *kind = static_cast<uint8_t *>(dalloc(al, PB->ncell));
                FMM_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long) * 8, s));
                k_let_kind<<<grid1(PB->ncell, 256), 256, 0, s>>>(B, PA->lo[0], PA->lo[1], PA->lo[2], PA->S, PA->t4,
                                                                 kind, acc);
                FMM_HIP(hipGetLastError());
                // frontier walk from (root of r, root of the grafted tree)
                std::vector<std::pair<uint64_t *, int64_t>> parts[3];
                int2 *F = static_cast<int2 *>(dalloc(al, sizeof(int2)));
                FMM_HIP(hipMemsetAsync(F, 0, sizeof(int2), s));
                int64_t nf = 1;
                int64_t *tot = static_cast<int64_t *>(dalloc(al, sizeof(int64_t) * 5));
                while (nf > 0) {
                    int32_t *cnt = static_cast<int32_t *>(dalloc(al, sizeof(int32_t) * 4 * nf));
                    int64_t *off = static_cast<int64_t *>(dalloc(al, sizeof(int64_t) * 4 * nf));
                    k_lx_count<<<grid1(nf, 256), 256, 0, s>>>(A, B, kind, PA->t4, F, nf, cnt);
                    FMM_HIP(hipGetLastError());
                    scan_exclusive_i32to64(cnt, off, 4 * nf, tot + 4, al, s);
                    k_lx_totals<<<1, 64, 0, s>>>(off, nf, tot);
                    FMM_HIP(hipGetLastError());
                    int64_t h[4];
                    FMM_HIP(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
                    FMM_HIP(hipStreamSynchronize(s));
                    uint64_t *o3[3];
                    for (int t = 0; t < 3; ++t) {
                        o3[t] = h[t] ? static_cast<uint64_t *>(dalloc(al, sizeof(uint64_t) * h[t])) : nullptr;
                        if (o3[t]) parts[t].push_back({o3[t], h[t]});
                    }
                    int2 *nx = h[3] ? static_cast<int2 *>(dalloc(al, sizeof(int2) * h[3])) : nullptr;
                    k_lx_write<<<grid1(nf, 256), 256, 0, s>>>(A, B, kind, PA->t4, F, nf, off, o3[0], o3[1], o3[2], nx);
                    FMM_HIP(hipGetLastError());
                    al.free(off);
                    al.free(cnt);
                    al.free(F);
                    F = nx;
                    nf = h[3];
                }
                if (F) al.free(F);
                al.free(tot);
                unsigned long long hacc[5];
                FMM_HIP(hipMemcpyAsync(hacc, acc, sizeof(hacc), hipMemcpyDeviceToHost, s));
                FMM_HIP(hipStreamSynchronize(s));
                for (int t = 0; t < 5; ++t) L.let[t] = (int64_t)hacc[t];
                al.free(kind);
                // each list: concatenated, sorted by (target, source), as CSR
                const int bits = 32 + bits_of(std::max<int64_t>(PA->ncell, 2));
                for (int t = 0; t < 3; ++t) {
                    int64_t np = 0;
                    for (auto &pp : parts[t]) np += pp.second;
                    L.n[t] = np;
                    uint64_t *all = static_cast<uint64_t *>(hold(sizeof(uint64_t) * std::max<int64_t>(1, np)));
                    int64_t o = 0;
                    for (auto &pp : parts[t]) {
                        FMM_HIP(hipMemcpyAsync(all + o, pp.first, sizeof(uint64_t) * pp.second, hipMemcpyDeviceToDevice,
                                               s));
                        o += pp.second;
                    }
                    for (auto &pp : parts[t]) al.free(pp.first);
                    if (np > 1) radix_sort_u64(all, nullptr, np, std::min(64, bits), al, s);
                    L.off[t] = static_cast<int64_t *>(hold(sizeof(int64_t) * (PA->ncell + 1)));
                    L.src[t] = static_cast<int32_t *>(hold(sizeof(int32_t) * std::max<int64_t>(1, np)));
                    k_pair_offsets<<<grid1(PA->ncell + 1, 256), 256, 0, s>>>(all, np, PA->ncell, L.off[t]);
                    FMM_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
                    if (np > 0) k_pair_sources<<<grid1(np, 256), 256, 0, s>>>(all, np, L.src[t], acc);
                    FMM_HIP(hipGetLastError());
                    unsigned long long d = 0;
                    FMM_HIP(hipMemcpyAsync(&d, acc, sizeof(d), hipMemcpyDeviceToHost, s));
                    FMM_HIP(hipStreamSynchronize(s));
                    L.dig[t] = d;
                }
                // work items: runs of at most kRChunk M2L pairs of a target, of
                // 16 P2P source leaves or 8 M2P cells of a leaf
                const std::vector<int64_t> om = host_offsets(L.off[0], PA->ncell, s);
                const std::vector<int64_t> op = host_offsets(L.off[1], PA->ncell, s);
                const std::vector<int64_t> oq = host_offsets(L.off[2], PA->ncell, s);
                std::vector<int32_t> h_mi_tgt, h_mt_tgt, h_pi_leaf, h_qi_leaf, h_lf;
                std::vector<int64_t> h_mi_k0, h_mi_k1, h_mt_i, h_pi_k0, h_pi_k1, h_qi_k0, h_qi_k1, h_lf_i, h_base_p,
                    h_base_q;
                std::vector<int32_t> h_cnt(PA->ncell);
                FMM_HIP(hipMemcpyAsync(h_cnt.data(), PA->c_end, sizeof(int32_t) * PA->ncell, hipMemcpyDeviceToHost, s));
                std::vector<int32_t> h_beg(PA->ncell);
                FMM_HIP(hipMemcpyAsync(h_beg.data(), PA->c_beg, sizeof(int32_t) * PA->ncell, hipMemcpyDeviceToHost, s));
                FMM_HIP(hipStreamSynchronize(s));
                int64_t rows = 0;
                for (int64_t c = 0; c < PA->ncell; ++c) {
                    if (om[c + 1] > om[c]) {
                        h_mt_tgt.push_back((int32_t)c);
                        h_mt_i.push_back((int64_t)h_mi_tgt.size());
                        for (int64_t k = om[c]; k < om[c + 1]; k += kRChunk) {
                            h_mi_tgt.push_back((int32_t)c);
                            h_mi_k0.push_back(k);
                            h_mi_k1.push_back(std::min<int64_t>(om[c + 1], k + kRChunk));
                        }
                    }
                    if (op[c + 1] > op[c] || oq[c + 1] > oq[c]) {
                        const int64_t nb = h_cnt[c] - h_beg[c];
                        h_lf.push_back((int32_t)c);
                        h_lf_i.push_back((int64_t)(h_base_p.size() + h_base_q.size()));
                        for (int64_t k = op[c]; k < op[c + 1]; k += 16) {
                            h_pi_leaf.push_back((int32_t)c);
                            h_pi_k0.push_back(k);
                            h_pi_k1.push_back(std::min<int64_t>(op[c + 1], k + 16));
                            h_base_p.push_back(rows);
                            rows += nb;
                        }
                        for (int64_t k = oq[c]; k < oq[c + 1]; k += 8) {
                            h_qi_leaf.push_back((int32_t)c);
                            h_qi_k0.push_back(k);
                            h_qi_k1.push_back(std::min<int64_t>(oq[c + 1], k + 8));
                            h_base_q.push_back(rows);
                            rows += nb;
                        }
                    }
                }
                h_mt_i.push_back((int64_t)h_mi_tgt.size());
                // the reduction walks a leaf's items as one range of bases:
                // its P2P items' bases, then its M2P items' bases
                std::vector<int64_t> h_base;
                {
                    size_t ip = 0, iq = 0;
                    std::vector<int64_t> starts;
                    for (size_t k = 0; k < h_lf.size(); ++k) {
                        starts.push_back((int64_t)h_base.size());
                        const int c = h_lf[k];
                        while (ip < h_pi_leaf.size() && h_pi_leaf[ip] == c) h_base.push_back(h_base_p[ip++]);
                        while (iq < h_qi_leaf.size() && h_qi_leaf[iq] == c) h_base.push_back(h_base_q[iq++]);
                    }
                    starts.push_back((int64_t)h_base.size());
                    h_lf_i = starts;
                }
                L.nmi = (int64_t)h_mi_tgt.size();
                L.nmt = (int64_t)h_mt_tgt.size();
                L.npi = (int64_t)h_pi_leaf.size();
                L.nqi = (int64_t)h_qi_leaf.size();
                L.nlf = (int64_t)h_lf.size();
                L.nrow = rows;
                auto up32 = [&](const std::vector<int32_t> &v) {
                    int32_t *d = static_cast<int32_t *>(hold(sizeof(int32_t) * std::max<size_t>(1, v.size())));
                    if (!v.empty()) FMM_HIP(hipMemcpyAsync(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, s));
                    return d;
                };
                auto up64 = [&](const std::vector<int64_t> &v) {
                    int64_t *d = static_cast<int64_t *>(hold(sizeof(int64_t) * std::max<size_t>(1, v.size())));
                    if (!v.empty()) FMM_HIP(hipMemcpyAsync(d, v.data(), sizeof(int64_t) * v.size(), hipMemcpyHostToDevice, s));
                    return d;
                };
                L.mi_tgt = up32(h_mi_tgt);
                L.mi_k0 = up64(h_mi_k0);
                L.mi_k1 = up64(h_mi_k1);
                L.mt_tgt = up32(h_mt_tgt);
                L.mt_i = up64(h_mt_i);
                L.pi_leaf = up32(h_pi_leaf);
                L.pi_k0 = up64(h_pi_k0);
                L.pi_k1 = up64(h_pi_k1);
                L.qi_leaf = up32(h_qi_leaf);
                L.qi_k0 = up64(h_qi_k0);
                L.qi_k1 = up64(h_qi_k1);
                L.lf = up32(h_lf);
                L.lf_i = up64(h_lf_i);
                std::vector<int64_t> h_bp(h_base_p), h_bq(h_base_q);
                L.it_base = up64(h_base);
                L.pb = up64(h_bp);
                L.qb = up64(h_bq);
                FMM_HIP(hipStreamSynchronize(s));
            }
        }
        const double ms_let = ms_since(t2);

        // ---- evaluation: local M2L, remote M2L, downward pass, remote P2P and M2P
        const auto t3 = clock::now();
        const bool f64 = prm.precision == FMM_PREC_FP64;
        for (int r = 0; r < R; ++r)  // every sender's multipoles before any remote M2L
            if (plans[r]) eval_up(plans[r], qr[r], plans[r]->ubody, s);
        std::vector<double4 *> xs(R, nullptr);
        for (int r = 0; r < R; ++r) {
            if (!plans[r]) continue;
            xs[r] = static_cast<double4 *>(hold(sizeof(double4) * rcount[r]));
            k_sorted_bodies<<<grid1(rcount[r], 256), 256, 0, s>>>(xr[r], qr[r], plans[r]->perm, rcount[r], xs[r]);
            FMM_HIP(hipGetLastError());
        }
        for (int r = 0; r < R; ++r) {
            fmm_plan *PA = plans[r];
            if (!PA) continue;
            eval_m2l(PA, s);
            for (int sdr = 0; sdr < R; ++sdr) {
                const RemoteLists &L = RL[(int64_t)r * R + sdr];
                if (sdr == r || !plans[sdr] || L.nmi == 0) continue;
                fmm_plan *PB = plans[sdr];
                double *part = static_cast<double *>(dalloc(al, sizeof(double) * L.nmi * PA->P2pad));
                const int P2 = PA->p * PA->p;
                if (f64) {
                    k_m2l_remote<double><<<(unsigned)L.nmi, 64, 0, s>>>(tree_ref(PA), tree_ref(PB), L.mi_tgt, L.mi_k0,
                                                                         L.mi_k1, L.src[0], PA->p, PA->P2pad,
                                                                         static_cast<const double *>(PB->Mc), part);
                    k_m2l_remote_reduce<double><<<grid1(L.nmt * P2, 256), 256, 0, s>>>(
                        L.mt_tgt, L.mt_i, L.nmt, part, P2, PA->P2pad, static_cast<double *>(PA->Lc));
                } else {
                    k_m2l_remote<float><<<(unsigned)L.nmi, 64, 0, s>>>(tree_ref(PA), tree_ref(PB), L.mi_tgt, L.mi_k0,
                                                                        L.mi_k1, L.src[0], PA->p, PA->P2pad,
                                                                        static_cast<const float *>(PB->Mc), part);
                    k_m2l_remote_reduce<float><<<grid1(L.nmt * P2, 256), 256, 0, s>>>(
                        L.mt_tgt, L.mt_i, L.nmt, part, P2, PA->P2pad, static_cast<float *>(PA->Lc));
                }
                FMM_HIP(hipGetLastError());
                al.free(part);
            }
            eval_down(PA, PA->ubody, PA->phi_s, PA->E_s, s);
            for (int sdr = 0; sdr < R; ++sdr) {
                const RemoteLists &L = RL[(int64_t)r * R + sdr];
                if (sdr == r || !plans[sdr] || L.nlf == 0) continue;
                fmm_plan *PB = plans[sdr];
                double4 *part = static_cast<double4 *>(dalloc(al, sizeof(double4) * L.nrow));
#define LEAF_REMOTE(TM, FAST, NI, LEAF, K0, K1, BASE, KIND, SRC)                                          \
    if (NI > 0)                                                                                        \
        k_leaf_remote<TM, FAST><<<(unsigned)NI, 64, 0, s>>>(tree_ref(PA), tree_ref(PB), LEAF, K0, K1, BASE, \
                                                           KIND, SRC, xs[r], xs[sdr], PA->p, PA->P2pad,  \
                                                           static_cast<const TM *>(PB->Mc), part)
                if (f64) {
                    LEAF_REMOTE(double, false, L.npi, L.pi_leaf, L.pi_k0, L.pi_k1, L.pb, 0, L.src[1]);
                    LEAF_REMOTE(double, false, L.nqi, L.qi_leaf, L.qi_k0, L.qi_k1, L.qb, 1, L.src[2]);
                    k_leaf_reduce<double><<<(unsigned)L.nlf, 64, 0, s>>>(tree_ref(PA), L.lf, L.lf_i, L.it_base, L.nlf,
                                                                         part, static_cast<double *>(PA->phi_s),
                                                                         static_cast<double *>(PA->E_s));
                } else {
                    LEAF_REMOTE(float, true, L.npi, L.pi_leaf, L.pi_k0, L.pi_k1, L.pb, 0, L.src[1]);
                    LEAF_REMOTE(float, true, L.nqi, L.qi_leaf, L.qi_k0, L.qi_k1, L.qb, 1, L.src[2]);
                    k_leaf_reduce<float><<<(unsigned)L.nlf, 64, 0, s>>>(tree_ref(PA), L.lf, L.lf_i, L.it_base, L.nlf,
                                                                        part, static_cast<float *>(PA->phi_s),
                                                                        static_cast<float *>(PA->E_s));
                }
#undef LEAF_REMOTE
                FMM_HIP(hipGetLastError());
                al.free(part);
            }
            // results to the caller's order
            int32_t *mem = idx + rstart[r];
            const int64_t nr = rcount[r];
#define LET_OUT(TC, TO)                                                                                      \
    k_let_out<TC, TO><<<grid1(nr, 256), 256, 0, s>>>(static_cast<const TC *>(PA->phi_s),                     \
                                                    static_cast<const TC *>(PA->E_s), PA->perm, mem, nr,     \
                                                    static_cast<TO *>(phi), static_cast<TO *>(field))
            if (f64 && dtype == FMM_F64) LET_OUT(double, double);
            else if (f64) LET_OUT(double, float);
            else if (dtype == FMM_F64) LET_OUT(float, double);
            else LET_OUT(float, float);
#undef LET_OUT
            FMM_HIP(hipGetLastError());
        }
        FMM_HIP(hipStreamSynchronize(s));
        const double ms_eval = ms_since(t3);

        // ---- work of every body (Eq. (1): l_i local, r_i remote)
        if (work_l || work_r) {
            for (int r = 0; r < R; ++r) {
                fmm_plan *PA = plans[r];
                if (!PA) continue;
                const int64_t nc = PA->ncell;
                int64_t *own = static_cast<int64_t *>(dalloc(al, sizeof(int64_t) * nc));
                for (int which = 0; which < 2; ++which) {
                    int64_t *out = which == 0 ? work_l : work_r;
                    if (!out) continue;
                    FMM_HIP(hipMemsetAsync(own, 0, sizeof(int64_t) * nc, s));
                    if (which == 0) {
                        if (PA->ntile > 0 && PA->K > 0)
                            k_slot_counts<<<grid1(PA->ntile * PA->TW, 256), 256, 0, s>>>(PA->slots, PA->tile_tgt,
                                                                                         PA->ntile, PA->K, PA->TW, own);
                        k_csr_counts<<<grid1(nc, 256), 256, 0, s>>>(PA->m2lx_off, PA->m2lx_src, PA->c_beg, PA->c_end,
                                                                   nc, 0, own);
                        k_csr_counts<<<grid1(nc, 256), 256, 0, s>>>(PA->p2p_off, PA->p2p_src, PA->c_beg, PA->c_end,
                                                                   nc, 1, own);
                    } else {
                        for (int sdr = 0; sdr < R; ++sdr) {
                            const RemoteLists &L = RL[(int64_t)r * R + sdr];
                            if (sdr == r || !plans[sdr]) continue;
                            fmm_plan *PB = plans[sdr];
                            k_csr_counts<<<grid1(nc, 256), 256, 0, s>>>(L.off[0], L.src[0], PB->c_beg, PB->c_end, nc,
                                                                       0, own);
                            k_csr_counts<<<grid1(nc, 256), 256, 0, s>>>(L.off[2], L.src[2], PB->c_beg, PB->c_end, nc,
                                                                       0, own);
                            k_csr_counts<<<grid1(nc, 256), 256, 0, s>>>(L.off[1], L.src[1], PB->c_beg, PB->c_end, nc,
                                                                       1, own);
                        }
                    }
                    FMM_HIP(hipGetLastError());
                    for (int l = 1; l <= PA->depth; ++l) {
                        const int64_t cnt = PA->lv[l].count;
                        if (cnt == 0) continue;
                        k_down_counts<<<grid1(cnt, 256), 256, 0, s>>>(PA->lv[l].start, cnt, PA->c_par, own);
                        FMM_HIP(hipGetLastError());
                    }
                    k_work_out<<<grid1(rcount[r], 256), 256, 0, s>>>(PA->leaf_of, PA->perm, idx + rstart[r],
                                                                     rcount[r], own, out);
                    FMM_HIP(hipGetLastError());
                }
                FMM_HIP(hipStreamSynchronize(s));
                al.free(own);
            }
        }

        // ---- statistics
        if (pair_stats) {
            for (int64_t rs = 0; rs < RR; ++rs) {
                int64_t *o = pair_stats + 11 * rs;
                for (int k = 0; k < 11; ++k) o[k] = 0;
                const int r = (int)(rs / R), sdr = (int)(rs % R);
                if (r == sdr) {
                    if (plans[r]) {
                        uint64_t dg[2];
                        list_digest(plans[r], dg, s);
                        o[4] = plans[r]->n_m2l_same + plans[r]->n_m2l_cross;
                        o[5] = plans[r]->n_p2p;
                        o[7] = (int64_t)dg[0];
                        o[8] = (int64_t)dg[1];
                    }
                    continue;
                }
                const RemoteLists &L = RL[rs];
                for (int k = 0; k < 4; ++k) o[k] = L.let[k];
                for (int t = 0; t < 3; ++t) {
                    o[4 + t] = L.n[t];
                    o[7 + t] = (int64_t)L.dig[t];
                }
                o[10] = L.let[4];
            }
        }
        if (stats) {
            fmm_let_stats S{};
            S.nrank = R;
            for (int64_t rs = 0; rs < RR; ++rs) {
                const int r = (int)(rs / R), sdr = (int)(rs % R);
                if (r == sdr) {
                    if (plans[r]) {
                        S.n_m2l_local += plans[r]->n_m2l_same + plans[r]->n_m2l_cross;
                        S.n_p2p_local += plans[r]->n_p2p;
                    }
                    continue;
                }
                const RemoteLists &L = RL[rs];
                S.let_cells += L.let[0];
                S.let_far += L.let[1];
                S.let_body_leaves += L.let[2];
                S.let_bodies += L.let[3];
                S.n_m2l_remote += L.n[0];
                S.n_p2p_remote += L.n[1];
                S.n_m2p_remote += L.n[2];
            }
            for (int r = 0; r < R; ++r)
                if (plans[r]) S.device_bytes += plans[r]->bytes_held;
            const int64_t coef = (int64_t)prm.p * prm.p * (f64 ? 8 : 4);
            S.let_bytes = S.let_cells * (40 + coef) + S.let_bodies * 32;
            S.ms_partition = ms_part;
            S.ms_build = ms_build;
            S.ms_let = ms_let;
            S.ms_evaluate = ms_eval;
            S.ms_total = ms_since(t0);
            *stats = S;
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        for (fmm_plan *P : plans) fmm_destroy(P);
        for (void *p : held) al.free(p);
        allocator_done(al);
        throw;
    }
    FMM_HIP(hipStreamSynchronize(s));
    for (fmm_plan *P : plans) fmm_destroy(P);
    for (void *p : held) al.free(p);
    allocator_done(al);
}

}  // namespace fmm
