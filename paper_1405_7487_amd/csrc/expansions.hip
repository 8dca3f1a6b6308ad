// expansions.hip -- solid-harmonic expansions on gfx950: operator tables,
// P2M, M2M (upward pass), L2L and L2P (downward pass); Section II.A and II.C
// of the paper, with the operator algebra of Greengard & Rokhlin and Cheng,
// Greengard & Rokhlin (1999).
//
// Basis.  Regular and irregular solid harmonics
//     R_n^m(v) = r^n P_n^m(cos t) e^{i m f} / (n+m)!,
//     I_n^m(v) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1}    (m >= 0),
//     X_n^{-m} = (-1)^m conj(X_n^m),
// are generated here by their Cartesian three-term recurrences (no angles):
//     R_m^m = -(x + i y)/(2m) R_{m-1}^{m-1},  R_{m+1}^m = z R_m^m,
//     (n^2 - m^2) R_n^m = (2n-1) z R_{n-1}^m - r^2 R_{n-2}^m,
//     I_m^m = -(2m-1)(x + i y)/r^2 I_{m-1}^{m-1},  I_{m+1}^m = (2m+1) z/r^2 I_m^m,
//     r^2 I_n^m = (2n-1) z I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m.
// A multipole M_n^m = sum q conj(R_n^m(x - c)) and a local expansion L_j^s
// (phi = sum L_j^s conj(R_j^s(x - c))) are stored as p^2 reals per cell:
// degree n occupies [n^2, (n+1)^2): Re X_n^0, then (Re, Im) of X_n^m, m = 1..n.
// Coefficients are scaled per level (multipole by h^-n, local by h^{n+1}),
// which makes every translation operator between lattice centers independent
// of the level and keeps float32 values in range at any depth.
#include "internal.hpp"

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace fmm {

namespace {

__host__ __device__ __forceinline__ int ridx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }

// Constants of the regular recurrences, 1 / (n^2 - m^2) and -1 / (2m), for
// n, m < 16, rounded once each (compile-time IEEE division), so per-body code
// reads them instead of dividing.
struct RecTab {
    float inv_f[16][16];
    double inv_d[16][16];
    float half_f[16];
    double half_d[16];
};
constexpr RecTab make_rec_tab()
{
    RecTab t{};
    for (int n = 0; n < 16; ++n)
        for (int m = 0; m < 16; ++m) {
            t.inv_f[n][m] = n > m ? 1.0f / (float)(n * n - m * m) : 0.0f;
            t.inv_d[n][m] = n > m ? 1.0 / (double)(n * n - m * m) : 0.0;
        }
    for (int m = 0; m < 16; ++m) {
        t.half_f[m] = m > 0 ? -0.5f / (float)m : 0.0f;
        t.half_d[m] = m > 0 ? -0.5 / (double)m : 0.0;
    }
    return t;
}
__constant__ RecTab c_rec = make_rec_tab();
template <class T> __device__ __forceinline__ T rec_inv(int n, int m);
template <> __device__ __forceinline__ float rec_inv<float>(int n, int m) { return c_rec.inv_f[n][m]; }
template <> __device__ __forceinline__ double rec_inv<double>(int n, int m) { return c_rec.inv_d[n][m]; }
template <class T> __device__ __forceinline__ T rec_half(int m);
template <> __device__ __forceinline__ float rec_half<float>(int m) { return c_rec.half_f[m]; }
template <> __device__ __forceinline__ double rec_half<double>(int m) { return c_rec.half_d[m]; }

struct cd {
    double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.re, -a.im}; }

// Harmonic table access with the negative-order rule; zero outside |m| <= n.
__device__ __forceinline__ cd hget(const cd *H, int nmax, int n, int m)
{
    if (n < 0 || n >= nmax || m > n || m < -n) return {0.0, 0.0};
    if (m >= 0) return H[n * (n + 1) / 2 + m];
    cd v = H[n * (n + 1) / 2 - m];
    return (m & 1) ? cd{-v.re, v.im} : cd{v.re, -v.im};
}

// Regular harmonics (float64) of v for degrees < nmax into H (m >= 0).
__device__ void regular_table(double x, double y, double z, int nmax, cd *H)
{
    const double r2 = x * x + y * y + z * z;
    cd mm = {1.0, 0.0};
    for (int m = 0; m < nmax; ++m) {
        if (m > 0) mm = cscale(cmul(mm, cd{x, y}), -1.0 / (2.0 * m));
        cd p2 = {0.0, 0.0}, p1 = mm;
        H[m * (m + 1) / 2 + m] = mm;
        for (int n = m + 1; n < nmax; ++n) {
            cd cur;
            if (n == m + 1) cur = cscale(mm, z);
            else cur = cscale(cadd(cscale(p1, (2.0 * n - 1.0) * z), cscale(p2, -r2)), 1.0 / (double)(n * n - m * m));
            H[n * (n + 1) / 2 + m] = cur;
            p2 = p1;
            p1 = cur;
        }
    }
}

// Irregular harmonics (float64) of v != 0 for degrees < nmax into H.
__device__ void irregular_table(double x, double y, double z, int nmax, cd *H)
{
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    cd mm = {1.0 / sqrt(r2), 0.0};
    for (int m = 0; m < nmax; ++m) {
        if (m > 0) mm = cscale(cmul(mm, cd{x, y}), -(2.0 * m - 1.0) * ir2);
        cd p2 = {0.0, 0.0}, p1 = mm;
        H[m * (m + 1) / 2 + m] = mm;
        for (int n = m + 1; n < nmax; ++n) {
            cd cur;
            if (n == m + 1) cur = cscale(mm, (2.0 * m + 1.0) * z * ir2);
            else
                cur = cscale(cadd(cscale(p1, (2.0 * n - 1.0) * z), cscale(p2, -(double)((n + m - 1) * (n - m - 1)))), ir2);
            H[n * (n + 1) / 2 + m] = cur;
            p2 = p1;
            p1 = cur;
        }
    }
}

// Decode a real coefficient index into (degree, order, is-imaginary).
__host__ __device__ __forceinline__ void rdecode(int r, int &n, int &m, int &im)
{
    n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    const int o = r - n * n;
    if (o == 0) { m = 0; im = 0; }
    else { m = (o + 1) / 2; im = (o & 1) ? 0 : 1; }
}

// M2L operator for lattice offset t (target minus source, in cell sides):
// scaled local coefficients lt = T(t) mt with
//     L_j^s = (-1)^j sum_{n,m} M_n^m I_{n+j}^{m+s}(t).
// Written in the table layout of m2l_opsz / m2l_sch / m2l_gst (P2pad rows,
// 4 m2l_q(p) input columns; rows and columns beyond p^2 stay zero).
// Each operator is given as tr = (tau_x, tau_y, tau_z, e): the center offset
// c_A - c_B in units of the target's cell size h_A, and the source-to-target
// size ratio rho = h_B / h_A = 2^e (0 for same-level pairs), which scales
// input degree n by rho^n.
template <class T>
__global__ __launch_bounds__(256) void k_make_m2l_ops(const double4 *tr, int nops, int p, int P2pad, int SCH, int GST,
                                                      int64_t OPSZ, int tail, T *Tf)
{
    const int op = blockIdx.x;
    if (op >= nops) return;
    __shared__ cd H[(2 * kMaxP) * (2 * kMaxP + 1) / 2];
    const int nI = 2 * p - 1;
    const double4 t = tr[op];
    const int e2 = (int)t.w;
    if (threadIdx.x == 0) irregular_table(t.x, t.y, t.z, nI, H);
    __syncthreads();
    // (SCH, GST, OPSZ: the table layout, computed by the host)
    const int P2 = p * p, Q = m2l_q(p), NCOL = 4 * Q;
    const int RT = P2pad / 16;
    for (int e = threadIdx.x; e < P2pad * NCOL; e += blockDim.x) {
        const int row = e / NCOL, col = e % NCOL;
        // tail: the last row tile holds its (at most 4) coefficient rows
        // repeated in every group of 4 fragment lanes
        const int vrow = (tail && row >= P2pad - 16) ? P2pad - 16 + (row & 3) : row;
        double v = 0.0;
        if (vrow < P2 && col < P2) {
            int j, s, rim, n, m, cim;
            rdecode(vrow, j, s, rim);
            rdecode(col, n, m, cim);
            cd d;
            if (m == 0) {
                d = hget(H, nI, n + j, s);
            } else {
                cd a = hget(H, nI, n + j, m + s), b = hget(H, nI, n + j, s - m);
                const double sg = (m & 1) ? -1.0 : 1.0;
                if (!cim) d = {a.re + sg * b.re, a.im + sg * b.im};
                else d = {-(a.im - sg * b.im), a.re - sg * b.re};  // i (a - sg b)
            }
            if (j & 1) d = {-d.re, -d.im};
            v = ldexp(rim ? d.im : d.re, e2 * n);
        }
        const int g = col / Q, sq = col % Q, c = sq / SCH, ss = sq % SCH;
        Tf[(size_t)op * OPSZ + (size_t)(c * 4 + g) * GST + ss * P2pad + (row % 16) * RT + row / 16] = (T)v;
    }
}

// M2M and L2L matrices for the 8 child octants (child - parent center =
// (h_child/2) sigma, sigma_d = +1 where the octant bit is set):
//   M2M: M'_n^m = 2^-n sum_{k,l} M_k^l conj(R_{n-k}^{m-l}(sigma/2))
//   L2L: L'_k^l = sum_{j,s} 2^-(j+1) L_j^s conj(R_{j-k}^{s-l}(sigma/2))
__global__ __launch_bounds__(256) void k_make_shift_ops(int p, int P2pad, double *m2m, double *l2l)
{
    const int oct = blockIdx.x;
    __shared__ cd H[kMaxP * (kMaxP + 1) / 2];
    if (threadIdx.x == 0) {
        const double sx = (oct & 4) ? 0.5 : -0.5, sy = (oct & 2) ? 0.5 : -0.5, sz = (oct & 1) ? 0.5 : -0.5;
        regular_table(sx, sy, sz, p, H);
    }
    __syncthreads();
    const int P2 = p * p;
    for (int e = threadIdx.x; e < P2pad * P2pad; e += blockDim.x) {
        const int row = e / P2pad, col = e % P2pad;
        double vm = 0.0, vl = 0.0;
        if (row < P2 && col < P2) {
            int n, m, rim, k, l, cim;
            rdecode(row, n, m, rim);
            rdecode(col, k, l, cim);
            // M2M: output (n,m), input (k,l)
            {
                cd d;
                if (l == 0) {
                    d = cconj(hget(H, p, n - k, m));
                } else {
                    cd a = cconj(hget(H, p, n - k, m - l)), b = cconj(hget(H, p, n - k, m + l));
                    const double sg = (l & 1) ? -1.0 : 1.0;
                    if (!cim) d = {a.re + sg * b.re, a.im + sg * b.im};
                    else d = {-(a.im - sg * b.im), a.re - sg * b.re};
                }
                const double sc = ldexp(1.0, -n);
                vm = (rim ? d.im : d.re) * sc;
            }
            // L2L: output (k'=n, l'=m), input (j=k, s=l)
            {
                const int ko = n, lo = m, j = k, s = l;
                cd d;
                if (s == 0) {
                    d = cconj(hget(H, p, j - ko, -lo));
                } else {
                    cd a = cconj(hget(H, p, j - ko, s - lo)), b = cconj(hget(H, p, j - ko, -s - lo));
                    const double sg = (s & 1) ? -1.0 : 1.0;
                    if (!cim) d = {a.re + sg * b.re, a.im + sg * b.im};
                    else d = {-(a.im - sg * b.im), a.re - sg * b.re};
                }
                const double sc = ldexp(1.0, -(j + 1));
                vl = (rim ? d.im : d.re) * sc;
            }
        }
        // stored transposed ([oct][col][row]) so that threads of consecutive
        // rows read consecutive addresses
        m2m[((size_t)oct * P2pad + col) * P2pad + row] = vm;
        l2l[((size_t)oct * P2pad + col) * P2pad + row] = vl;
    }
}

__global__ __launch_bounds__(256) void k_d2f(const double *a, float *b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ P2M
// One wave per leaf.  Each body of a chunk (<= 32) gets an LDS row of the p^2
// real components of q conj(R(u / h)) (rolling Cartesian recurrence, its
// orders split between two lanes), then each lane sums coefficient columns
// over the chunk in body order.  Deterministic; no atomics.
template <class T, class V4>
__global__ __launch_bounds__(64) void k_p2m(const int32_t *leaves, const int32_t *beg, const int32_t *end,
                                            const int32_t *lvl, const V4 *ub, double S, int p, int P2pad, int chunk,
                                            T *Mc, double *M64, int64_t ncoarse)
{
    extern __shared__ __align__(16) unsigned char p2m_smem[];
    T *rows = reinterpret_cast<T *>(p2m_smem);  // [chunk][P2 + 1], chunk <= 64
    const int lane = threadIdx.x;
    const int c = leaves[blockIdx.x];
    const int P2 = p * p, stride = P2 + 1;
    const T ih = (T)ldexp(1.0 / S, lvl[c]);
    T acc[4] = {0, 0, 0, 0};  // coefficients lane + 64 q, q < 4 (p <= 16)
    // Chunks of at most 32 bodies: the two halves of the wave take the same
    // bodies and split the orders m, the first half m < ms and the second
    // m >= ms, ms balancing the (p - m) terms of each.
    const bool halves = chunk <= 32;
    int ms = p;
    if (halves) {
        int w = 0;
        ms = 0;
        while (ms < p && 2 * (w + p - ms) <= p * (p + 1) / 2) w += p - ms++;
    }
    const int h = halves ? lane >> 5 : 0, bl = halves ? lane & 31 : lane;
    const int mlo = h ? ms : 0, mhi = halves && !h ? ms : p;
    for (int32_t b0 = beg[c]; b0 < end[c]; b0 += chunk) {
        const int nb = min(chunk, end[c] - b0);
        if (bl < nb) {
            const V4 u = ub[b0 + bl];
            const T x = u.x * ih, y = u.y * ih, z = u.z * ih, q = u.w;
            const T r2 = x * x + y * y + z * z;
            T *row = rows + bl * stride;
            T mre = q, mim = 0;  // q R_m^m
            for (int m = 1; m < mlo; ++m) {
                const T f = rec_half<T>(m);
                const T nr = (mre * x - mim * y) * f;
                const T ni = (mre * y + mim * x) * f;
                mre = nr;
                mim = ni;
            }
            for (int m = mlo; m < mhi; ++m) {
                if (m > 0) {
                    const T f = rec_half<T>(m);
                    const T nr = (mre * x - mim * y) * f;
                    const T ni = (mre * y + mim * x) * f;
                    mre = nr;
                    mim = ni;
                }
                T p2r = 0, p2i = 0, p1r = mre, p1i = mim;
                for (int n = m; n < p; ++n) {
                    T cr, ci;
                    if (n == m) { cr = mre; ci = mim; }
                    else if (n == m + 1) { cr = z * mre; ci = z * mim; }
                    else {
                        const T a = (T)(2 * n - 1), inv = rec_inv<T>(n, m);
                        cr = (a * z * p1r - r2 * p2r) * inv;
                        ci = (a * z * p1i - r2 * p2i) * inv;
                    }
                    if (n > m) { p2r = p1r; p2i = p1i; }
                    p1r = cr;
                    p1i = ci;
                    const int r = ridx_re(n, m);
                    row[r] = cr;                 // Re of q conj(R) = q Re R
                    if (m > 0) row[r + 1] = -ci; // Im of q conj(R) = -q Im R
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            const int col = lane + 64 * qd;
            if (col < P2)
                for (int j = 0; j < nb; ++j) acc[qd] += rows[j * stride + col];
        }
        __syncthreads();
    }
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
        const int col = lane + 64 * qd;
        if (col < P2) {
            Mc[(int64_t)c * P2pad + col] = acc[qd];
            if (c < ncoarse && M64) M64[(int64_t)c * P2pad + col] = (double)acc[qd];
        }
    }
}

// ------------------------------------------------------------------ M2M
// Parents of one level; thread per (parent, row).  Children are read from
// float64 (src64) when their level is coarse, else from the compute array.
template <class TC, class TI>
__global__ __launch_bounds__(256) void k_m2m(int64_t pstart, int64_t pcount, const int32_t *nch, const int32_t *cbeg,
                                             const uint64_t *key, const TI *src, const TC *W, int P2, int P2pad,
                                             TC *dst, float *dst32)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pc = t / P2;
    const int row = (int)(t % P2);
    if (pc >= pcount) return;
    const int64_t c = pstart + pc;
    TC acc = 0;
    const int nc = nch[c];
    if (nc == 0) return;  // a leaf keeps its P2M multipole
    for (int k = 0; k < nc; ++k) {
        const int64_t ch = cbeg[c] + k;
        const int oct = (int)(key[ch] & 7u);
        const TC *w = W + (int64_t)oct * P2pad * P2pad + row;
        const TI *mc = src + ch * P2pad;
        TC a4[4] = {0, 0, 0, 0};  // independent chains; P2pad is a multiple of 16
        for (int col = 0; col < P2pad; col += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a4[u & 3] += w[(int64_t)(col + u) * P2pad] * (TC)mc[col + u];
        }
        acc += (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    dst[c * P2pad + row] = acc;
    if (dst32) dst32[c * P2pad + row] = (float)acc;
}

// ------------------------------------------------------------------ L2L
// Children of one level; local(child) = M2L(child) + V_oct local(parent).
template <class TC, class TP, class TO>
__global__ __launch_bounds__(256) void k_l2l(int64_t cstart, int64_t ccount, const int32_t *par, const uint64_t *key,
                                             const TP *lpar, const TC *V, int P2, int P2pad, const void *m2l_in,
                                             int m2l_is_double, TO *dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cc = t / P2;
    const int row = (int)(t % P2);
    if (cc >= ccount) return;
    const int64_t c = cstart + cc;
    const int64_t pa = par[c];
    const int oct = (int)(key[c] & 7u);
    const TC *v = V + (int64_t)oct * P2pad * P2pad + row;
    const TP *lp = lpar + pa * P2pad;
    TC acc = m2l_is_double ? (TC) static_cast<const double *>(m2l_in)[c * P2pad + row]
                           : (TC) static_cast<const float *>(m2l_in)[c * P2pad + row];
    TC a4[4] = {0, 0, 0, 0};  // independent chains; P2pad is a multiple of 16
    for (int col = 0; col < P2pad; col += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a4[u & 3] += v[(int64_t)(col + u) * P2pad] * (TC)lp[col + u];
    }
    acc += (a4[0] + a4[1]) + (a4[2] + a4[3]);
    dst[c * P2pad + row] = (TO)acc;
}

template <class TO>
__global__ void k_root_local(const void *m2l_in, int m2l_is_double, int P2, TO *dst)
{
    for (int r = threadIdx.x; r < P2; r += blockDim.x)
        dst[r] = m2l_is_double ? (TO) static_cast<const double *>(m2l_in)[r] : (TO) static_cast<const float *>(m2l_in)[r];
}

// ------------------------------------------------------------------ L2P
// Thread per body: phi += (1/h) sum L conj(R(v)), E -= (1/h^2) grad_v, with
// v = (x - c)/h and the gradient from dR_n^m/dz = R_{n-1}^m,
// dR/dx = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2, dR/dy = -i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2.
template <class T, class V4, class TL>
__device__ __forceinline__ void lget(const TL *L, int p, int n, int m, T &re, T &im)
{
    // complex local coefficient X_n^m (any sign of m), zero out of range
    if (n >= p || m > n || m < -n) { re = 0; im = 0; return; }
    const int am = m < 0 ? -m : m;
    const int r = ridx_re(n, am);
    re = (T)L[r];
    im = am == 0 ? (T)0 : (T)L[r + 1];
    if (m < 0) {
        if (am & 1) { re = -re; }
        else { im = -im; }
    }
}

template <class T, class V4, class TL>
__device__ __forceinline__ void l2p_one(const TL *L, int p, const V4 u, T ih, T &phi, T &ex, T &ey, T &ez)
{
    const T x = u.x * ih, y = u.y * ih, z = u.z * ih;
    const T r2 = x * x + y * y + z * z;
    T f = 0, gx = 0, gy = 0, gz = 0;
    T mre = 1, mim = 0;
    for (int m = 0; m < p; ++m) {
        if (m > 0) {
            const T fct = rec_half<T>(m);
            const T nr = (mre * x - mim * y) * fct;
            const T ni = (mre * y + mim * x) * fct;
            mre = nr;
            mim = ni;
        }
        const T w = m == 0 ? (T)1 : (T)2;
        T p2r = 0, p2i = 0, p1r = mre, p1i = mim;
        for (int n = m; n < p; ++n) {
            T cr, ci;
            if (n == m) { cr = mre; ci = mim; }
            else if (n == m + 1) { cr = z * mre; ci = z * mim; }
            else {
                const T a = (T)(2 * n - 1), inv = rec_inv<T>(n, m);
                cr = (a * z * p1r - r2 * p2r) * inv;
                ci = (a * z * p1i - r2 * p2i) * inv;
            }
            if (n > m) { p2r = p1r; p2i = p1i; }
            p1r = cr;
            p1i = ci;
            // potential
            T lr, li;
            lget<T, V4, TL>(L, p, n, m, lr, li);
            f += w * (lr * cr + li * ci);
            if (n + 1 < p) {
                T am_r, am_i, ap_r, ap_i, a0r, a0i;
                lget<T, V4, TL>(L, p, n + 1, m - 1, am_r, am_i);
                lget<T, V4, TL>(L, p, n + 1, m + 1, ap_r, ap_i);
                lget<T, V4, TL>(L, p, n + 1, m, a0r, a0i);
                // X for x: (L^{m-1} - L^{m+1})/2 ; y: (i/2)(L^{m+1} + L^{m-1}) ; z: L^m
                const T xr = (am_r - ap_r) * (T)0.5, xi = (am_i - ap_i) * (T)0.5;
                const T yr = -(ap_i + am_i) * (T)0.5, yi = (ap_r + am_r) * (T)0.5;
                gx += w * (xr * cr + xi * ci);
                gy += w * (yr * cr + yi * ci);
                gz += w * (a0r * cr + a0i * ci);
            }
        }
    }
    phi = f * ih;
    const T ih2 = ih * ih;
    ex = -gx * ih2;
    ey = -gy * ih2;
    ez = -gz * ih2;
}

template <class T, class V4>
__global__ __launch_bounds__(256) void k_l2p(int64_t n, const int32_t *leaf_of, const int32_t *lvl, const V4 *ub,
                                             double S, int p, int P2pad, const T *Lc, const double *L64,
                                             int64_t ncoarse, T *phi_s, T *E_s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = leaf_of[i];
    const T ih = (T)ldexp(1.0 / S, lvl[c]);
    T ph, ex, ey, ez;
    if (c < ncoarse) l2p_one<T, V4, double>(L64 + (int64_t)c * P2pad, p, ub[i], ih, ph, ex, ey, ez);
    else l2p_one<T, V4, T>(Lc + (int64_t)c * P2pad, p, ub[i], ih, ph, ex, ey, ez);
    phi_s[i] += ph;
    E_s[3 * i] += ex;
    E_s[3 * i + 1] += ey;
    E_s[3 * i + 2] += ez;
}

}  // namespace

// Operator tables depend only on (p, theta, precision); they are generated
// once per device and kept for the life of the process.
namespace {
struct OpCache {
    void *ops = nullptr, *m2m_c = nullptr, *l2l_c = nullptr;
    double *m2m_d = nullptr, *l2l_d = nullptr;
};
std::mutex g_ops_mu;
std::map<std::tuple<int, int, uint64_t, int, int>, OpCache> g_ops;
}  // namespace

void make_operators(fmm_plan *P, hipStream_t s)
{
    const int P2pad = P->P2pad;
    const bool f64 = P->precision == FMM_PREC_FP64;
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    uint64_t bits;
    std::memcpy(&bits, &P->t4, sizeof(bits));
    std::unique_lock<std::mutex> lk(g_ops_mu, std::defer_lock);
    const auto key = std::make_tuple(dev, P->p, bits, f64 ? 1 : 0, P->tight);  // the stencil depends on tight
    // a plan that may not allocate builds its own tables in its own memory
    auto dmalloc = [&](void **ptr, size_t bytes) {
        if (P->noalloc) *ptr = plan_alloc(P, bytes);
        else FMM_HIP(hipMalloc(ptr, bytes));
    };
    std::map<std::tuple<int, int, uint64_t, int, int>, OpCache> own;
    auto it = own.end();
    if (!P->noalloc) {
        lk.lock();
        it = g_ops.find(key);
    }
    if (P->noalloc || it == g_ops.end()) {
        OpCache C;
        const int esz = f64 ? (int)sizeof(double) : (int)sizeof(float);
        const int Q = m2l_q(P->p);
        const size_t opn = (size_t)std::max(1, P->nops) * m2l_opsz(P2pad / 16, Q, esz) + m2l_tail(P2pad / 16, Q, esz);
        std::vector<double4> tr(std::max(1, P->nops));
        for (int k = 0; k < P->nops; ++k)
            tr[k] = make_double4(P->h_ops_t[3 * k], P->h_ops_t[3 * k + 1], P->h_ops_t[3 * k + 2], 0.0);
        double4 *d_ot = nullptr;
        dmalloc((void **)&d_ot, sizeof(double4) * tr.size());
        FMM_HIP(hipMemcpyAsync(d_ot, tr.data(), sizeof(double4) * tr.size(), hipMemcpyHostToDevice, s));
        dmalloc(&C.ops, (f64 ? sizeof(double) : sizeof(float)) * opn);
        FMM_HIP(hipMemsetAsync(C.ops, 0, (f64 ? sizeof(double) : sizeof(float)) * opn, s));
        if (P->nops > 0) {
            if (f64)
                k_make_m2l_ops<double><<<P->nops, 256, 0, s>>>(d_ot, P->nops, P->p, P2pad, m2l_sch(P2pad / 16, Q, 8),
                                                               m2l_gst(P2pad / 16, Q, 8), m2l_opsz(P2pad / 16, Q, 8), 0,
                                                               static_cast<double *>(C.ops));
            else
                k_make_m2l_ops<float><<<P->nops, 256, 0, s>>>(d_ot, P->nops, P->p, P2pad, m2l_sch(P2pad / 16, Q, 4),
                                                              m2l_gst(P2pad / 16, Q, 4), m2l_opsz(P2pad / 16, Q, 4),
                                                              m2l_tail_rows(P->p), static_cast<float *>(C.ops));
            FMM_HIP(hipGetLastError());
        }
        const size_t shn = (size_t)8 * P2pad * P2pad;
        dmalloc((void **)&C.m2m_d, sizeof(double) * shn);
        dmalloc((void **)&C.l2l_d, sizeof(double) * shn);
        k_make_shift_ops<<<8, 256, 0, s>>>(P->p, P2pad, C.m2m_d, C.l2l_d);
        FMM_HIP(hipGetLastError());
        if (f64) {
            C.m2m_c = C.m2m_d;
            C.l2l_c = C.l2l_d;
        } else {
            dmalloc(&C.m2m_c, sizeof(float) * shn);
            dmalloc(&C.l2l_c, sizeof(float) * shn);
            k_d2f<<<grid1(shn, 256), 256, 0, s>>>(C.m2m_d, static_cast<float *>(C.m2m_c), shn);
            k_d2f<<<grid1(shn, 256), 256, 0, s>>>(C.l2l_d, static_cast<float *>(C.l2l_c), shn);
            FMM_HIP(hipGetLastError());
        }
        FMM_HIP(hipStreamSynchronize(s));
        if (P->noalloc) {
            it = own.emplace(key, C).first;  // d_ot stays in the plan's memory
        } else {
            FMM_HIP(hipFree(d_ot));
            it = g_ops.emplace(key, C).first;
        }
    }
    const OpCache &C = it->second;
    P->ops = C.ops;
    P->m2m_c = C.m2m_c;
    P->l2l_c = C.l2l_c;
    P->m2m_d = C.m2m_d;
    P->l2l_d = C.l2l_d;
}

// M2L operators for arbitrary (tau, e) in the batched fragment layout, into
// a caller-provided buffer of nops * P2pad^2 values of the compute type.
void make_m2l_ops(fmm_plan *P, const double4 *tr_dev, int nops, void *out, hipStream_t s)
{
    if (nops <= 0) return;
    const int RT = P->P2pad / 16, Q = m2l_q(P->p);
    if (P->precision == FMM_PREC_FP64)
        k_make_m2l_ops<double><<<nops, 256, 0, s>>>(tr_dev, nops, P->p, P->P2pad, m2l_sch(RT, Q, 8), m2l_gst(RT, Q, 8),
                                                    m2l_opsz(RT, Q, 8), 0, static_cast<double *>(out));
    else
        k_make_m2l_ops<float><<<nops, 256, 0, s>>>(tr_dev, nops, P->p, P->P2pad, m2l_sch(RT, Q, 4), m2l_gst(RT, Q, 4),
                                                   m2l_opsz(RT, Q, 4), m2l_tail_rows(P->p), static_cast<float *>(out));
    FMM_HIP(hipGetLastError());
}

// P2M at every leaf, then M2M from the finest level up.
void upward(fmm_plan *P, const void *ub, hipStream_t s)
{
    const int p = P->p, P2 = P->P2, P2pad = P->P2pad;
    const bool f64 = P->precision == FMM_PREC_FP64;
    if (P->nleaf > 0) {
        const unsigned nb = (unsigned)P->nleaf;
        const size_t esz = f64 ? sizeof(double) : sizeof(float);
        // 32 bodies per chunk (both half-waves on the same bodies) keeps the
        // rows small enough for many resident blocks
        const int chunk = (int)std::min<size_t>(32, (60 * 1024) / ((P2 + 1) * esz));
        const size_t smem = (size_t)chunk * (P2 + 1) * esz;
        if (f64)
            k_p2m<double, double4><<<nb, 64, smem, s>>>(P->leaves, P->c_beg, P->c_end, P->c_lvl,
                                                        static_cast<const double4 *>(ub), P->S, p, P2pad, chunk,
                                                        static_cast<double *>(P->Mc), nullptr, 0);
        else
            k_p2m<float, float4><<<nb, 64, smem, s>>>(P->leaves, P->c_beg, P->c_end, P->c_lvl,
                                                      static_cast<const float4 *>(ub), P->S, p, P2pad, chunk,
                                                      static_cast<float *>(P->Mc), P->M64, P->ncoarse);
        FMM_HIP(hipGetLastError());
    }
    const int cfl = f64 ? P->depth + 1 : std::min(P->cfl, P->depth + 1);
    for (int l = P->depth - 1; l >= 0; --l) {
        const int64_t cnt = P->lv[l].count, st = P->lv[l].start;
        const int64_t nt = cnt * P2;
        if (cnt == 0) continue;
        if (f64) {
            k_m2m<double, double><<<grid1(nt, 256), 256, 0, s>>>(st, cnt, P->c_nch, P->c_cbeg, P->c_key,
                                                                 static_cast<const double *>(P->Mc), P->m2m_d, P2,
                                                                 P2pad, static_cast<double *>(P->Mc), nullptr);
        } else if (l < cfl) {
            // coarse parent: float64 translation; children coarse or not
            if (l + 1 < cfl)
                k_m2m<double, double><<<grid1(nt, 256), 256, 0, s>>>(st, cnt, P->c_nch, P->c_cbeg, P->c_key, P->M64,
                                                                     P->m2m_d, P2, P2pad, P->M64,
                                                                     static_cast<float *>(P->Mc));
            else
                k_m2m<double, float><<<grid1(nt, 256), 256, 0, s>>>(st, cnt, P->c_nch, P->c_cbeg, P->c_key,
                                                                    static_cast<const float *>(P->Mc), P->m2m_d, P2,
                                                                    P2pad, P->M64, static_cast<float *>(P->Mc));
        } else {
            k_m2m<float, float><<<grid1(nt, 256), 256, 0, s>>>(st, cnt, P->c_nch, P->c_cbeg, P->c_key,
                                                               static_cast<const float *>(P->Mc),
                                                               static_cast<const float *>(P->m2m_c), P2, P2pad,
                                                               static_cast<float *>(P->Mc), nullptr);
        }
        FMM_HIP(hipGetLastError());
    }
}

// L2L from the root down; the M2L results sit in Lc and become the totals.
void downward_l2l(fmm_plan *P, hipStream_t s)
{
    const int P2 = P->P2, P2pad = P->P2pad;
    const bool f64 = P->precision == FMM_PREC_FP64;
    const int cfl = f64 ? P->depth + 1 : std::min(P->cfl, P->depth + 1);
    if (f64) {
        // root total = its M2L sum, already in place
    } else if (cfl > 0) {
        k_root_local<double><<<1, 256, 0, s>>>(P->Lc, 0, P2, P->L64);
        FMM_HIP(hipGetLastError());
    }
    for (int l = 1; l <= P->depth; ++l) {
        const int64_t cnt = P->lv[l].count, st = P->lv[l].start;
        const int64_t nt = cnt * P2;
        if (cnt == 0) continue;
        if (f64) {
            k_l2l<double, double, double><<<grid1(nt, 256), 256, 0, s>>>(
                st, cnt, P->c_par, P->c_key, static_cast<const double *>(P->Lc), P->l2l_d, P2, P2pad, P->Lc, 1,
                static_cast<double *>(P->Lc));
        } else if (l - 1 < cfl) {
            if (l < cfl)
                k_l2l<double, double, double><<<grid1(nt, 256), 256, 0, s>>>(st, cnt, P->c_par, P->c_key, P->L64,
                                                                             P->l2l_d, P2, P2pad, P->Lc, 0, P->L64);
            else
                k_l2l<double, double, float><<<grid1(nt, 256), 256, 0, s>>>(st, cnt, P->c_par, P->c_key, P->L64,
                                                                            P->l2l_d, P2, P2pad, P->Lc, 0,
                                                                            static_cast<float *>(P->Lc));
        } else {
            k_l2l<float, float, float><<<grid1(nt, 256), 256, 0, s>>>(
                st, cnt, P->c_par, P->c_key, static_cast<const float *>(P->Lc), static_cast<const float *>(P->l2l_c),
                P2, P2pad, P->Lc, 0, static_cast<float *>(P->Lc));
        }
        FMM_HIP(hipGetLastError());
    }
}

void l2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    const int64_t n = P->n;
    if (P->precision == FMM_PREC_FP64)
        k_l2p<double, double4><<<grid1(n, 256), 256, 0, s>>>(n, P->leaf_of, P->c_lvl, static_cast<const double4 *>(ub),
                                                              P->S, P->p, P->P2pad, static_cast<const double *>(P->Lc),
                                                              static_cast<const double *>(P->Lc), P->ncoarse,
                                                              static_cast<double *>(phi_s), static_cast<double *>(E_s));
    else
        k_l2p<float, float4><<<grid1(n, 256), 256, 0, s>>>(n, P->leaf_of, P->c_lvl, static_cast<const float4 *>(ub),
                                                            P->S, P->p, P->P2pad, static_cast<const float *>(P->Lc),
                                                            P->L64, P->ncoarse, static_cast<float *>(phi_s),
                                                            static_cast<float *>(E_s));
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
