// rotation.hip -- M2L by rotation, O(p^3) per pair: the O(P^3) end of the
// range that Section III.A gives for the operators' cost with the basis.
// Every M2L pair of a plan (the pair list with all same-level rows moved to
// it) runs here when fmm_params.m2l_rotation is set.
#include "internal.hpp"

#include <cmath>
#include <vector>

namespace fmm {

namespace {

struct cd {
    double re, im;
};

constexpr int kOutSlots = (kMaxP * (kMaxP + 1) / 2 + 63) / 64;

// M2L by rotation, O(p^3) per pair (the O(P^3) end of the operator cost range
// of Section III.A): the frame is turned so that the offset lies on +z, the
// expansion is translated along z, where only order 0 of the irregular
// harmonics survives, and turned back.  With s_m = sqrt((n+m)!(n-m)!),
// t and f the polar and azimuth angles of tau = (c_A - c_B) / h_A and d its
// length:
//     Mt_m  = sum_k d^n_{k m}(t) e^{i k f} (s_k / s_m) M_k
//     Lt_j^s = (-1)^j sum_{n >= |s|} Mt_n^{-s} (n + j)! / d^{n+j+1}
//     L_k  += sum_s d^j_{k s}(t) e^{i k f} (s_k / s_s) Lt_s.
// d^n(t) is applied through the fixed table X^n = d^n(pi/2):
//     d^n_{a b}(t) = i^{a-b} sum_k X_{k a} X_{k b} e^{-i k t},
// two products with X and a diagonal per rotation.  One block per target
// cell; its four waves take every fourth pair of the cell's list (each wave
// with its own LDS vectors, coefficients complex at n^2 + n + m), all in
// float64; the waves' sums are added in wave order and then to the local
// expansion, so the result does not depend on timing.
constexpr int kRotWaves = 4;

__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// The lanes of one wave exchange data through LDS: wavefront-scope release
// and acquire around the wave barrier order the writes before the reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// i^{-m}
__device__ __forceinline__ cd ipow_neg(int m)
{
    switch (m & 3) {
    case 0: return cd{1.0, 0.0};
    case 1: return cd{0.0, -1.0};
    case 2: return cd{-1.0, 0.0};
    default: return cd{0.0, 1.0};
    }
}

template <class TM>
__global__ __launch_bounds__(64 * kRotWaves) void k_m2l_rot(const int64_t *off, const int32_t *src, int64_t nc,
                                                            const int32_t *lvl, const double *ctr, double S, int p,
                                                            int P2pad, const TM *M, const double *xtab, TM *Lout)
{
    const int c = blockIdx.x;
    if (c >= nc || off[c] == off[c + 1]) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int P2 = p * p, XN = p * (2 * p - 1) * (2 * p + 1) / 3, NO = p * (p + 1) / 2;
    extern __shared__ double X[];  // XN values (dynamic)
    __shared__ double fct[2 * kMaxP], sfc[kMaxP * kMaxP];
    __shared__ double G[kRotWaves][2 * kMaxP];
    __shared__ cd ET[kRotWaves][2 * kMaxP], EF[kRotWaves][2 * kMaxP];  // e^{-i k t}, e^{i k (f + pi/2)}, k + p - 1
    __shared__ cd V1[kRotWaves][kMaxP * kMaxP], V2[kRotWaves][kMaxP * kMaxP];
    for (int e = tid; e < XN; e += 64 * kRotWaves) X[e] = xtab[e];
    if (tid < 2 * kMaxP) {
        double f = 1.0;
        for (int k = 2; k <= tid; ++k) f *= k;
        fct[tid] = f;
    }
    __syncthreads();
    for (int r = tid; r < P2; r += 64 * kRotWaves) {  // s_m = sqrt((n+m)!(n-m)!)
        const int n = (int)sqrtf((float)r + 0.5f), m = r - n * n - n;
        sfc[r] = sqrt(fct[n + m] * fct[n - m]);
    }
    __syncthreads();
    auto xo = [](int n) { return n * (2 * n - 1) * (2 * n + 1) / 3; };  // X^n's first element
    const double hA = ldexp(S, -lvl[c]);
    cd *v1 = V1[wv], *v2 = V2[wv], *et = ET[wv], *ef = EF[wv];
    double *g = G[wv];
    double are[kOutSlots] = {}, aim[kOutSlots] = {};
    // Each wave walks its own pairs and its own LDS vectors: between the steps
    // of a pair only the wave's lanes exchange data, whose LDS accesses run in
    // order, so a wave barrier (no block barrier) separates them.
    for (int64_t q = off[c] + wv; q < off[c + 1]; q += kRotWaves) {
        const int b = src[q];
        const int dl = lvl[c] - lvl[b];
        {
            // e^{i t} = (tz + i rho) / d and e^{i f} = (tx + i ty) / rho come from
            // the offset itself; lane k raises them to the k-th power by squaring
            const double tx = (ctr[3 * c] - ctr[3 * b]) / hA, ty = (ctr[3 * c + 1] - ctr[3 * b + 1]) / hA,
                         tz = (ctr[3 * c + 2] - ctr[3 * b + 2]) / hA;
            const double rho = sqrt(tx * tx + ty * ty), d = sqrt(rho * rho + tz * tz), id = 1.0 / d;
            if (lane < p) {
                cd a = {1.0, 0.0}, e = {1.0, 0.0}, ba = {tz * id, -rho * id};  // e^{-i t}
                cd be = rho > 0.0 ? cd{-ty / rho, tx / rho} : cd{0.0, 1.0};    // i e^{i f}
                for (int k = lane; k; k >>= 1) {
                    if (k & 1) {
                        a = cmul(a, ba);
                        e = cmul(e, be);
                    }
                    ba = cmul(ba, ba);
                    be = cmul(be, be);
                }
                et[p - 1 + lane] = a;
                et[p - 1 - lane] = cd{a.re, -a.im};
                ef[p - 1 + lane] = e;
                ef[p - 1 - lane] = cd{e.re, -e.im};
            }
            if (lane < 2 * p - 1) {  // k! / d^{k+1}
                double pw = id, bb = id;
                for (int k = lane; k; k >>= 1) {
                    if (k & 1) pw *= bb;
                    bb *= bb;
                }
                g[lane] = fct[lane] * pw;
            }
        }
        wave_sync();
        const TM *mb = M + (int64_t)b * P2pad;
        for (int r = lane; r < P2; r += 64) {  // v1 = i^k e^{i k f} s_k M_k (source scaled to the target's level)
            const int n = (int)sqrtf((float)r + 0.5f), m = r - n * n - n, am = m < 0 ? -m : m;
            const double sc = ldexp(1.0, n * dl);
            double re = sc * (double)mb[n * n + (am ? 2 * am - 1 : 0)], im = am ? sc * (double)mb[n * n + 2 * am] : 0.0;
            if (m < 0) {  // M_n^{-m} = (-1)^m conj(M_n^m)
                im = -im;
                if (am & 1) { re = -re; im = -im; }
            }
            const cd z = cmul(cd{re, im}, ef[m + p - 1]);
            v1[r] = cd{sfc[r] * z.re, sfc[r] * z.im};
        }
        wave_sync();
        for (int r = lane; r < P2; r += 64) {  // v2_k = e^{-i k t} sum_m X_{k m} v1_m
            const int n = (int)sqrtf((float)r + 0.5f), k = r - n * n - n, w = 2 * n + 1;
            const double *xr = X + xo(n) + (k + n) * w;
            const cd *vv = v1 + n * n;
            double sr = 0.0, si = 0.0;
            for (int m = 0; m < w; ++m) {
                sr += xr[m] * vv[m].re;
                si += xr[m] * vv[m].im;
            }
            v2[r] = cmul(cd{sr, si}, et[k + p - 1]);
        }
        wave_sync();
        for (int r = lane; r < P2; r += 64) {  // v1_m = Mt_m = i^{-m} / s_m sum_k X_{k m} v2_k
            const int n = (int)sqrtf((float)r + 0.5f), m = r - n * n - n, w = 2 * n + 1;
            const double *xc = X + xo(n) + (m + n);
            const cd *vv = v2 + n * n;
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < w; ++k) {
                sr += xc[k * w] * vv[k].re;
                si += xc[k * w] * vv[k].im;
            }
            const cd z = cmul(cd{sr, si}, ipow_neg(m));
            const double is = 1.0 / sfc[r];
            v1[r] = cd{is * z.re, is * z.im};
        }
        wave_sync();
        // v2_s = i^{-s} / s_s Lt_j^s, Lt_j^s = (-1)^j sum_{n >= |s|} Mt_n^{-s} (n + j)! / d^{n+j+1}
        for (int r = lane; r < P2; r += 64) {
            const int j = (int)sqrtf((float)r + 0.5f), sO = r - j * j - j, as = sO < 0 ? -sO : sO;
            double sr = 0.0, si = 0.0;
            for (int n = as; n < p; ++n) {
                const cd mv = v1[n * n + n - sO];
                sr += mv.re * g[n + j];
                si += mv.im * g[n + j];
            }
            const double sg = ((j & 1) ? -1.0 : 1.0) / sfc[r];
            const cd z = cmul(cd{sr, si}, ipow_neg(sO));
            v2[r] = cd{sg * z.re, sg * z.im};
        }
        wave_sync();
        for (int r = lane; r < P2; r += 64) {  // v1_k = e^{-i k t} sum_s X_{k s} v2_s
            const int n = (int)sqrtf((float)r + 0.5f), k = r - n * n - n, w = 2 * n + 1;
            const double *xr = X + xo(n) + (k + n) * w;
            const cd *vv = v2 + n * n;
            double sr = 0.0, si = 0.0;
            for (int m = 0; m < w; ++m) {
                sr += xr[m] * vv[m].re;
                si += xr[m] * vv[m].im;
            }
            v1[r] = cmul(cd{sr, si}, et[k + p - 1]);
        }
        wave_sync();
        for (int qq = 0; qq < kOutSlots; ++qq) {  // L_k += e^{i k (f + pi/2)} s_k sum_u X_{u k} v1_u, k >= 0
            const int e = lane + 64 * qq;
            if (e >= NO) continue;
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int k = e - j * (j + 1) / 2, w = 2 * j + 1;
            const double *xc = X + xo(j) + (k + j);
            const cd *vv = v1 + j * j;
            double sr = 0.0, si = 0.0;
            for (int u = 0; u < w; ++u) {
                sr += xc[u * w] * vv[u].re;
                si += xc[u * w] * vv[u].im;
            }
            const cd z = cmul(cd{sr, si}, ef[k + p - 1]);
            const double sc = sfc[j * j + j + k];
            are[qq] += sc * z.re;
            aim[qq] += sc * z.im;
        }
        wave_sync();
    }
    __syncthreads();
    // the waves' sums, in wave order
    for (int qq = 0; qq < kOutSlots; ++qq) {
        const int e = lane + 64 * qq;
        if (e < NO) V1[wv][e] = cd{are[qq], aim[qq]};
    }
    __syncthreads();
    if (wv == 0) {
        TM *dst = Lout + (int64_t)c * P2pad;
        for (int qq = 0; qq < kOutSlots; ++qq) {
            const int e = lane + 64 * qq;
            if (e >= NO) continue;
            double sr = 0.0, si = 0.0;
            for (int w = 0; w < kRotWaves; ++w) {
                sr += V1[w][e].re;
                si += V1[w][e].im;
            }
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int k = e - j * (j + 1) / 2;
            if (k == 0) dst[j * j] = (TM)((double)dst[j * j] + sr);
            else {
                dst[j * j + 2 * k - 1] = (TM)((double)dst[j * j + 2 * k - 1] + sr);
                dst[j * j + 2 * k] = (TM)((double)dst[j * j + 2 * k] + si);
            }
        }
    }
}

}  // namespace

// X^n = d^n(pi/2) for n < p, each (2n + 1)^2 row-major (rows m', columns m,
// -n..n), from d^n(b) = exp(b A) with A = -i J_y of spin n:
// A_{m+1, m} = -sqrt(n(n+1) - m(m+1)) / 2, A_{m-1, m} = +sqrt(n(n+1) - m(m-1)) / 2;
// the exponential by scaling and squaring of its Taylor series.
static std::vector<double> rotation_table(int p)
{
    std::vector<double> out;
    for (int n = 0; n < p; ++n) {
        const int w = 2 * n + 1;
        std::vector<double> A(w * w, 0.0), E(w * w, 0.0), T(w * w, 0.0), U(w * w);
        for (int m = -n; m <= n; ++m) {
            if (m + 1 <= n) A[(m + 1 + n) * w + (m + n)] = -0.5 * std::sqrt((double)(n * (n + 1) - m * (m + 1)));
            if (m - 1 >= -n) A[(m - 1 + n) * w + (m + n)] = 0.5 * std::sqrt((double)(n * (n + 1) - m * (m - 1)));
        }
        double norm = 0.0;
        for (int r = 0; r < w; ++r) {
            double row = 0.0;
            for (int c = 0; c < w; ++c) row += std::fabs(A[r * w + c]);
            norm = std::max(norm, row);
        }
        int sq = 0;
        double sc = 0.5 * M_PI;
        while (sc * norm > 0.25) { sc *= 0.5; ++sq; }
        for (int e = 0; e < w * w; ++e) A[e] *= sc;
        for (int r = 0; r < w; ++r) E[r * w + r] = T[r * w + r] = 1.0;
        for (int k = 1; k <= 24; ++k) {  // T <- T A / k, E += T
            for (int r = 0; r < w; ++r)
                for (int c = 0; c < w; ++c) {
                    double acc = 0.0;
                    for (int u = 0; u < w; ++u) acc += T[r * w + u] * A[u * w + c];
                    U[r * w + c] = acc / k;
                }
            T.swap(U);
            for (int e = 0; e < w * w; ++e) E[e] += T[e];
        }
        for (int q = 0; q < sq; ++q) {
            for (int r = 0; r < w; ++r)
                for (int c = 0; c < w; ++c) {
                    double acc = 0.0;
                    for (int u = 0; u < w; ++u) acc += E[r * w + u] * E[u * w + c];
                    U[r * w + c] = acc;
                }
            E.swap(U);
        }
        out.insert(out.end(), E.begin(), E.end());
    }
    return out;
}

void rotation_prepare(fmm_plan *P, hipStream_t s)
{
    const std::vector<double> xt = rotation_table(P->p);
    P->rot_x = static_cast<double *>(plan_alloc(P, sizeof(double) * xt.size()));
    FMM_HIP(hipMemcpyAsync(P->rot_x, xt.data(), sizeof(double) * xt.size(), hipMemcpyHostToDevice, s));
    FMM_HIP(hipStreamSynchronize(s));
}

// One block of kRotWaves waves per cell; cells without pairs return at once.
void rotation_m2l(fmm_plan *P, hipStream_t s)
{
    if (P->n_gx == 0) return;
    FMM_CHECK(P->ncell < (1ll << 31), FMM_ERR_UNSUPPORTED, "m2l: too many cells");
    const size_t lds = sizeof(double) * P->p * (2 * P->p - 1) * (2 * P->p + 1) / 3;
    if (P->precision == FMM_PREC_FP64)
        k_m2l_rot<double><<<(unsigned)P->ncell, 64 * kRotWaves, lds, s>>>(
            P->gx_off, P->gx_src, P->ncell, P->c_lvl, P->c_ctr, P->S, P->p, P->P2pad,
            static_cast<const double *>(P->Mc), P->rot_x, static_cast<double *>(P->Lc));
    else
        k_m2l_rot<float><<<(unsigned)P->ncell, 64 * kRotWaves, lds, s>>>(
            P->gx_off, P->gx_src, P->ncell, P->c_lvl, P->c_ctr, P->S, P->p, P->P2pad,
            static_cast<const float *>(P->Mc), P->rot_x, static_cast<float *>(P->Lc));
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
