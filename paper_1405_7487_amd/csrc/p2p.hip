// p2p.hip -- particle-to-particle near field on gfx950 (Section II.A: P2P
// between the leaves that the dual traversal did not accept for M2L).
//
// One wave per target leaf.  Source bodies of the leaf's P2P list are staged
// in LDS in batches of up to 256, shifted into the target leaf's frame
// (offsets from leaf centers keep float32 differences exact to ~1e-7 of the
// leaf size at any depth).  When the leaf holds few bodies, G lanes share a
// target and split the batch; a butterfly of wave shuffles sums them.  Batch
// partial sums enter the running totals through a compensated (Kahan) add.
#include "internal.hpp"

namespace fmm {

namespace {

constexpr int kStage = 256;

template <class T> __device__ __forceinline__ T rsqrt_t(T x);
template <> __device__ __forceinline__ float rsqrt_t<float>(float x) { return __frsqrt_rn(x); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

template <class T>
__device__ __forceinline__ void kahan_add(T &sum, T &comp, T v)
{
    const T y = v - comp;
    const T t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

template <class T, class V4, bool KAHAN>
__global__ __launch_bounds__(64) void k_p2p(const int32_t *leaves, const int32_t *beg, const int32_t *end,
                                            const int64_t *off, const int32_t *src, const double *ctr, const V4 *ub,
                                            T *phi_s, T *E_s)
{
    __shared__ V4 sb[kStage];
    const int lane = threadIdx.x;
    const int A = leaves[blockIdx.x];
    const int32_t tb = beg[A], te = end[A];
    const int nt = te - tb;
    const double cax = ctr[3 * A], cay = ctr[3 * A + 1], caz = ctr[3 * A + 2];
    const int64_t k0 = off[A], k1 = off[A + 1];
    for (int base = 0; base < nt; base += 64) {
        const int cnt = min(64, nt - base);
        int G = 1;
        while (G < 16 && 2 * G * cnt <= 64) G *= 2;
        const int ti = lane / G, sub = lane % G;
        const bool active = ti < cnt;
        V4 u = ub[tb + base + (active ? ti : 0)];
        T s_p = 0, s_x = 0, s_y = 0, s_z = 0, c_p = 0, c_x = 0, c_y = 0, c_z = 0;
        int64_t k = k0;
        int32_t o = 0;
        while (k < k1) {
            int staged = 0;
            while (staged < kStage && k < k1) {
                const int b = src[k];
                const int32_t bb = beg[b] + o, be = end[b];
                const int take = min(min(be - bb, kStage - staged), 64);
                if (lane < take) {
                    V4 v = ub[bb + lane];
                    v.x += (T)(ctr[3 * b] - cax);
                    v.y += (T)(ctr[3 * b + 1] - cay);
                    v.z += (T)(ctr[3 * b + 2] - caz);
                    sb[staged + lane] = v;
                }
                staged += take;
                o += take;
                if (bb + take == be) { ++k; o = 0; }
            }
            __syncthreads();
            T p_p = 0, p_x = 0, p_y = 0, p_z = 0;
            if (active) {
                for (int jj = sub; jj < staged; jj += G) {
                    const V4 v = sb[jj];
                    const T dx = u.x - v.x, dy = u.y - v.y, dz = u.z - v.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    const T ri = r2 > (T)0 ? rsqrt_t<T>(r2) : (T)0;
                    const T qr = v.w * ri;
                    const T qr3 = qr * ri * ri;
                    p_p += qr;
                    p_x += qr3 * dx;
                    p_y += qr3 * dy;
                    p_z += qr3 * dz;
                }
            }
            if (KAHAN) {
                kahan_add(s_p, c_p, p_p);
                kahan_add(s_x, c_x, p_x);
                kahan_add(s_y, c_y, p_y);
                kahan_add(s_z, c_z, p_z);
            } else {
                s_p += p_p; s_x += p_x; s_y += p_y; s_z += p_z;
            }
            __syncthreads();
        }
        if (KAHAN) {
            s_p -= c_p; s_x -= c_x; s_y -= c_y; s_z -= c_z;
        }
        for (int w = G >> 1; w >= 1; w >>= 1) {
            s_p += __shfl_xor(s_p, w, 64);
            s_x += __shfl_xor(s_x, w, 64);
            s_y += __shfl_xor(s_y, w, 64);
            s_z += __shfl_xor(s_z, w, 64);
        }
        if (active && sub == 0) {
            const int64_t i = tb + base + ti;
            phi_s[i] = s_p;
            E_s[3 * i] = s_x;
            E_s[3 * i + 1] = s_y;
            E_s[3 * i + 2] = s_z;
        }
    }
}

}  // namespace

void p2p(fmm_plan *P, const void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    if (P->nleaf == 0) return;
    const unsigned nb = (unsigned)P->nleaf;
    if (P->precision == FMM_PREC_FP64)
        k_p2p<double, double4, false><<<nb, 64, 0, s>>>(P->leaves, P->c_beg, P->c_end, P->p2p_off, P->p2p_src,
                                                        P->c_ctr, static_cast<const double4 *>(ub),
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

}  // namespace fmm
