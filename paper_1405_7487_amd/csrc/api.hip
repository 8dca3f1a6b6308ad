// api.hip -- C ABI of the gfx950 FMM library (declared in include/fmm.h).
//
// A plan holds the tree, the lists, the operator tables and every buffer an
// evaluation needs, so fmm_evaluate_plan and fmm_adjoint allocate nothing
// after their first call.  Device memory comes from the caller's allocator
// callbacks or from a process-wide caching pool (per device) that hands back
// freed blocks only after the stream that used them was synchronised.
#include "internal.hpp"

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <unordered_map>
#include <unordered_set>

namespace fmm {

namespace {

thread_local std::string g_err;

// Set by fmm_evaluate_noalloc around its fmm_build: the plan then takes every
// device buffer from this range instead of allocating.
struct ArenaRange {
    char *base;
    size_t cap;
};
thread_local ArenaRange fmm_plan_arena_ = {nullptr, 0};

// ------------------------------------------------------------ caching pool
struct Pool {
    std::mutex mu;
    std::multimap<size_t, void *> freel;
    std::unordered_map<void *, size_t> sizes;
};
Pool g_pool[64];

size_t pool_round(size_t b)
{
    if (b < 256) return 256;
    size_t hi = 1;
    while (hi * 2 <= b) hi *= 2;
    const size_t gran = std::max<size_t>(256, hi / 4);
    return (b + gran - 1) / gran * gran;
}

void *pool_get(size_t bytes)
{
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    Pool &P = g_pool[dev & 63];
    const size_t r = pool_round(bytes);
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.freel.lower_bound(r);
        if (it != P.freel.end() && it->first <= 2 * r) {
            void *p = it->second;
            P.freel.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, r) != hipSuccess) {
        (void)hipGetLastError();
        // give cached blocks back to the runtime and retry once
        std::lock_guard<std::mutex> lk(P.mu);
        for (auto &kv : P.freel) {
            (void)hipFree(kv.second);
            P.sizes.erase(kv.second);
        }
        P.freel.clear();
        if (hipMalloc(&p, r) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(P.mu);
    P.sizes[p] = r;
    return p;
}

void pool_put(void *p)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Pool &P = g_pool[dev & 63];
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.sizes.find(p);
    if (it == P.sizes.end()) return;
    P.freel.insert({it->second, p});
}

}  // namespace

// Allocator: every live allocation is tracked so that a failed build can
// release everything; pool blocks freed mid-build are parked until the next
// stream synchronisation.
struct AllocState {
    std::unordered_set<void *> live;
    std::vector<void *> parked;
};
static std::mutex g_as_mu;
static std::unordered_map<const Allocator *, AllocState> g_as;

static AllocState &state_of(const Allocator *a)
{
    std::lock_guard<std::mutex> lk(g_as_mu);
    return g_as[a];
}

void *Allocator::alloc(size_t bytes)
{
    if (bytes == 0) bytes = 1;
    if (arena) {
        const size_t need = (bytes + 255) / 256 * 256;
        if (arena_free.empty() && arena_used.empty()) arena_free[0] = arena_cap;
        for (auto it = arena_free.begin(); it != arena_free.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, left = it->second - need;
            arena_free.erase(it);
            if (left) arena_free[off + need] = left;
            arena_used[off] = need;
            arena_peak = std::max(arena_peak, off + need);
            return arena + off;
        }
        size_t used = 0;
        for (auto &kv : arena_used) used += kv.second;
        throw Error(FMM_ERR_NOMEM, "the static scratch of " + std::to_string(arena_cap >> 20) +
                                       " MiB is exhausted (" + std::to_string(used) + " bytes in use, " +
                                       std::to_string(need) + " more asked for)");
    }
    void *p = has_user ? user.alloc(bytes, (void *)stream, user.ctx) : pool_get(bytes);
    if (!p) throw Error(FMM_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    state_of(this).live.insert(p);
    return p;
}

void Allocator::free(void *p)
{
    if (!p) return;
    if (arena) {
        const size_t off = (size_t)(static_cast<char *>(p) - arena);
        auto u = arena_used.find(off);
        if (u == arena_used.end()) return;
        size_t start = off, len = u->second;
        arena_used.erase(u);
        auto nx = arena_free.lower_bound(start);
        if (nx != arena_free.end() && nx->first == start + len) {  // merge with the next free range
            len += nx->second;
            nx = arena_free.erase(nx);
        }
        if (nx != arena_free.begin()) {  // and with the previous one
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                arena_free.erase(pv);
            }
        }
        arena_free[start] = len;
        return;
    }
    AllocState &st = state_of(this);
    st.live.erase(p);
    if (has_user) user.free(p, (void *)stream, user.ctx);
    else st.parked.push_back(p);
}

static void allocator_flush(Allocator &a)
{
    if (a.arena) return;
    AllocState &st = state_of(&a);
    for (void *p : st.parked) pool_put(p);
    st.parked.clear();
}

static void allocator_release_all(Allocator &a)
{
    if (a.arena) {
        a.arena_used.clear();
        a.arena_free.clear();  // the whole range is free again
        return;
    }
    AllocState &st = state_of(&a);
    for (void *p : st.live) {
        if (a.has_user) a.user.free(p, (void *)a.stream, a.user.ctx);
        else pool_put(p);
    }
    st.live.clear();
    allocator_flush(a);
    std::lock_guard<std::mutex> lk(g_as_mu);
    g_as.erase(&a);
}

void *plan_alloc(fmm_plan *P, size_t bytes)
{
    void *p = P->al.alloc(bytes);
    P->bytes_held += (int64_t)bytes;
    return p;
}

// ------------------------------------------------------------ small kernels
namespace {

template <class TQ, class V4>
__global__ __launch_bounds__(256) void k_set_charge(const TQ *q, const int32_t *perm, int64_t n, V4 *ub)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ub[i].w = (decltype(ub[i].w))q[perm[i]];
}

template <class V4>
__global__ __launch_bounds__(256) void k_copy_xyz(const V4 *a, V4 *b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <class TC, class TO>
__global__ __launch_bounds__(256) void k_unpermute(const TC *phi_s, const TC *E_s, const int32_t *perm, int64_t n,
                                                   TO *phi, TO *field)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    phi[o] = (TO)phi_s[i];
    if (field) {
        field[3 * o] = (TO)E_s[3 * i];
        field[3 * o + 1] = (TO)E_s[3 * i + 1];
        field[3 * o + 2] = (TO)E_s[3 * i + 2];
    }
}

// dq = psi (potential of w), dx = -(w E^q + q E^w), all scattered to the
// caller's order.
template <class TC, class TO>
__global__ __launch_bounds__(256) void k_adjoint_out(const TC *psi_s, const TC *Ew_s, const TC *Eq_s, const TO *Eq_user,
                                                     const TO *q, const TO *w, const int32_t *perm, int64_t n, TO *dq,
                                                     TO *dx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    if (dq) dq[o] = (TO)psi_s[i];
    if (dx) {
        const double wo = (double)w[o], qo = (double)q[o];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double eq = Eq_user ? (double)Eq_user[3 * o + d] : (double)Eq_s[3 * i + d];
            dx[3 * o + d] = (TO)(-(wo * eq + qo * (double)Ew_s[3 * i + d]));
        }
    }
}

// ------------------------------------------------------------ timing
enum Phase { PH_P2M, PH_M2L, PH_L2L, PH_P2P, PH_L2P, PH_EVAL, PH_ADJ, PH_M2LX, PH_N };

struct Events {
    hipEvent_t a[PH_N], b[PH_N];
    bool used[PH_N];
};
std::mutex g_ev_mu;
std::unordered_map<const fmm_plan *, Events> g_ev;

void ev_rec(fmm_plan *P, int ph, bool start, hipStream_t s)
{
    if (!P->timing) return;
    std::lock_guard<std::mutex> lk(g_ev_mu);
    auto it = g_ev.find(P);
    if (it == g_ev.end()) {
        Events e{};
        for (int k = 0; k < PH_N; ++k) {
            FMM_HIP(hipEventCreate(&e.a[k]));
            FMM_HIP(hipEventCreate(&e.b[k]));
        }
        it = g_ev.emplace(P, e).first;
    }
    FMM_HIP(hipEventRecord(start ? it->second.a[ph] : it->second.b[ph], s));
    if (!start) it->second.used[ph] = true;
}

template <class V4>
void set_charge(fmm_plan *P, const void *q, void *ub, hipStream_t s)
{
    const int64_t n = P->n;
    if (P->dtype == FMM_F64)
        k_set_charge<double, V4><<<grid1(n, 256), 256, 0, s>>>(static_cast<const double *>(q), P->perm, n,
                                                                static_cast<V4 *>(ub));
    else
        k_set_charge<float, V4><<<grid1(n, 256), 256, 0, s>>>(static_cast<const float *>(q), P->perm, n,
                                                               static_cast<V4 *>(ub));
    FMM_HIP(hipGetLastError());
}

void pipeline(fmm_plan *P, const void *q, void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    eval_up(P, q, ub, s);
    eval_m2l(P, s);
    eval_down(P, ub, phi_s, E_s, s);
}

fmm_status fail(const Error &e)
{
    g_err = e.what();
    return e.code;
}

// Runs the body of an entry point and maps every exception to a status, so
// that none crosses the C ABI: the library's own errors keep their code, a
// failed host allocation is FMM_ERR_NOMEM, anything else FMM_ERR_DEVICE.
template <class F>
fmm_status guarded(F &&body)
{
    try {
        return body();
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return FMM_ERR_NOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return FMM_ERR_DEVICE;
    } catch (...) {
        g_err = "unknown exception";
        return FMM_ERR_DEVICE;
    }
}

void destroy_plan(fmm_plan *P)
{
    if (!P) return;
    (void)hipStreamSynchronize(P->al.stream);
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        auto it = g_ev.find(P);
        if (it != g_ev.end()) {
            for (int k = 0; k < PH_N; ++k) {
                (void)hipEventDestroy(it->second.a[k]);
                (void)hipEventDestroy(it->second.b[k]);
            }
            g_ev.erase(it);
        }
    }
    allocator_release_all(P->al);
    delete P;
}

void validate_params(const fmm_params &p)
{
    FMM_CHECK(p.p >= 1 && p.p <= kMaxP, FMM_ERR_INVALID, "p must be in [1, 16]");
    FMM_CHECK(p.theta > 0.0 && p.theta < 1.0, FMM_ERR_INVALID, "theta must be in (0, 1)");
    FMM_CHECK(p.ncrit >= 1, FMM_ERR_INVALID, "ncrit must be >= 1");
    FMM_CHECK(p.precision == FMM_PREC_FP64 || p.precision == FMM_PREC_MIXED, FMM_ERR_INVALID, "bad precision");
    FMM_CHECK(p.coarse_fp64_levels >= 0 && p.coarse_fp64_levels <= kLevels + 1, FMM_ERR_INVALID,
              "coarse_fp64_levels must be in [0, 22]");
    FMM_CHECK(p.m2l_sparse >= -1 && p.m2l_sparse <= 64, FMM_ERR_INVALID, "m2l_sparse must be in [-1, 64]");
    FMM_CHECK(p.m2l_rotation == 0 || p.m2l_rotation == 1, FMM_ERR_INVALID, "m2l_rotation must be 0 or 1");
    FMM_CHECK(p.mutual == 0 || p.mutual == 1, FMM_ERR_INVALID, "mutual must be 0 or 1");
}

// ------------------------------------------------------------ no-alloc scratch
// Device memory of fmm_evaluate_noalloc: one array per GPU, resident from the
// library's load until the process ends.  In host code the array's name only
// stands for the symbol; kernels and copies use the per-device address that
// hipGetSymbolAddress returns.
constexpr size_t kScratchBytes = FMM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

struct ScratchSlot {
    std::mutex mu;   // calls on one device run one after another
    char *ptr = nullptr;
};
ScratchSlot g_scratch[64];
std::mutex g_scratch_mu;

// The scratch of the current device (looked up once per device).
ScratchSlot &scratch_slot()
{
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    FMM_CHECK(dev >= 0 && dev < 64, FMM_ERR_UNSUPPORTED, "device index beyond 63");
    ScratchSlot &sl = g_scratch[dev];
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!sl.ptr) {
        void *ptr = nullptr;
        FMM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        FMM_CHECK(ptr != nullptr, FMM_ERR_DEVICE, "no address for the scratch array");
        sl.ptr = static_cast<char *>(ptr);
    }
    return sl;
}

}  // namespace

// The evaluation in three phases (the order of Section II.C): charges into
// the sorted bodies and the upward pass; M2L over the traversal's lists (the
// local expansions start from zero here); the downward pass with P2P and L2P.
void eval_up(fmm_plan *P, const void *q, void *ub, hipStream_t s)
{
    if (P->precision == FMM_PREC_FP64) set_charge<double4>(P, q, ub, s);
    else set_charge<float4>(P, q, ub, s);
    ev_rec(P, PH_P2M, true, s);
    upward(P, ub, s);
    ev_rec(P, PH_P2M, false, s);
}

void eval_m2l(fmm_plan *P, hipStream_t s)
{
    ev_rec(P, PH_M2L, true, s);
    m2l_same(P, s);
    ev_rec(P, PH_M2L, false, s);
    ev_rec(P, PH_M2LX, true, s);
    m2l_cross(P, s);
    ev_rec(P, PH_M2LX, false, s);
}

void eval_down(fmm_plan *P, void *ub, void *phi_s, void *E_s, hipStream_t s)
{
    ev_rec(P, PH_L2L, true, s);
    downward_l2l(P, s);
    ev_rec(P, PH_L2L, false, s);
    ev_rec(P, PH_P2P, true, s);
    p2p(P, ub, phi_s, E_s, s);
    ev_rec(P, PH_P2P, false, s);
    ev_rec(P, PH_L2P, true, s);
    l2p(P, ub, phi_s, E_s, s);
    ev_rec(P, PH_L2P, false, s);
}

void allocator_done(Allocator &a) { allocator_release_all(a); }

void mfma_probe(int f64, void *out_host);

}  // namespace fmm

using namespace fmm;

extern "C" {

void fmm_params_default(fmm_params *prm)
{
    if (!prm) return;
    prm->p = 8;
    prm->theta = 0.4;
    prm->ncrit = 64;
    prm->precision = FMM_PREC_MIXED;
    prm->coarse_fp64_levels = 3;
    prm->kahan = 1;
    prm->tight = 0;
    prm->m2l_sparse = -1;
    prm->m2l_rotation = 0;
    prm->mutual = 0;
}

const char *fmm_last_error(void) { return g_err.c_str(); }

fmm_status fmm_build(const void *x, fmm_dtype dtype, int64_t n, const fmm_params *prm, const fmm_allocator *alloc,
                     void *hip_stream, fmm_plan **out)
{
    g_err.clear();
    fmm_plan *P = nullptr;
    try {
        FMM_CHECK(out != nullptr, FMM_ERR_INVALID, "out is NULL");
        *out = nullptr;
        FMM_CHECK(n >= 0, FMM_ERR_INVALID, "n < 0");
        FMM_CHECK(n == 0 || x != nullptr, FMM_ERR_INVALID, "x is NULL");
        FMM_CHECK(dtype == FMM_F64 || dtype == FMM_F32, FMM_ERR_INVALID, "bad dtype");
        FMM_CHECK(n < (1ll << 31), FMM_ERR_UNSUPPORTED, "n >= 2^31");
        fmm_params pr;
        fmm_params_default(&pr);
        if (prm) pr = *prm;
        validate_params(pr);
        FMM_CHECK(!alloc || (alloc->alloc && alloc->free), FMM_ERR_INVALID, "allocator without callbacks");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        P = new fmm_plan();
        P->n = n;
        P->p = pr.p;
        P->P2 = pr.p * pr.p;
        P->P2pad = p2pad_of(pr.p);
        P->theta = pr.theta;
        P->t4 = 4.0 * pr.theta * pr.theta;
        P->ncrit = pr.ncrit;
        P->precision = pr.precision;
        P->TW = m2l_tile_width(pr.p, pr.precision == FMM_PREC_FP64);
        P->cfl = pr.coarse_fp64_levels;
        P->kahan = pr.kahan ? 1 : 0;
        P->tight = pr.tight ? 1 : 0;
        P->m2l_sparse = pr.m2l_sparse;
        P->m2l_rotation = pr.m2l_rotation;
        P->mutual = pr.mutual;
        P->dtype = dtype;
        P->al.stream = s;
        if (fmm_plan_arena_.base) {
            P->al.arena = fmm_plan_arena_.base;
            P->al.arena_cap = fmm_plan_arena_.cap;
            P->noalloc = true;
        } else if (alloc) {
            P->al.user = *alloc;
            P->al.has_user = true;
        }
        P->st.n = n;
        P->st.p = pr.p;
        if (n == 0) {
            *out = P;
            return FMM_OK;
        }
        auto t0 = std::chrono::steady_clock::now();
        auto ms_since = [](std::chrono::steady_clock::time_point a) {
            return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
        };
        tree_build(P, x, s);
        FMM_HIP(hipStreamSynchronize(s));
        allocator_flush(P->al);
        P->st.ms_tree = ms_since(t0);
        auto t1a = std::chrono::steady_clock::now();
        traverse(P, s);
        FMM_HIP(hipStreamSynchronize(s));
        allocator_flush(P->al);
        P->st.ms_traverse = ms_since(t1a);
        auto t2a = std::chrono::steady_clock::now();
        make_operators(P, s);
        m2l_prepare(P, s);
        m2l_cross_prepare(P, s);
        p2p_prepare(P, s);
        FMM_HIP(hipStreamSynchronize(s));
        P->st.ms_ops = ms_since(t2a);
        if (P->d_m2l_rows) {
            unsigned long long rows = 0;
            FMM_HIP(hipMemcpyAsync(&rows, P->d_m2l_rows, sizeof(rows), hipMemcpyDeviceToHost, s));
            FMM_HIP(hipStreamSynchronize(s));
            P->m2l_rows = (int64_t)rows;
        }
        const bool f64 = P->precision == FMM_PREC_FP64;
        const size_t esz = f64 ? sizeof(double) : sizeof(float);
        const size_t ncoef = (size_t)(P->ncell + 1) * P->P2pad;  // + one all-zero row
        P->Mc = plan_alloc(P, esz * ncoef);
        P->Lc = plan_alloc(P, esz * ncoef);
        if (f64) {
            P->M64 = static_cast<double *>(P->Mc);
            P->L64 = static_cast<double *>(P->Lc);
        } else if (P->ncoarse > 0) {
            P->M64 = static_cast<double *>(plan_alloc(P, sizeof(double) * P->ncoarse * P->P2pad));
            P->L64 = static_cast<double *>(plan_alloc(P, sizeof(double) * P->ncoarse * P->P2pad));
        }
        // padded coefficient slots stay zero forever
        FMM_HIP(hipMemsetAsync(P->Mc, 0, esz * ncoef, s));
        if (!f64 && P->M64) FMM_HIP(hipMemsetAsync(P->M64, 0, sizeof(double) * P->ncoarse * P->P2pad, s));
        if (!f64 && P->L64) FMM_HIP(hipMemsetAsync(P->L64, 0, sizeof(double) * P->ncoarse * P->P2pad, s));
        FMM_HIP(hipMemsetAsync(P->Lc, 0, esz * ncoef, s));
        P->phi_s = plan_alloc(P, esz * n);
        P->E_s = plan_alloc(P, esz * 3 * n);
        FMM_HIP(hipStreamSynchronize(s));
        allocator_flush(P->al);
        auto t1 = std::chrono::steady_clock::now();
        P->st.ms_build = std::chrono::duration<double, std::milli>(t1 - t0).count();
        *out = P;
        return FMM_OK;
    } catch (const Error &e) {
        if (P) destroy_plan(P);
        return fail(e);
    } catch (const std::bad_alloc &) {
        if (P) destroy_plan(P);
        g_err = "host allocation failed";
        return FMM_ERR_NOMEM;
    } catch (const std::exception &e) {
        if (P) destroy_plan(P);
        g_err = e.what();
        return FMM_ERR_DEVICE;
    } catch (...) {
        if (P) destroy_plan(P);
        g_err = "unknown exception";
        return FMM_ERR_DEVICE;
    }
}

fmm_status fmm_evaluate_plan(fmm_plan *P, const void *q, void *phi, void *field, void *hip_stream)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(P != nullptr, FMM_ERR_INVALID, "plan is NULL");
        if (P->n == 0) return FMM_OK;
        FMM_CHECK(q && phi, FMM_ERR_INVALID, "q or phi is NULL");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        P->al.stream = s;
        ev_rec(P, PH_EVAL, true, s);
        pipeline(P, q, P->ubody, P->phi_s, P->E_s, s);
        const int64_t n = P->n;
        if (P->precision == FMM_PREC_FP64) {
            if (P->dtype == FMM_F64)
                k_unpermute<double, double><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const double *>(P->phi_s), static_cast<const double *>(P->E_s), P->perm, n,
                    static_cast<double *>(phi), static_cast<double *>(field));
            else
                k_unpermute<double, float><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const double *>(P->phi_s), static_cast<const double *>(P->E_s), P->perm, n,
                    static_cast<float *>(phi), static_cast<float *>(field));
        } else {
            if (P->dtype == FMM_F64)
                k_unpermute<float, double><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const float *>(P->phi_s), static_cast<const float *>(P->E_s), P->perm, n,
                    static_cast<double *>(phi), static_cast<double *>(field));
            else
                k_unpermute<float, float><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const float *>(P->phi_s), static_cast<const float *>(P->E_s), P->perm, n,
                    static_cast<float *>(phi), static_cast<float *>(field));
        }
        FMM_HIP(hipGetLastError());
        ev_rec(P, PH_EVAL, false, s);
        return FMM_OK;
    });
}

fmm_status fmm_evaluate(const void *x, const void *q, fmm_dtype dtype, int64_t n, int32_t p, double theta,
                        int32_t ncrit, int32_t precision, const fmm_allocator *alloc, void *phi, void *field,
                        void *hip_stream)
{
    fmm_params pr;
    fmm_params_default(&pr);
    pr.p = p;
    pr.theta = theta;
    pr.ncrit = ncrit;
    pr.precision = precision;
    if (n > 0 && (!q || !phi)) {
        g_err = "q or phi is NULL";
        return FMM_ERR_INVALID;
    }
    fmm_plan *P = nullptr;
    fmm_status st = fmm_build(x, dtype, n, &pr, alloc, hip_stream, &P);
    if (st != FMM_OK) return st;
    st = fmm_evaluate_plan(P, q, phi, field, hip_stream);
    fmm_destroy(P);
    return st;
}

fmm_status fmm_evaluate_noalloc(const void *x, const void *q, fmm_dtype dtype, int64_t n, int32_t p, double theta,
                                int32_t ncrit, int32_t precision, void *phi, void *field, void *hip_stream)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(n >= 0, FMM_ERR_INVALID, "n < 0");
        if (n == 0) return FMM_OK;
        FMM_CHECK(x && q && phi, FMM_ERR_INVALID, "x, q or phi is NULL");
        FMM_CHECK(n <= FMM_NOALLOC_MAX_N, FMM_ERR_UNSUPPORTED,
                  "fmm_evaluate_noalloc: n = " + std::to_string(n) + " exceeds its limit of " +
                      std::to_string((long long)FMM_NOALLOC_MAX_N) + " bodies");
        ScratchSlot &sl = scratch_slot();
        std::lock_guard<std::mutex> lk(sl.mu);
        fmm_plan_arena_ = {sl.ptr, kScratchBytes};
        fmm_params pr;
        fmm_params_default(&pr);
        pr.p = p;
        pr.theta = theta;
        pr.ncrit = ncrit;
        pr.precision = precision;
        fmm_plan *P = nullptr;
        fmm_status st = fmm_build(x, dtype, n, &pr, nullptr, hip_stream, &P);
        fmm_plan_arena_ = {nullptr, 0};
        if (st != FMM_OK) return st;
        st = fmm_evaluate_plan(P, q, phi, field, hip_stream);
        const std::string err = g_err;
        fmm_destroy(P);  // synchronises the stream: the scratch is free again
        g_err = err;
        return st;
    });
}

fmm_status fmm_let_evaluate(const void *x, const void *q, fmm_dtype dtype, int64_t n, int32_t nrank,
                            const int64_t *weights, const fmm_params *prm, const fmm_allocator *alloc, void *phi,
                            void *field, int32_t *rank, int64_t *work_local, int64_t *work_remote,
                            int64_t *pair_stats, fmm_let_stats *stats, void *hip_stream)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(n >= 0, FMM_ERR_INVALID, "n < 0");
        FMM_CHECK(nrank >= 1 && nrank <= 1024, FMM_ERR_INVALID, "nrank must be in [1, 1024]");
        FMM_CHECK(dtype == FMM_F64 || dtype == FMM_F32, FMM_ERR_INVALID, "bad dtype");
        FMM_CHECK(n < (1ll << 31), FMM_ERR_UNSUPPORTED, "n >= 2^31");
        FMM_CHECK(!alloc || (alloc->alloc && alloc->free), FMM_ERR_INVALID, "allocator without callbacks");
        fmm_params pr;
        fmm_params_default(&pr);
        if (prm) pr = *prm;
        validate_params(pr);
        if (stats) *stats = fmm_let_stats{};
        if (n == 0) return FMM_OK;
        FMM_CHECK(x && q && phi, FMM_ERR_INVALID, "x, q or phi is NULL");
        let_evaluate(x, q, dtype, n, nrank, weights, pr, alloc, phi, field, rank, work_local, work_remote,
                     pair_stats, stats, static_cast<hipStream_t>(hip_stream));
        return FMM_OK;
    });
}

fmm_status fmm_adjoint(fmm_plan *P, const void *q, const void *grad_phi, const void *field_q, void *dq, void *dx,
                       void *hip_stream)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(P != nullptr, FMM_ERR_INVALID, "plan is NULL");
        if (P->n == 0) return FMM_OK;
        FMM_CHECK(q && grad_phi, FMM_ERR_INVALID, "q or grad_phi is NULL");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        P->al.stream = s;
        const int64_t n = P->n;
        const bool f64 = P->precision == FMM_PREC_FP64;
        const size_t esz = f64 ? sizeof(double) : sizeof(float);
        if (!P->ubody2) {
            P->ubody2 = plan_alloc(P, (f64 ? sizeof(double4) : sizeof(float4)) * n);
            P->phi_s2 = plan_alloc(P, esz * n);
            P->E_s2 = plan_alloc(P, esz * 3 * n);
            if (f64) k_copy_xyz<double4><<<grid1(n, 256), 256, 0, s>>>(static_cast<const double4 *>(P->ubody),
                                                                       static_cast<double4 *>(P->ubody2), n);
            else k_copy_xyz<float4><<<grid1(n, 256), 256, 0, s>>>(static_cast<const float4 *>(P->ubody),
                                                                   static_cast<float4 *>(P->ubody2), n);
            FMM_HIP(hipGetLastError());
        }
        ev_rec(P, PH_ADJ, true, s);
        // second pass with w as the charges (symmetric lists: exact transpose)
        pipeline(P, grad_phi, P->ubody2, P->phi_s2, P->E_s2, s);
        if (!field_q) pipeline(P, q, P->ubody, P->phi_s, P->E_s, s);
        if (f64) {
            if (P->dtype == FMM_F64)
                k_adjoint_out<double, double><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const double *>(P->phi_s2), static_cast<const double *>(P->E_s2),
                    static_cast<const double *>(P->E_s), static_cast<const double *>(field_q),
                    static_cast<const double *>(q), static_cast<const double *>(grad_phi), P->perm, n,
                    static_cast<double *>(dq), static_cast<double *>(dx));
            else
                k_adjoint_out<double, float><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const double *>(P->phi_s2), static_cast<const double *>(P->E_s2),
                    static_cast<const double *>(P->E_s), static_cast<const float *>(field_q),
                    static_cast<const float *>(q), static_cast<const float *>(grad_phi), P->perm, n,
                    static_cast<float *>(dq), static_cast<float *>(dx));
        } else {
            if (P->dtype == FMM_F64)
                k_adjoint_out<float, double><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const float *>(P->phi_s2), static_cast<const float *>(P->E_s2),
                    static_cast<const float *>(P->E_s), static_cast<const double *>(field_q),
                    static_cast<const double *>(q), static_cast<const double *>(grad_phi), P->perm, n,
                    static_cast<double *>(dq), static_cast<double *>(dx));
            else
                k_adjoint_out<float, float><<<grid1(n, 256), 256, 0, s>>>(
                    static_cast<const float *>(P->phi_s2), static_cast<const float *>(P->E_s2),
                    static_cast<const float *>(P->E_s), static_cast<const float *>(field_q),
                    static_cast<const float *>(q), static_cast<const float *>(grad_phi), P->perm, n,
                    static_cast<float *>(dq), static_cast<float *>(dx));
        }
        FMM_HIP(hipGetLastError());
        ev_rec(P, PH_ADJ, false, s);
        return FMM_OK;
    });
}

fmm_status fmm_set_timing(fmm_plan *P, int32_t on)
{
    if (!P) return FMM_ERR_INVALID;
    P->timing = on ? 1 : 0;
    return FMM_OK;
}

fmm_status fmm_plan_stats(const fmm_plan *Pc, fmm_stats *out)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(Pc && out, FMM_ERR_INVALID, "NULL argument");
        fmm_plan *P = const_cast<fmm_plan *>(Pc);
        fmm_stats st = P->st;
        st.n = P->n;
        st.ncell = P->ncell;
        st.nleaf = P->nleaf;
        st.depth = P->depth;
        st.p = P->p;
        st.n_m2l_same = P->n_m2l_same;
        st.n_m2l_cross = P->n_m2l_cross;
        st.n_m2l = P->n_m2l_same + P->n_m2l_cross;
        st.n_p2p = P->n_p2p;
        st.p2p_body_pairs = P->n > 0 ? P->p2p_body_pairs : 0;  // -1 until counted
        st.m2l_stencil = P->K;
        st.m2l_offsets = P->nops;
        st.m2l_slots = P->ntile * (int64_t)P->K * P->TW;
        st.m2l_cross_keys = P->nxk;
        st.m2l_cross_batched = P->nxb;
        st.p2p_cut_leaves = P->p2p_ncut;
        st.n_m2l_sparse = P->n_m2l_sparse;
        st.p2p_mutual_pairs = P->mu_nup;
        st.m2l_rows = P->m2l_rows;
        st.device_bytes = P->bytes_held;
        {
            std::lock_guard<std::mutex> lk(g_ev_mu);
            auto it = g_ev.find(P);
            if (it != g_ev.end()) {
                double *dst[PH_N] = {&st.ms_p2m, &st.ms_m2l, &st.ms_l2l, &st.ms_p2p, &st.ms_l2p, &st.ms_evaluate,
                                     &st.ms_adjoint, &st.ms_m2l_cross};
                for (int k = 0; k < PH_N; ++k) {
                    if (!it->second.used[k]) continue;
                    float ms = 0.f;
                    if (hipEventSynchronize(it->second.b[k]) == hipSuccess &&
                        hipEventElapsedTime(&ms, it->second.a[k], it->second.b[k]) == hipSuccess)
                        *dst[k] = ms;
                }
            }
        }
        *out = st;
        return FMM_OK;
    });
}

fmm_status fmm_list_digest(const fmm_plan *Pc, uint64_t *out)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(Pc && out, FMM_ERR_INVALID, "NULL argument");
        fmm_plan *P = const_cast<fmm_plan *>(Pc);
        uint64_t h[2] = {0, 0};
        list_digest(P, h, P->al.stream);
        out[0] = h[0];
        out[1] = h[1];
        return FMM_OK;
    });
}

fmm_status fmm_count_body_pairs(const fmm_plan *Pc, int64_t *out)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(Pc && out, FMM_ERR_INVALID, "NULL argument");
        fmm_plan *P = const_cast<fmm_plan *>(Pc);
        *out = P->n > 0 ? p2p_body_pairs(P, P->al.stream) : 0;
        return FMM_OK;
    });
}

fmm_status fmm_export_tree(const fmm_plan *Pc, const fmm_tree_export *o)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(Pc && o, FMM_ERR_INVALID, "NULL argument");
        fmm_plan *P = const_cast<fmm_plan *>(Pc);
        FMM_HIP(hipStreamSynchronize(P->al.stream));
        const int64_t n = P->n, nc = P->ncell;
        if (n == 0) return FMM_OK;
        auto cp = [&](void *dst, const void *src, size_t bytes) {
            if (dst && bytes) FMM_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        };
        cp(o->keys, P->keys, sizeof(uint64_t) * n);
        cp(o->perm, P->perm, sizeof(int32_t) * n);
        cp(o->level, P->c_lvl, sizeof(int32_t) * nc);
        cp(o->cell_key, P->c_key, sizeof(uint64_t) * nc);
        cp(o->begin, P->c_beg, sizeof(int32_t) * nc);
        cp(o->end, P->c_end, sizeof(int32_t) * nc);
        cp(o->parent, P->c_par, sizeof(int32_t) * nc);
        cp(o->child_begin, P->c_cbeg, sizeof(int32_t) * nc);
        cp(o->nchild, P->c_nch, sizeof(int32_t) * nc);
        cp(o->centers, P->c_ctr, sizeof(double) * 3 * nc);
        auto csr_pairs = [&](const int64_t *off_d, const int32_t *src_d, int64_t np, std::vector<uint64_t> &outv) {
            std::vector<int64_t> off(nc + 1);
            std::vector<int32_t> src(std::max<int64_t>(1, np));
            FMM_HIP(hipMemcpy(off.data(), off_d, sizeof(int64_t) * (nc + 1), hipMemcpyDeviceToHost));
            if (np) FMM_HIP(hipMemcpy(src.data(), src_d, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
            for (int64_t c = 0; c < nc; ++c)
                for (int64_t k = off[c]; k < off[c + 1]; ++k) outv.push_back(((uint64_t)c << 32) | (uint32_t)src[k]);
        };
        if (o->p2p) {
            std::vector<uint64_t> v;
            csr_pairs(P->p2p_off, P->p2p_src, P->n_p2p, v);
            std::sort(v.begin(), v.end());  // canonical (target, source) order
            for (size_t k = 0; k < v.size(); ++k) {
                o->p2p[2 * k] = (int32_t)(v[k] >> 32);
                o->p2p[2 * k + 1] = (int32_t)(v[k] & 0xffffffffu);
            }
        }
        if (o->m2l) {
            std::vector<uint64_t> v;
            csr_pairs(P->m2lx_off, P->m2lx_src, P->n_m2lx, v);
            const int64_t ns = P->ntile * (int64_t)P->K * P->TW;
            if (ns > 0) {
                std::vector<int32_t> sl(ns), tg(P->ntile * P->TW);
                FMM_HIP(hipMemcpy(sl.data(), P->slots, sizeof(int32_t) * ns, hipMemcpyDeviceToHost));
                FMM_HIP(hipMemcpy(tg.data(), P->tile_tgt, sizeof(int32_t) * tg.size(), hipMemcpyDeviceToHost));
                for (int64_t t = 0; t < P->ntile; ++t)
                    for (int64_t k = 0; k < P->K; ++k)
                        for (int l = 0; l < P->TW; ++l) {
                            const int32_t sv = sl[(t * P->K + k) * P->TW + l];
                            if (sv >= 0) v.push_back(((uint64_t)(uint32_t)tg[t * P->TW + l] << 32) | (uint32_t)sv);
                        }
            }
            std::sort(v.begin(), v.end());
            for (size_t k = 0; k < v.size(); ++k) {
                o->m2l[2 * k] = (int32_t)(v[k] >> 32);
                o->m2l[2 * k + 1] = (int32_t)(v[k] & 0xffffffffu);
            }
        }
        return FMM_OK;
    });
}

void fmm_destroy(fmm_plan *P)
{
    try {
        destroy_plan(P);
    } catch (...) {
        g_err = "fmm_destroy: release failed";
    }
}

/* Diagnostic: runs one 16x16x4 MFMA (f64 != 0: float64, else float32) with
 * A[i][k] = i + 1 + 100 k, B[0][j] = 1 + 1000 j, B[k>0][j] = 0, and copies the
 * 64 x 4 accumulator values (lane-major) to out_host. */
fmm_status fmm_debug_mfma_layout(int32_t f64, void *out_host)
{
    g_err.clear();
    return guarded([&]() -> fmm_status {
        FMM_CHECK(out_host != nullptr, FMM_ERR_INVALID, "out is NULL");
        FMM_CHECK(f64 >= 0 && f64 <= 2, FMM_ERR_INVALID, "f64 must be 0, 1 or 2");
        mfma_probe(f64, out_host);
        return FMM_OK;
    });
}

}  // extern "C"
