// sort.hip -- device-wide exclusive scan and stable LSD radix sort (gfx950).
//
// The tree build sorts 64-bit Morton keys with their body index (Section
// II.B: building the hashed octree is analogous to a radix sort over the key
// bits, three bits per level).  The sort is stable, so equal keys keep the
// input order and the permutation is deterministic.
#include "internal.hpp"

namespace fmm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

// Inclusive scan of one int64 value per thread across a 256-thread block.
// Returns the inclusive prefix; *total receives the block sum.
__device__ __forceinline__ int64_t block_scan_incl(int64_t v, int64_t *total)
{
    __shared__ int64_t s_w[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) s_w[w] = v;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < w) off += s_w[k];
        tot += s_w[k];
    }
    __syncthreads();
    *total = tot;
    return v + off;
}

template <class Tin>
__global__ __launch_bounds__(kScanThreads) void k_block_sums(const Tin *in, int64_t n, int64_t *sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += (int64_t)in[base + k];
    int64_t tot;
    block_scan_incl(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of one tile plus a per-block offset: offs[blockIdx.x] when
// offs is given, else the sum of sums[0, blockIdx.x) when sums is given (each
// block adds up its predecessors' totals itself), else 0.
template <class Tin>
__global__ __launch_bounds__(kScanThreads) void k_block_scan(const Tin *in, int64_t *out, int64_t n,
                                                             const int64_t *offs, const int64_t *sums,
                                                             int64_t *total)
{
    int64_t boff = 0;
    if (offs) {
        boff = offs[blockIdx.x];
    } else if (sums) {
        int64_t part = 0;
        for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x; j += kScanThreads) part += sums[j];
        block_scan_incl(part, &boff);
    }
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? (int64_t)in[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t incl = block_scan_incl(s, &tot);
    int64_t run = incl - s + boff;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (total && threadIdx.x == kScanThreads - 1 && blockIdx.x == gridDim.x - 1) *total = run;
}

// Up to this many tiles, the blocks of the final pass find their offsets from
// the raw tile sums (two launches in all); beyond it the tile sums are
// scanned first.
constexpr int64_t kSelfOffsetTiles = 2048;

template <class Tin>
void scan_impl(const Tin *in, int64_t *out, int64_t n, int64_t *total_dev, Allocator &al, hipStream_t s)
{
    if (n <= 0) {
        if (total_dev) FMM_HIP(hipMemsetAsync(total_dev, 0, sizeof(int64_t), s));
        return;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_block_scan<Tin><<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, nullptr, total_dev);
        FMM_HIP(hipGetLastError());
        return;
    }
    int64_t *sums = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * 2 * nb));
    int64_t *soff = sums + nb;
    k_block_sums<Tin><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, sums);
    FMM_HIP(hipGetLastError());
    if (nb <= kSelfOffsetTiles) {
        k_block_scan<Tin><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, nullptr, sums, total_dev);
    } else {
        scan_impl<int64_t>(sums, soff, nb, nullptr, al, s);
        // the last block's running sum after its tile is the grand total
        k_block_scan<Tin><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, soff, nullptr, total_dev);
    }
    FMM_HIP(hipGetLastError());
    al.free(sums);
}

// ------------------------------------------------------------ radix sort
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 16;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;  // 4096 keys per block
static_assert(kRadixThreads == kScanThreads, "the scatter uses the block scan");

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint64_t *kin, int64_t n, int shift,
                                                              int32_t *hist, int64_t nb)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixRounds; ++r) {
        int64_t i = t0 + r * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((kin[i] >> shift) & 255u)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Per digit d (one block each): exclusive scan of hist[d][0, nb), the counts
// of digit d in the tiles in order, and the digit's total.
__global__ __launch_bounds__(kScanThreads) void k_radix_rowscan(const int32_t *hist, int64_t nb, int64_t *rowoff,
                                                                int64_t *rowtot)
{
    const int32_t *h = hist + (int64_t)blockIdx.x * nb;
    int64_t *o = rowoff + (int64_t)blockIdx.x * nb;
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < nb; t0 += kScanTile) {
        const int64_t base = t0 + (int64_t)threadIdx.x * kScanItems;
        int64_t v[kScanItems];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < nb ? (int64_t)h[base + k] : 0;
            sum += v[k];
        }
        int64_t tot;
        int64_t run = block_scan_incl(sum, &tot) - sum + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < nb) o[base + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Stable scatter: element order inside a tile is (round, wave, lane); ranks of
// equal digits inside a wave come from ballots on the 8 digit bits.
template <bool kVals>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint64_t *kin, const int32_t *vin,
                                                                 uint64_t *kout, int32_t *vout, int64_t n,
                                                                 int shift, const int64_t *rowoff,
                                                                 const int64_t *rowtot, int64_t nb)
{
    __shared__ int64_t s_base[256];
    __shared__ int32_t s_wcnt[kRadixThreads / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
    {
        // start of digit tid: the totals of the smaller digits, then the
        // counts of digit tid in the tiles before this one
        const int64_t dt = rowtot[tid];
        int64_t all;
        s_base[tid] = block_scan_incl(dt, &all) - dt + rowoff[(int64_t)tid * nb + blockIdx.x];
    }
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < kRadixRounds; ++r) {
#pragma unroll
        for (int w = 0; w < kRadixThreads / 64; ++w) s_wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = t0 + r * kRadixThreads + tid;
        const bool valid = i < n;
        uint64_t k = 0;
        int32_t v = 0;
        int d = 0;
        if (valid) {
            k = kin[i];
            if (kVals) v = vin[i];
            d = (int)((k >> shift) & 255u);
        }
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(valid && bit);
            m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & lt);
        if (valid && rank == 0) s_wcnt[wave][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int64_t pos = s_base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += s_wcnt[w][d];
            kout[pos] = k;
            if (kVals) vout[pos] = v;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < kRadixThreads / 64; ++w) add += s_wcnt[w][tid];
        s_base[tid] += add;
        __syncthreads();
    }
}

}  // namespace

void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, Allocator &al, hipStream_t s)
{
    scan_impl<int64_t>(in, out, n, total_dev, al, s);
}

void scan_exclusive_i32to64(const int32_t *in, int64_t *out, int64_t n, int64_t *total_dev, Allocator &al,
                            hipStream_t s)
{
    scan_impl<int32_t>(in, out, n, total_dev, al, s);
}

void radix_sort_u64(uint64_t *keys, int32_t *vals, int64_t n, int bits, Allocator &al, hipStream_t s, int lo_bit,
                    uint64_t **sorted)
{
    if (sorted) *sorted = keys;
    if (n <= 1 || bits <= lo_bit) return;
    const int npass = (bits - lo_bit + 7) / 8;
    const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
    FMM_CHECK(nb < (1ll << 31), FMM_ERR_UNSUPPORTED, "radix sort: too many keys");
    uint64_t *k2 = static_cast<uint64_t *>(al.alloc(sizeof(uint64_t) * n));
    int32_t *v2 = vals ? static_cast<int32_t *>(al.alloc(sizeof(int32_t) * n)) : nullptr;
    int32_t *hist = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * 256 * nb));
    int64_t *offs = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * (256 * nb + 256)));
    int64_t *dtot = offs + 256 * nb;
    uint64_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    for (int ps = 0; ps < npass; ++ps) {
        const int shift = lo_bit + 8 * ps;
        k_radix_hist<<<(unsigned)nb, kRadixThreads, 0, s>>>(ka, n, shift, hist, nb);
        FMM_HIP(hipGetLastError());
        k_radix_rowscan<<<256, kScanThreads, 0, s>>>(hist, nb, offs, dtot);
        FMM_HIP(hipGetLastError());
        if (vals)
            k_radix_scatter<true><<<(unsigned)nb, kRadixThreads, 0, s>>>(ka, va, kb, vb, n, shift, offs, dtot, nb);
        else
            k_radix_scatter<false><<<(unsigned)nb, kRadixThreads, 0, s>>>(ka, nullptr, kb, nullptr, n, shift, offs,
                                                                          dtot, nb);
        FMM_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    bool keep_k2 = false;
    if (ka != keys) {
        if (sorted && !vals) {
            *sorted = ka;  // the caller takes the scratch buffer instead of a copy
            keep_k2 = true;
        } else {
            FMM_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
            if (vals) FMM_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        }
    }
    al.free(offs);
    al.free(hist);
    if (v2) al.free(v2);
    if (!keep_k2) al.free(k2);
}

}  // namespace fmm
