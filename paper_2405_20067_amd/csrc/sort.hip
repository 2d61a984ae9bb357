// Stable LSD radix sort of (key, value) pairs, digits of up to 10 bits.
//
// The key bits are split into the fewest passes of at most kRadixMaxBits
// (18 bits: two passes of 9).  Per pass: each block counts the digits of
// its 4096 keys (a histogram in LDS), one exclusive scan turns the
// digit-major counts into output offsets, and each block scatters its keys
// in order: every wave ranks its 64 keys among equal digits with ballots (a
// match mask built from the digit's bits, popcount of the lower lanes), so
// equal keys keep their input order.
// The element count may live on the device (n_dev) with the host giving an
// upper bound: blocks past the count only write zero histogram columns.
#include <utility>

#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

// ---- stable LSD radix sort ----------------------------------------------
constexpr int kThreads = 256;
constexpr int kRadixMaxBits = 10;
constexpr int kRadixItems = 16;                        // per lane
constexpr int kRadixPerWave = kRadixItems * kWave;     // 1024
static_assert(kRadixPerWave * (kThreads / kWave) == kRadixPerBlock, "block size");
static_assert((1 << kRadixMaxBits) == kRadixMaxBins, "bins");

// Element count: the host bound, or the device count when one is given.
__device__ __forceinline__ int64_t count_of(int64_t n_max, const int64_t *n_dev)
{
    if (!n_dev) return n_max;
    const int64_t n = *n_dev;
    return n < n_max ? n : n_max;
}

__global__ __launch_bounds__(kThreads) void k_radix_count(int64_t n_max, const int64_t *n_dev,
                                                          int shift, int width,
                                                          const uint32_t *__restrict__ keys,
                                                          int32_t *__restrict__ hist,
                                                          int64_t nblocks)
{
    __shared__ int cnt[kRadixMaxBins];
    const int64_t n = count_of(n_max, n_dev);
    const int bins = 1 << width;
    const uint32_t mask = uint32_t(bins - 1);
    if (int64_t(blockIdx.x) * kRadixPerBlock >= n) {
        // past the device count: zero columns only
        for (int b = threadIdx.x; b < bins; b += kThreads)
            hist[int64_t(b) * nblocks + blockIdx.x] = 0;
        return;
    }
    for (int b = threadIdx.x; b < bins; b += kThreads) cnt[b] = 0;
    __syncthreads();
    // every key of the thread loaded first, all in flight together
    constexpr int kPerThread = kRadixPerBlock / kThreads;
    const int64_t base = int64_t(blockIdx.x) * kRadixPerBlock + threadIdx.x;
    uint32_t kk[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const int64_t i = base + int64_t(u) * kThreads;
        kk[u] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kPerThread; ++u)
        if (base + int64_t(u) * kThreads < n) atomicAdd(&cnt[(kk[u] >> shift) & mask], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += kThreads)
        hist[int64_t(b) * nblocks + blockIdx.x] = cnt[b];
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    int64_t n_max, const int64_t *n_dev, int shift, int width,
    const uint32_t *__restrict__ keys_in,
    const int32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out, const int64_t *__restrict__ off, int64_t nblocks)
{
    constexpr int W = kThreads / kWave;
    __shared__ int wcnt[W][kRadixMaxBins];
    __shared__ int wbase[W][kRadixMaxBins];
    const int64_t n = count_of(n_max, n_dev);
    // a block past the device count has no keys to move (its histogram
    // columns are zero): nothing to do
    if (int64_t(blockIdx.x) * kRadixPerBlock >= n) return;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int bins = 1 << width;
    const uint32_t mask = uint32_t(bins - 1);
    for (int b = threadIdx.x; b < bins; b += kThreads) {
#pragma unroll
        for (int i = 0; i < W; ++i) wcnt[i][b] = 0;
    }
    __syncthreads();
    const int64_t wstart = int64_t(blockIdx.x) * kRadixPerBlock + int64_t(w) * kRadixPerWave;
    // the lane's keys and values loaded first, all in flight together; the
    // ranking rounds below then wait on no memory
    uint32_t kk[kRadixItems];
    int32_t vv[kRadixItems];
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t i = wstart + int64_t(it) * kWave + lane;
        kk[it] = i < n ? keys_in[i] : 0u;
        vv[it] = i < n ? vals_in[i] : 0;
    }
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t i = wstart + int64_t(it) * kWave + lane;
        if (i < n) atomicAdd(&wcnt[w][(kk[it] >> shift) & mask], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < bins; d += kThreads) {
        int run = int(off[int64_t(d) * nblocks + blockIdx.x]);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            wbase[i][d] = run;
            run += wcnt[i][d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t i = wstart + int64_t(it) * kWave + lane;
        const bool valid = i < n;
        const uint32_t key = kk[it];
        const int d = int((key >> shift) & mask);
        uint64_t match = ballot(valid);
        for (int b = 0; b < width; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = ballot(valid && bit);
            match &= bit ? m : ~m;
        }
        if (valid) {
            const int rank = __popcll(match & lanemask_lt());
            const int64_t dest = int64_t(wbase[w][d]) + rank;
            if (dest < n) {
                keys_out[dest] = key;
                vals_out[dest] = vv[it];
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && ((match >> lane) >> 1) == 0) wbase[w][d] += __popcll(match);
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

// Sorts (keys, vals) by the low `nbits` bits of the keys; returns which
// ping-pong buffer holds the result (0 or 1) through *which.
hipError_t radix_sort(int64_t n, const int64_t *n_dev, int nbits, DevBuf &k0, DevBuf &k1,
                      DevBuf &v0, DevBuf &v1, DevBuf &hist_buf, DevBuf &off_buf,
                      DevBuf &scan_tmp, hipStream_t s, int *which)
{
    *which = 0;
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kRadixPerBlock - 1) / kRadixPerBlock;
    const size_t kv = sizeof(uint32_t) * size_t(n);
    if (nbits < 0 || nbits > 32 || k0.cap < kv || k1.cap < kv || v0.cap < kv || v1.cap < kv ||
        hist_buf.cap < sizeof(int32_t) * size_t(kRadixMaxBins * nb))
        return hipErrorInvalidValue;
    // the fewest passes of at most kRadixMaxBits, the bits spread evenly
    const int passes = (nbits + kRadixMaxBits - 1) / kRadixMaxBits;
    const int width = passes > 0 ? (nbits + passes - 1) / passes : 0;
    int32_t *hist = hist_buf.as<int32_t>();
    const int64_t *off = off_buf.as<int64_t>();
    uint32_t *kin = k0.as<uint32_t>(), *kout = k1.as<uint32_t>();
    int32_t *vin = v0.as<int32_t>(), *vout = v1.as<int32_t>();
    for (int p = 0; p < passes; ++p) {
        const int shift = p * width;
        const int wd = shift + width <= 32 ? width : 32 - shift;
        k_radix_count<<<dim3(unsigned(nb)), kThreads, 0, s>>>(n, n_dev, shift, wd, kin, hist, nb);
        hipError_t e = scan_counts(hist_buf, off_buf, (int64_t(1) << wd) * nb, scan_tmp, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<dim3(unsigned(nb)), kThreads, 0, s>>>(n, n_dev, shift, wd, kin, vin,
                                                               kout, vout, off, nb);
        std::swap(kin, kout);
        std::swap(vin, vout);
        *which ^= 1;
    }
    return hipGetLastError();
}

}  // namespace ngd
