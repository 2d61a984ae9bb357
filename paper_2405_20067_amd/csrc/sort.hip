// Stable LSD radix sort of (key, value) pairs, 8-bit digits.
//
// Per pass: each block counts the digits of its 4096 keys (a histogram in
// LDS), one exclusive scan turns the digit-major counts into output offsets,
// and each block scatters its keys in order: every wave ranks its 64 keys
// among equal digits with ballots (a match mask built from the 8 digit bits,
// popcount of the lower lanes), so equal keys keep their input order.
// The element count may live on the device (n_dev) with the host giving an
// upper bound: blocks past the count only write zero histogram columns.
#include <utility>

#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

// ---- stable LSD radix sort (8-bit digits) ------------------------------
constexpr int kThreads = 256;
constexpr int kRadixItems = 16;                        // per lane
constexpr int kRadixPerWave = kRadixItems * kWave;     // 1024
static_assert(kRadixPerWave * (kThreads / kWave) == kRadixPerBlock, "block size");

// Element count: the host bound, or the device count when one is given.
__device__ __forceinline__ int64_t count_of(int64_t n_max, const int64_t *n_dev)
{
    if (!n_dev) return n_max;
    const int64_t n = *n_dev;
    return n < n_max ? n : n_max;
}

__global__ __launch_bounds__(kThreads) void k_radix_count(int64_t n_max, const int64_t *n_dev,
                                                          int shift,
                                                          const uint32_t *__restrict__ keys,
                                                          int32_t *__restrict__ hist,
                                                          int64_t nblocks)
{
    __shared__ int cnt[256];
    const int64_t n = count_of(n_max, n_dev);
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kRadixPerBlock;
    for (int it = threadIdx.x; it < kRadixPerBlock; it += kThreads) {
        const int64_t i = base + it;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xffu], 1);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    int64_t n_max, const int64_t *n_dev, int shift, const uint32_t *__restrict__ keys_in,
    const int32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out, const int64_t *__restrict__ off, int64_t nblocks)
{
    constexpr int W = kThreads / kWave;
    __shared__ int wcnt[W][256];
    __shared__ int wbase[W][256];
    const int64_t n = count_of(n_max, n_dev);
    const int w = threadIdx.x / kWave, lane = lane_id();
#pragma unroll
    for (int i = 0; i < W; ++i) wcnt[i][threadIdx.x] = 0;
    __syncthreads();
    const int64_t wstart = int64_t(blockIdx.x) * kRadixPerBlock + int64_t(w) * kRadixPerWave;
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t i = wstart + int64_t(it) * kWave + lane;
        if (i < n) atomicAdd(&wcnt[w][(keys_in[i] >> shift) & 0xffu], 1);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        int run = int(off[int64_t(d) * nblocks + blockIdx.x]);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            wbase[i][d] = run;
            run += wcnt[i][d];
        }
    }
    __syncthreads();
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t i = wstart + int64_t(it) * kWave + lane;
        const bool valid = i < n;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const int d = int((key >> shift) & 0xffu);
        uint64_t match = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = ballot(valid && bit);
            match &= bit ? m : ~m;
        }
        if (valid) {
            const int rank = __popcll(match & lanemask_lt());
            const int64_t dest = int64_t(wbase[w][d]) + rank;
            if (dest < n) {
                keys_out[dest] = key;
                vals_out[dest] = vals_in[i];
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
    if (k0.cap < kv || k1.cap < kv || v0.cap < kv || v1.cap < kv ||
        hist_buf.cap < sizeof(int32_t) * size_t(256 * nb))
        return hipErrorInvalidValue;
    int32_t *hist = hist_buf.as<int32_t>();
    const int64_t *off = off_buf.as<int64_t>();
    uint32_t *kin = k0.as<uint32_t>(), *kout = k1.as<uint32_t>();
    int32_t *vin = v0.as<int32_t>(), *vout = v1.as<int32_t>();
    for (int shift = 0; shift < nbits; shift += 8) {
        k_radix_count<<<dim3(unsigned(nb)), kThreads, 0, s>>>(n, n_dev, shift, kin, hist, nb);
        hipError_t e = scan_counts(hist_buf, off_buf, 256 * nb, scan_tmp, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<dim3(unsigned(nb)), kThreads, 0, s>>>(n, n_dev, shift, kin, vin, kout,
                                                               vout,
                                                               off, nb);
        std::swap(kin, kout);
        std::swap(vin, vout);
        *which ^= 1;
    }
    return hipGetLastError();
}

}  // namespace ngd
