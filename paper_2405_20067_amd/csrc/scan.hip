// Device-wide exclusive scan of counts into offsets, and the L2 loss.
//
// The scan is three launches: per-block totals, one block scanning those,
// then every block scanning its own items with its carry.  Items per block
// are fixed (4096), so the result does not depend on the launch shape.
#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t wave_inclusive_scan64(int64_t x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a block of kScanThreads;
// returns the block total through *total.
__device__ int64_t block_exclusive_scan64(int64_t v, int64_t *total)
{
    __shared__ int64_t wave_tot[kScanThreads / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int64_t inc = wave_inclusive_scan64(v);
    if (lane == kWave - 1) wave_tot[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        before += (i < w) ? wave_tot[i] : 0;
        all += wave_tot[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t *__restrict__ in,
                                                              int64_t n,
                                                              int64_t *__restrict__ bsum)
{
    // a sum: the block's items are read coalesced, in any order
    const int64_t b0 = int64_t(blockIdx.x) * kScanBlock + threadIdx.x;
    int64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t g = b0 + int64_t(j) * kScanThreads;
        if (g < n) acc += in[g];
    }
    int64_t tot;
    block_exclusive_scan64(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t *__restrict__ bsum,
                                                           int64_t nb)
{
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = (i < nb) ? bsum[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan64(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

// Item i of a block at LDS slot i + i / kScanItems: a thread's run of
// kScanItems consecutive items then sits at stride kScanItems + 1.
__device__ __forceinline__ int scan_slot(int i) { return i + i / kScanItems; }

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int32_t *__restrict__ in,
                                                            int64_t n,
                                                            const int64_t *__restrict__ boff,
                                                            int64_t *__restrict__ out)
{
    // Coalesced in and out through LDS; in between each thread scans its
    // run of kScanItems consecutive items.
    __shared__ int64_t sb[kScanBlock + kScanBlock / kScanItems];
    const int64_t b0 = int64_t(blockIdx.x) * kScanBlock;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int i = threadIdx.x + j * kScanThreads;
        sb[scan_slot(i)] = (b0 + i < n) ? in[b0 + i] : 0;
    }
    __syncthreads();
    const int t0 = threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = sb[scan_slot(t0 + j)];
        acc += v[j];
    }
    int64_t tot;
    int64_t run = boff[blockIdx.x] + block_exclusive_scan64(acc, &tot);   // syncs
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        sb[scan_slot(t0 + j)] = run;
        run += v[j];
    }
    const int64_t base = b0 + t0;
    if (base < n && base + kScanItems >= n) out[n] = run;   // thread holding the last item
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int i = threadIdx.x + j * kScanThreads;
        if (b0 + i < n) out[b0 + i] = sb[scan_slot(i)];
    }
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_f32(float *p, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// ---- L2 loss ----------------------------------------------------------
constexpr int kLossThreads = 256;

__device__ double block_sum_f64(double v)
{
    __shared__ double part[kLossThreads / kWave];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    if (lane_id() == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kLossThreads / kWave; ++i) s += part[i];
    __syncthreads();
    return s;
}

// Per chunk of the q x 3 values: the gradient, and the chunk's sum of
// squared errors.  REL: each error weighted by w = 1 / (|f| + eps)^2, the
// prediction's own scale, taken as a constant (no gradient through it).
template <bool REL>
__global__ __launch_bounds__(kLossThreads) void k_l2_partial(const float *__restrict__ f,
                                                             const float *__restrict__ t,
                                                             int64_t m, float inv_scale2,
                                                             float eps, int64_t chunk,
                                                             float *__restrict__ grad,
                                                             double *__restrict__ parts)
{
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = (lo + chunk < m) ? lo + chunk : m;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kLossThreads) {
        const float fi = f[i];
        const float d = fi - t[i];
        if constexpr (REL) {
            const float den = fabsf(fi) + eps;
            const float w = 1.0f / (den * den);
            grad[i] = d * w * inv_scale2;
            acc += double(d) * double(d) * double(w);
        } else {
            grad[i] = d * inv_scale2;
            acc += double(d) * double(d);
        }
    }
    const double s = block_sum_f64(acc);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(kLossThreads) void k_l2_final(const double *__restrict__ parts,
                                                           int nparts, double inv_m,
                                                           float *__restrict__ loss)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kLossThreads) acc += parts[i];
    const double s = block_sum_f64(acc);
    if (threadIdx.x == 0) *loss = float(s * inv_m);
}

}  // namespace

size_t scan_tmp_bytes(int64_t n)
{
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    return size_t(nb > 0 ? nb : 1) * sizeof(int64_t);
}

hipError_t scan_counts(const DevBuf &in_buf, DevBuf &out_buf, int64_t n, DevBuf &tmp_buf,
                       hipStream_t s)
{
    // every buffer must hold what the launches below touch
    if (n < 0 || out_buf.cap < sizeof(int64_t) * size_t(n + 1) ||
        in_buf.cap < sizeof(int32_t) * size_t(n) || tmp_buf.cap < scan_tmp_bytes(n))
        return hipErrorInvalidValue;
    const int32_t *in = in_buf.as<int32_t>();
    int64_t *out = out_buf.as<int64_t>();
    void *tmp = tmp_buf.p;
    if (n == 0) {
        k_fill_i64<<<1, 64, 0, s>>>(out, 1, 0);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    int64_t *bsum = static_cast<int64_t *>(tmp);
    k_scan_reduce<<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(in, n, bsum);
    k_scan_top<<<1, kScanThreads, 0, s>>>(bsum, nb);
    k_scan_down<<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(in, n, bsum, out);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_zero_f32<<<unsigned((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_l2_loss(const float *f, const float *target, int64_t q, float *loss,
                          float *grad, float *partials, int nparts, hipStream_t s,
                          float rel_eps)
{
    const int64_t m = 3 * q;
    if (m == 0) {
        k_l2_final<<<1, kLossThreads, 0, s>>>(reinterpret_cast<const double *>(partials), 0,
                                             0.0, loss);
        return hipGetLastError();
    }
    const int64_t chunk = (m + nparts - 1) / nparts;
    const int used = int((m + chunk - 1) / chunk);
    double *parts = reinterpret_cast<double *>(partials);
    if (rel_eps > 0.0f)
        k_l2_partial<true><<<dim3(unsigned(used)), kLossThreads, 0, s>>>(
            f, target, m, float(2.0 / double(m)), rel_eps, chunk, grad, parts);
    else
        k_l2_partial<false><<<dim3(unsigned(used)), kLossThreads, 0, s>>>(
            f, target, m, float(2.0 / double(m)), 0.0f, chunk, grad, parts);
    k_l2_final<<<1, kLossThreads, 0, s>>>(parts, used, 1.0 / double(m), loss);
    return hipGetLastError();
}

}  // namespace ngd
