// Tile cull (Sec. 3.2, Eq. 3-5) on the device.
//
// Steps, all on the caller's stream:
//   1. Gaussian projections m_r = m . r (float32 fma chain) and thresholds
//      kappa^2 sigma_r^2 with sigma_r^2 = |L^T r|^2 in float64 (Eq. 3, 4).
//   2. Query projections q_r (Eq. 3) and their range per projection.
//   3. Locality keys: key_proj projections quantised to key_bits each over
//      the queries' range, bits interleaved (a Morton code); the same key for
//      the projected means.
//   4. Stable LSD radix sorts (8-bit digits, wavefront ballot ranking) of the
//      queries and of the Gaussians by key.
//   5. Tiles of `tile` consecutive sorted queries; per tile and projection
//      the extent [lo, hi] of its projected queries; sorted SoA query copy.
//   6. The (tile, Gaussian) interval test: one wave per 64 sorted Gaussians
//      walks a range of tiles, tile bounds wave-uniform, leaving each tile as
//      soon as no lane survives; one 64-bit ballot mask per (chunk, tile).
//   7. Per-tile counts, an exclusive scan into CSR offsets, and the
//      candidate lists (ascending sorted positions); then the transposed
//      Gaussian -> tile lists for the backward pass.
//
// Every operation that decides membership is an IEEE basic operation in a
// fixed order (no contraction in this file), so the lists are reproducible
// bit for bit by a CPU implementation of the same recipe.
#pragma clang fp contract(off)

#include <algorithm>
#include <utility>

#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kThreads = 256;

// Per Gaussian: its projected means and the interval test's squared
// half-widths (Eq. 3-4), and the box of the forward's per-wave test.
//
// The box: M = (x - m)^T V^-1 (x - m) >= (x_i - m_i)^2 / V_ii for every
// coordinate i (V = L L^T; Cauchy-Schwarz), so a query with
// |x_i - m_i| > sr sqrt(V_ii) has M above sr^2 whatever its other
// coordinates.  sr^2 is the forward's skip threshold in units of M, widened
// by (1 + 2^-8)^2 for the rounding of its float32 distances.  V_ii =
// |row i of L|^2 and [m - r, m + r] are formed in float64 and the box is
// rounded outwards to float16 (a looser box is still a certificate, and
// half the bytes of float32 for the forward's per-pair reads); box holds
// lo_0..lo_{n-1}, hi_0..hi_{n-1} per Gaussian as float16 bits, padded to
// BSH halves (a multiple of 16 bytes), in the caller's order (gathered with
// the records).
// float16 bits of the largest float16 <= v (DOWN) or smallest >= v (up).
// The nearest float16 of float(v) is one of the two float16 values around v
// (rounding is monotone and float16 values are floats), so one step of the
// bit pattern towards the right side suffices; overflow goes to +-inf.
template <bool DOWN> __device__ __forceinline__ uint16_t half_outward(double v)
{
    const _Float16 h = _Float16(float(v));
    uint16_t u = __builtin_bit_cast(uint16_t, h);
    const double hv = double(float(h));
    if (DOWN ? hv > v : hv < v) {
        if ((u & 0x7fffu) == 0) u = DOWN ? 0x8001u : 0x0001u;   // +-0: smallest subnormal
        else if ((u & 0x8000u) != 0) u = DOWN ? u + 1 : u - 1;  // negative: magnitude
        else u = DOWN ? u - 1 : u + 1;                          // positive: magnitude
    }
    return u;
}

template <int N>
__global__ __launch_bounds__(kThreads) void k_gauss_proj(int64_t k, int P,
                                                         const float *__restrict__ rec, int R,
                                                         const float *__restrict__ lfac,
                                                         const float *__restrict__ proj,
                                                         float kappa2, float *__restrict__ g_mr,
                                                         float *__restrict__ g_thr, double sr,
                                                         float *__restrict__ box)
{
    constexpr int T = N * (N + 1) / 2;
    constexpr int BSH = (2 * N + 7) / 8 * 8;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= k) return;
    float m[N];
    double L[T];
#pragma unroll
    for (int a = 0; a < N; ++a) m[a] = rec[i * R + a];
#pragma unroll
    for (int e = 0; e < T; ++e) L[e] = lfac[i * T + e];
    uint16_t bx[BSH];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b <= a; ++b) v = fma(L[a * (a + 1) / 2 + b], L[a * (a + 1) / 2 + b], v);
        const double r = sr * sqrt(v);
        bx[a] = half_outward<true>(double(m[a]) - r);
        bx[N + a] = half_outward<false>(double(m[a]) + r);
    }
#pragma unroll
    for (int e = 2 * N; e < BSH; ++e) bx[e] = 0;
    uint4 *bo = reinterpret_cast<uint4 *>(box) + i * (BSH / 8);
#pragma unroll
    for (int e = 0; e < BSH / 8; ++e) {
        const uint16_t *h = bx + 8 * e;
        bo[e] = make_uint4(h[0] | uint32_t(h[1]) << 16, h[2] | uint32_t(h[3]) << 16,
                           h[4] | uint32_t(h[5]) << 16, h[6] | uint32_t(h[7]) << 16);
    }
    for (int j = 0; j < P; ++j) {
        const float *r = proj + j * N;
        float acc = 0.0f;
#pragma unroll
        for (int a = 0; a < N; ++a) acc = fmaf(m[a], r[a], acc);
        g_mr[j * k + i] = acc;
        double s2 = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            double u = 0.0;   // (L^T r)_b = sum_{a >= b} L_ab r_a
#pragma unroll
            for (int a = b; a < N; ++a) u = fma(L[a * (a + 1) / 2 + b], double(r[a]), u);
            s2 = fma(u, u, s2);
        }
        const float s2f = float(s2);
        g_thr[j * k + i] = kappa2 * s2f;
    }
}

// The queries' projections (P x q, SoA) and per block each projection's
// min and max: as floats (KEYS false: the range of the locality keys), or as
// order-preserving keys (KEYS true: the k-d root's extents).
template <int N, int PMAX, bool KEYS>
__global__ __launch_bounds__(kThreads) void k_query_proj(int64_t q, int P,
                                                         const float *__restrict__ queries,
                                                         const float *__restrict__ proj,
                                                         float *__restrict__ qr,
                                                         float *__restrict__ part)
{
    __shared__ uint32_t smin[kThreads / kWave][PMAX], smax[kThreads / kWave][PMAX];
    const int64_t p = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const bool valid = p < q;
    const int w = threadIdx.x / kWave;
    float x[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = valid ? queries[p * N + a] : 0.0f;
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
        if (j < P) {
            float acc = 0.0f;
#pragma unroll
            for (int a = 0; a < N; ++a) acc = fmaf(x[a], proj[j * N + a], acc);
            if (valid) qr[j * q + p] = acc;
            if constexpr (KEYS) {
                const uint32_t key = orderable(acc);
                const uint32_t lo = wave_umin_dpp(valid ? key : 0xffffffffu);
                const uint32_t hi = wave_umax_dpp(valid ? key : 0u);
                if (lane_id() == kWave - 1) {
                    smin[w][j] = lo;
                    smax[w][j] = hi;
                }
            } else {
                const float lo = wave_min(valid ? acc : INFINITY);
                const float hi = wave_max(valid ? acc : -INFINITY);
                if (lane_id() == 0) {
                    smin[w][j] = __float_as_uint(lo);
                    smax[w][j] = __float_as_uint(hi);
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < P) {
        const int j = threadIdx.x;
        uint32_t *pk = reinterpret_cast<uint32_t *>(part);
        if constexpr (KEYS) {
            uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
            for (int i = 0; i < kThreads / kWave; ++i) {
                lo = min(lo, smin[i][j]);
                hi = max(hi, smax[i][j]);
            }
            pk[(int64_t(blockIdx.x) * P + j) * 2 + 0] = lo;
            pk[(int64_t(blockIdx.x) * P + j) * 2 + 1] = hi;
        } else {
            float lo = INFINITY, hi = -INFINITY;
#pragma unroll
            for (int i = 0; i < kThreads / kWave; ++i) {
                lo = fminf(lo, __uint_as_float(smin[i][j]));
                hi = fmaxf(hi, __uint_as_float(smax[i][j]));
            }
            part[(int64_t(blockIdx.x) * P + j) * 2 + 0] = lo;
            part[(int64_t(blockIdx.x) * P + j) * 2 + 1] = hi;
        }
    }
}

// qrange = [lo (P) | hi (P) | scale (P)]; one block per projection.
__global__ __launch_bounds__(kThreads) void k_range_final(int64_t nparts, int P, int key_bits,
                                                          const float *__restrict__ part,
                                                          float *__restrict__ qrange)
{
    __shared__ float slo[kThreads / kWave], shi[kThreads / kWave];
    const int j = blockIdx.x;
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t b = threadIdx.x; b < nparts; b += kThreads) {
        lo = fminf(lo, part[(b * P + j) * 2 + 0]);
        hi = fmaxf(hi, part[(b * P + j) * 2 + 1]);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane_id() == 0) {
        slo[threadIdx.x / kWave] = lo;
        shi[threadIdx.x / kWave] = hi;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int i = 0; i < kThreads / kWave; ++i) {
        lo = fminf(lo, slo[i]);
        hi = fmaxf(hi, shi[i]);
    }
    qrange[j] = lo;
    qrange[P + j] = hi;
    qrange[2 * P + j] =
        (hi > lo) ? float(double(1u << key_bits) / (double(hi) - double(lo))) : 0.0f;
}

// The k-d root's extents from the per-block key partials: ext[2j] and
// ext[2j + 1] get projection j's min and max key; one block per projection.
__global__ __launch_bounds__(kThreads) void k_root_keys(int64_t nparts, int P,
                                                        const float *__restrict__ part,
                                                        uint32_t *__restrict__ ext)
{
    __shared__ uint32_t slo[kThreads / kWave], shi[kThreads / kWave];
    const int j = blockIdx.x;
    const uint32_t *pk = reinterpret_cast<const uint32_t *>(part);
    uint32_t lo = 0xffffffffu, hi = 0u;
    for (int64_t b = threadIdx.x; b < nparts; b += kThreads) {
        lo = min(lo, pk[(b * P + j) * 2 + 0]);
        hi = max(hi, pk[(b * P + j) * 2 + 1]);
    }
    lo = wave_umin_dpp(lo);
    hi = wave_umax_dpp(hi);
    if (lane_id() == kWave - 1) {
        slo[threadIdx.x / kWave] = lo;
        shi[threadIdx.x / kWave] = hi;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int i = 0; i < kThreads / kWave; ++i) {
        lo = min(lo, slo[i]);
        hi = max(hi, shi[i]);
    }
    ext[2 * j + 0] = lo;
    ext[2 * j + 1] = hi;
}

// Locality key of row i of a P x n SoA array of projections.
__global__ __launch_bounds__(kThreads) void k_keys(int64_t n, int P,
                                                   const float *__restrict__ vals,
                                                   const float *__restrict__ qrange,
                                                   int key_proj, int key_bits,
                                                   uint32_t *__restrict__ keys,
                                                   int32_t *__restrict__ idx)
{
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const float top = float((1u << key_bits) - 1u);
    uint32_t key = 0;
    int digit[NGD_MAX_PROJ];
#pragma unroll
    for (int j = 0; j < NGD_MAX_PROJ; ++j) {
        if (j < key_proj) {
            const float t = vals[j * n + i] - qrange[j];
            float u = t * qrange[2 * P + j];
            u = fminf(fmaxf(u, 0.0f), top);
            digit[j] = int(u);
        }
    }
    for (int b = key_bits - 1; b >= 0; --b) {
#pragma unroll
        for (int j = 0; j < NGD_MAX_PROJ; ++j)
            if (j < key_proj) key = (key << 1) | uint32_t((digit[j] >> b) & 1);
    }
    keys[i] = key;
    idx[i] = int32_t(i);
}

// ---- tiles ---------------------------------------------------------------
// Also the centre of each tile's box in the query space (the midpoint of
// each coordinate's range; the matrix-core forward expands its quadratic
// forms about it), into tcen.
template <int N, int PMAX>
__global__ __launch_bounds__(1024) void k_tile_bounds(int64_t q, int tile, int P, int PP,
                                                      const int32_t *__restrict__ perm,
                                                      const float *__restrict__ qr,
                                                      const float *__restrict__ qr_s,
                                                      const float *__restrict__ queries,
                                                      float *__restrict__ qs,
                                                      float *__restrict__ tlo,
                                                      float *__restrict__ thi,
                                                      float *__restrict__ tbnd,
                                                      float *__restrict__ tcen)
{
    __shared__ float smin[1024 / kWave][PMAX], smax[1024 / kWave][PMAX];
    __shared__ float xmin[1024 / kWave][N], xmax[1024 / kWave][N];
    const int64_t t = blockIdx.x;
    float lo[PMAX], hi[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
        lo[j] = INFINITY;
        hi[j] = -INFINITY;
    }
    for (int s = threadIdx.x; s < tile; s += blockDim.x) {
        const int64_t p = t * tile + s;
        if (p >= q) break;
        const int64_t idx = perm[p];
#pragma unroll
        for (int a = 0; a < N; ++a) qs[a * q + p] = queries[idx * N + a];
#pragma unroll
        for (int j = 0; j < PMAX; ++j) {
            if (j < P) {
                // projections in tile order when the ordering left them so
                const float v = qr_s ? qr_s[j * q + p] : qr[j * q + idx];
                lo[j] = fminf(lo[j], v);
                hi[j] = fmaxf(hi[j], v);
            }
        }
    }
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    // wave minima / maxima by DPP on order-preserving keys (the float order
    // exactly, no LDS traffic), totals in lane 63
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
        if (j < P) {
            const uint32_t a = wave_umin_dpp(orderable(lo[j]));
            const uint32_t b = wave_umax_dpp(orderable(hi[j]));
            if (lane_id() == kWave - 1) {
                smin[w][j] = from_orderable(a);
                smax[w][j] = from_orderable(b);
            }
        }
    }
    // the coordinates' ranges, read back from this thread's own stores of
    // the sorted copy (coalesced), once the projections' registers are free
    {
        float xl[N], xh[N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            xl[a] = INFINITY;
            xh[a] = -INFINITY;
        }
        for (int s = threadIdx.x; s < tile; s += blockDim.x) {
            const int64_t p = t * tile + s;
            if (p >= q) break;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const float v = qs[a * q + p];
                xl[a] = fminf(xl[a], v);
                xh[a] = fmaxf(xh[a], v);
            }
        }
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const uint32_t mn = wave_umin_dpp(orderable(xl[a]));
            const uint32_t mx = wave_umax_dpp(orderable(xh[a]));
            if (lane_id() == kWave - 1) {
                xmin[w][a] = from_orderable(mn);
                xmax[w][a] = from_orderable(mx);
            }
        }
    }
    __syncthreads();
    if (int(threadIdx.x) < N) {
        const int a = threadIdx.x;
        float mn = INFINITY, mx = -INFINITY;
        for (int i = 0; i < nw; ++i) {
            mn = fminf(mn, xmin[i][a]);
            mx = fmaxf(mx, xmax[i][a]);
        }
        tcen[t * N + a] = (mn <= mx) ? 0.5f * mn + 0.5f * mx : 0.0f;
    }
    if (int(threadIdx.x) < PP) {
        const int j = threadIdx.x;
        // the padding projections pass every test
        float a = -INFINITY, b = INFINITY;
        if (j < P) {
            a = INFINITY;
            b = -INFINITY;
            for (int i = 0; i < nw; ++i) {
                a = fminf(a, smin[i][j]);
                b = fmaxf(b, smax[i][j]);
            }
            tlo[t * P + j] = a;
            thi[t * P + j] = b;
        }
        tbnd[t * 2 * PP + j] = a;
        tbnd[t * 2 * PP + PP + j] = b;
    }
}

// Records and forward boxes of the Gaussians in their tile order: a block
// moves 64 records of R floats and 64 boxes of B 4-byte words as float4s,
// consecutive threads on consecutive float4s.
__global__ __launch_bounds__(kThreads) void k_rec_gather(int64_t k, int R, int B,
                                                         const int32_t *__restrict__ gperm,
                                                         const float *__restrict__ rec,
                                                         const float *__restrict__ box,
                                                         float *__restrict__ grec,
                                                         float *__restrict__ gbox)
{
    const int R4 = R / 4, B4 = B / 4;
    const int64_t s0 = int64_t(blockIdx.x) * kWave;
    const int cnt = int(k - s0 < kWave ? k - s0 : kWave);
    {
        const float4 *src = reinterpret_cast<const float4 *>(rec);
        float4 *dst = reinterpret_cast<float4 *>(grec) + s0 * R4;
        for (int e = threadIdx.x; e < cnt * R4; e += kThreads) {
            const int sl = e / R4;
            const int f = e - sl * R4;
            dst[e] = src[int64_t(gperm[s0 + sl]) * R4 + f];
        }
    }
    const float4 *src = reinterpret_cast<const float4 *>(box);
    float4 *dst = reinterpret_cast<float4 *>(gbox) + s0 * B4;
    for (int e = threadIdx.x; e < cnt * B4; e += kThreads) {
        const int sl = e / B4;
        const int f = e - sl * B4;
        dst[e] = src[int64_t(gperm[s0 + sl]) * B4 + f];
    }
}

// ---- the interval test restated as two comparisons ------------------------
// For a Gaussian with projected mean m and threshold thr = fl(kappa^2 sigma^2)
// on projection j, Eq. 5 keeps a box [lo, hi] iff
//     fl(d * d) <= thr,   d = max(fl(lo - m), fl(m - hi), 0).
// x -> fl(x * x) is monotone on x >= 0, so fl(d * d) <= thr iff d <= s, the
// largest float whose rounded square is <= thr.  d <= s iff fl(lo - m) <= s
// and fl(m - hi) <= s; x -> fl(x - m) and x -> fl(m - x) are monotone too, so
// these hold iff lo <= U and hi >= L, with U the largest float x such that
// fl(x - m) <= s and L the smallest float x such that fl(m - x) <= s.  The
// test per (lane, box, projection) is then two comparisons, with exactly the
// outcome of the formula (finite bounds and means; thr < 0 keeps nothing,
// U = L = NaN).  Each limit is found by bisection over the ordered bit
// patterns of the floats, which needs only the monotonicity; it starts from a
// bracket of 8 units in the last place about the arithmetic guess and falls
// back to the whole range when that bracket does not hold the change.

// ordered image of a non-NaN float: keys compare as the floats do
__device__ __forceinline__ int32_t fkey(float x)
{
    const int32_t b = __float_as_int(x);
    return b >= 0 ? b : (b ^ 0x7fffffff);
}

__device__ __forceinline__ float fkey_inv(int32_t key)
{
    return __int_as_float(key >= 0 ? key : (key ^ 0x7fffffff));
}

constexpr int32_t kKeyNegInf = int32_t(0xff800000u ^ 0x7fffffffu);
constexpr int32_t kKeyPosInf = 0x7f800000;

// The largest key in [lo, hi] whose float satisfies pred, for pred true at
// lo and monotone (true, then false) on the range.
template <class Pred>
__device__ int32_t last_true(const Pred &pred, float guess, int32_t lo, int32_t hi)
{
    if (pred(fkey_inv(hi))) return hi;
    // invariant: pred(lo) true, pred(hi) false
    if (guess == guess) {
        const int64_t g = fkey(guess);
        const int32_t a = int32_t(g - 8 > lo ? g - 8 : lo);
        const int32_t b = int32_t(g + 8 < hi ? g + 8 : hi);
        if (pred(fkey_inv(a))) lo = a;
        if (!pred(fkey_inv(b))) hi = b;
    }
    while (int64_t(hi) - lo > 1) {
        const int32_t mid = int32_t((int64_t(lo) + hi) >> 1);
        if (pred(fkey_inv(mid)))
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_gauss_limits(
    int64_t k, const int32_t *__restrict__ gperm, const float *__restrict__ g_mr,
    const float *__restrict__ g_mr_s, const float *__restrict__ g_thr, float *__restrict__ g_ub,
    float *__restrict__ g_lb)
{
    const int64_t s = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (s >= k) return;
    const int64_t j = blockIdx.y;
    const int64_t i = gperm[s];
    // null g_mr_s: the means are not in order yet
    const float m = g_mr_s ? g_mr_s[j * k + s] : g_mr[j * k + i];
    const float thr = g_thr[j * k + i];
    float ub = __int_as_float(0x7fc00000), lb = ub;   // NaN: nothing passes
    if (thr >= 0.0f && m - m == 0.0f) {
        const float r = fkey_inv(last_true([thr](float x) { return x * x <= thr; }, sqrtf(thr),
                                           fkey(0.0f), kKeyPosInf));
        ub = fkey_inv(last_true([m, r](float x) { return x - m <= r; }, m + r, kKeyNegInf,
                                kKeyPosInf));
        // the smallest x with fl(m - x) <= r: one key above the largest
        // with fl(m - x) > r (none: -inf itself passes)
        const auto fails = [m, r](float x) { return !(m - x <= r); };
        lb = fails(-INFINITY)
                 ? fkey_inv(last_true(fails, m - r, kKeyNegInf, kKeyPosInf) + 1)
                 : -INFINITY;
    }
    g_ub[j * k + s] = ub;
    g_lb[j * k + s] = lb;
}

// Bounds of every super-tile: the union of its tiles' boxes.
__global__ __launch_bounds__(kThreads) void k_super_bounds(int64_t ntiles, int PP,
                                                           const float *__restrict__ tbnd,
                                                           float *__restrict__ sbnd)
{
    const int64_t nsup = (ntiles + kSuperTiles - 1) / kSuperTiles;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= nsup * 2 * PP) return;
    const int64_t sp = i / (2 * PP);
    const int e = int(i - sp * 2 * PP);
    const int64_t t1 = (sp + 1) * kSuperTiles < ntiles ? (sp + 1) * kSuperTiles : ntiles;
    float v = e < PP ? INFINITY : -INFINITY;
    for (int64_t t = sp * kSuperTiles; t < t1; ++t)
        v = e < PP ? fminf(v, tbnd[t * 2 * PP + e]) : fmaxf(v, tbnd[t * 2 * PP + e]);
    sbnd[i] = v;
}

// ---- the interval test (Eq. 5 per tile) -----------------------------------
// One wave per chunk of 64 ordered Gaussians (lane = Gaussian, its limits
// U, L in registers) walks a range of tiles with the boxes wave-uniform,
// first per super-tile of kSuperTiles tiles, then per tile for the lanes
// still alive; a test stops once no lane survives (checked every 4
// projections).  A super-tile's box contains each of its tiles' boxes, so a
// lane it culls is culled for each tile, and the masks are those of the
// plain per-tile test bit for bit.
//
// Each group of 4 projections narrows the execution mask directly: with
// exec = alive, v_cmpx keeps a lane only where its comparison holds (8
// vector compares and no scalar mask arithmetic per group); the surviving
// mask is read back and exec restored within the same asm block, so the
// compiler's view of exec is untouched.  NaN limits compare false, as
// before.
template <int PP>
__device__ __forceinline__ uint64_t box_test(uint64_t alive, const float (&ub)[PP],
                                             const float (&lb)[PP],
                                             const float *__restrict__ box_p)
{
    // the whole box as two wave-uniform vector loads (one wait per box,
    // not one per group); boxes are 2 PP floats, aligned to 2 PP * 4 bytes
    typedef float boxv __attribute__((ext_vector_type(PP)));
    const boxv lov = *reinterpret_cast<const boxv *>(box_p);
    const boxv hiv = *reinterpret_cast<const boxv *>(box_p + PP);
    float box[2 * PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        box[j] = lov[j];
        box[PP + j] = hiv[j];
    }
#pragma unroll
    for (int g = 0; g < PP; g += 4) {
        uint64_t sv;
        asm volatile("s_mov_b64 %[sv], exec\n\t"
                     "s_mov_b64 exec, %[al]\n\t"
                     "v_cmpx_le_f32_e32 vcc, %[l0], %[u0]\n\t"
                     "v_cmpx_ge_f32_e32 vcc, %[h0], %[b0]\n\t"
                     "v_cmpx_le_f32_e32 vcc, %[l1], %[u1]\n\t"
                     "v_cmpx_ge_f32_e32 vcc, %[h1], %[b1]\n\t"
                     "v_cmpx_le_f32_e32 vcc, %[l2], %[u2]\n\t"
                     "v_cmpx_ge_f32_e32 vcc, %[h2], %[b2]\n\t"
                     "v_cmpx_le_f32_e32 vcc, %[l3], %[u3]\n\t"
                     "v_cmpx_ge_f32_e32 vcc, %[h3], %[b3]\n\t"
                     "s_mov_b64 %[al], exec\n\t"
                     "s_mov_b64 exec, %[sv]"
                     : [al] "+s"(alive), [sv] "=&s"(sv)
                     : [l0] "s"(box[g + 0]), [u0] "v"(ub[g + 0]), [h0] "s"(box[PP + g + 0]),
                       [b0] "v"(lb[g + 0]), [l1] "s"(box[g + 1]), [u1] "v"(ub[g + 1]),
                       [h1] "s"(box[PP + g + 1]), [b1] "v"(lb[g + 1]), [l2] "s"(box[g + 2]),
                       [u2] "v"(ub[g + 2]), [h2] "s"(box[PP + g + 2]), [b2] "v"(lb[g + 2]),
                       [l3] "s"(box[g + 3]), [u3] "v"(ub[g + 3]), [h3] "s"(box[PP + g + 3]),
                       [b3] "v"(lb[g + 3])
                     : "vcc");
        if (alive == 0) break;
    }
    return alive;
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_cull_test(
    int64_t k, int64_t ntiles, int64_t tpad, int P, int tiles_per_wave,
    const float *__restrict__ g_ub, const float *__restrict__ g_lb,
    const float *__restrict__ tbnd, const float *__restrict__ sbnd, uint64_t *__restrict__ masks,
    int64_t per_seg, int32_t *__restrict__ seg_cnt)
{
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t nchunks = (k + kWave - 1) / kWave;
    const int64_t c = int64_t(blockIdx.x) * (kThreads / kWave) + w;
    if (c >= nchunks) return;
    const int64_t s = c * kWave + lane;
    const bool valid = s < k;
    float ub[PP], lb[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        // padding projections: the boxes span everything and so does this
        ub[j] = (valid && j < P) ? g_ub[j * k + s] : INFINITY;
        lb[j] = (valid && j < P) ? g_lb[j * k + s] : -INFINITY;
    }
    const uint64_t alive0 = ballot(valid);
    // tiles_per_wave is a multiple of 64 (and so of kSuperTiles)
    const int64_t t0 = int64_t(blockIdx.y) * tiles_per_wave;
    const int64_t t1 = (t0 + tiles_per_wave < ntiles) ? t0 + tiles_per_wave : ntiles;
    for (int64_t tb = t0; tb < t1; tb += kWave) {
        const int64_t te = (tb + kWave < t1) ? tb + kWave : t1;
        uint64_t mine = 0;   // lane l: mask of tile tb + l
        for (int64_t sb = tb; sb < te; sb += kSuperTiles) {
            const uint64_t sup =
                box_test<PP>(alive0, ub, lb, sbnd + (sb / kSuperTiles) * 2 * PP);
            if (sup == 0) continue;
            const int64_t se = (sb + kSuperTiles < te) ? sb + kSuperTiles : te;
            for (int64_t t = sb; t < se; ++t) {
                const uint64_t m = box_test<PP>(sup, ub, lb, tbnd + t * 2 * PP);
                if (lane == int(t - tb)) mine = m;
            }
        }
        if (tb + lane < te) {
            masks[c * tpad + tb + lane] = mine;
            // the candidates of each (chunk segment, tile), for the lists'
            // offsets (integer atomics: the sums do not depend on order)
            if (mine) atomicAdd(&seg_cnt[(c / per_seg) * ntiles + tb + lane], __popcll(mine));
        }
    }
}

// ---- lists ----------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_seg_prefix(int64_t ntiles, int nseg,
                                                         int32_t *__restrict__ seg_cnt,
                                                         int32_t *__restrict__ tile_cnt,
                                                         unsigned long long *__restrict__ maxc)
{
    // per tile, the exclusive prefix of its segments' counts; kU loads in
    // flight at a time; the longest list by one atomic per wave
    constexpr int kU = 16;
    const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const bool ok = t < ntiles;
    int run = 0;
    for (int seg = 0; seg < nseg; seg += kU) {
        int v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            v[u] = (ok && seg + u < nseg) ? seg_cnt[int64_t(seg + u) * ntiles + t] : 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (ok && seg + u < nseg) seg_cnt[int64_t(seg + u) * ntiles + t] = run;
            run += v[u];
        }
    }
    if (ok) tile_cnt[t] = run;
    // counts are non-negative: their bit patterns order as unsigned
    const int most = __float_as_int(wave_max_nonneg(__int_as_float(run)));
    if (lane_id() == 0) atomicMax(maxc, static_cast<unsigned long long>(most));
}

// Candidate lists from the masks: one workgroup per (64 tiles, chunk
// segment).  Per round of 64 chunks the masks are read row by row
// (coalesced) into LDS, transposed; each wave then takes 16 of the tiles,
// lane = chunk: the popcounts' exclusive scan gives each chunk's first
// position, every lane places its chunk's set bits (ascending) in the
// wave's LDS staging row, and the row goes out with contiguous stores.
constexpr int kFillTiles = 64;
constexpr int kFillStage = 1024;   // staged candidates per wave and round
__global__ __launch_bounds__(kThreads) void k_fill_cand(int64_t ntiles, int64_t tpad,
                                                        int64_t nchunks, int64_t per_seg,
                                                        const uint64_t *__restrict__ masks,
                                                        const int32_t *__restrict__ seg_cnt,
                                                        const int64_t *__restrict__ tile_off,
                                                        int64_t cap,
                                                        int32_t *__restrict__ cand,
                                                        int32_t *__restrict__ ent_tile)
{
    __shared__ uint64_t sm[kFillTiles][kWave + 1];   // [tile][chunk]
    __shared__ int32_t stage[kThreads / kWave][kFillStage];
    __shared__ int64_t run[kFillTiles];
    __shared__ int64_t tend[kFillTiles];   // the tiles' list ends, loaded once
    const int64_t t0 = int64_t(blockIdx.x) * kFillTiles;
    const int64_t seg = blockIdx.y;
    const int64_t c0 = seg * per_seg;
    const int64_t c1 = (c0 + per_seg < nchunks) ? c0 + per_seg : nchunks;
    const int w = int(threadIdx.x) / kWave, lane = lane_id();
    int has = 0;   // this segment has candidates in this thread's tile
    if (int(threadIdx.x) < kFillTiles) {
        const int64_t t = t0 + threadIdx.x;
        if (t < ntiles) {
            // the segments' exclusive offsets within the tile's list
            const int64_t b = seg_cnt[seg * ntiles + t];
            const int64_t e = seg + 1 < int64_t(gridDim.y) ? seg_cnt[(seg + 1) * ntiles + t]
                                                           : tile_off[t + 1] - tile_off[t];
            has = e > b;
        }
        run[threadIdx.x] = t < ntiles ? tile_off[t] + seg_cnt[seg * ntiles + t] : 0;
        // no entry at or past `cap` is written (lists longer than the
        // buffers are built again once the buffers have grown)
        tend[threadIdx.x] = t < ntiles ? (tile_off[t + 1] < cap ? tile_off[t + 1] : cap) : 0;
    }
    // a (tiles, segment) block without candidates reads none of its masks
    if (!__syncthreads_or(has)) return;
    int32_t *st = stage[w];
    for (int64_t cb = c0; cb < c1; cb += kWave) {
        __syncthreads();   // run[] set; the previous round's readers done
        for (int r = w; r < kWave; r += kThreads / kWave) {
            const int64_t c = cb + r, t = t0 + lane;
            sm[lane][r] = (c < c1 && t < ntiles) ? masks[c * tpad + t] : 0ull;
        }
        __syncthreads();
        for (int tl = w; tl < kFillTiles; tl += kThreads / kWave) {
            const int64_t t = t0 + tl;
            if (t >= ntiles) break;   // uniform
            uint64_t m = sm[tl][lane];
            const int cnt = __popcll(m);
            const int incl = wave_inclusive_scan(cnt);
            const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
            if (total == 0) continue;   // uniform
            const int32_t gbase = int32_t((cb + lane) * kWave);
            const int64_t base = run[tl], end = tend[tl];
            int k = incl - cnt;
            if (total <= kFillStage) {   // uniform
                while (m) {
                    st[k++] = gbase + (__ffsll(static_cast<unsigned long long>(m)) - 1);
                    m &= m - 1;
                }
                for (int i = lane; i < total; i += kWave) {
                    const int64_t pos = base + i;
                    if (pos < end) {
                        cand[pos] = st[i];
                        ent_tile[pos] = int32_t(t);
                    }
                }
            } else {   // a dense round: every lane writes its own bits
                while (m) {
                    const int64_t pos = base + k++;
                    if (pos < end) {
                        cand[pos] = gbase + (__ffsll(static_cast<unsigned long long>(m)) - 1);
                        ent_tile[pos] = int32_t(t);
                    }
                    m &= m - 1;
                }
            }
            if (lane == 0) run[tl] = base + total;   // this wave's own tile
        }
    }
}

// Transposed lists: entries of the candidate lists grouped by Gaussian.
// Counts per Gaussian (order-independent integer atomics), then a stable
// radix sort of (Gaussian, entry) by Gaussian keeps each Gaussian's entries
// in ascending entry order, i.e. ascending tile order.
__global__ __launch_bounds__(kThreads) void k_ghist(int64_t total, const int32_t *__restrict__ cand,
                                                    int32_t *__restrict__ g_cnt)
{
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e < total) atomicAdd(&g_cnt[cand[e]], 1);
}

__global__ __launch_bounds__(kThreads) void k_ent_init(int64_t total,
                                                       const int32_t *__restrict__ cand,
                                                       uint32_t *__restrict__ keys,
                                                       int32_t *__restrict__ vals)
{
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= total) return;
    keys[e] = uint32_t(cand[e]);
    vals[e] = int32_t(e);
}

__global__ __launch_bounds__(kThreads) void k_ent_gather(int64_t total,
                                                         const int32_t *__restrict__ g_ent,
                                                         const int32_t *__restrict__ ent_tile,
                                                         int32_t *__restrict__ g_tiles)
{
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < total) g_tiles[i] = ent_tile[g_ent[i]];
}

// Work items: ceil(count / per) items for each row of a CSR.
__global__ __launch_bounds__(kThreads) void k_item_count(int64_t n, const int64_t *__restrict__ off,
                                                         int per, int32_t *__restrict__ cnt)
{
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t len = off[i + 1] - off[i];
    cnt[i] = int32_t((len + per - 1) / per);
}

__global__ __launch_bounds__(kThreads) void k_item_fill(int64_t n, const int64_t *__restrict__ ioff,
                                                        int64_t cap, int32_t *__restrict__ owner)
{
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    for (int64_t j = ioff[i]; j < ioff[i + 1] && j < cap; ++j) owner[j] = int32_t(i);
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

// The list sizes next to the longest list, for one copy to the host:
// stats[1] longest list (set by k_seg_prefix), stats[2] total, stats[3] items.
__global__ void k_gather_sizes(int64_t *stats, const int64_t *tile_end, const int64_t *item_end)
{
    if (threadIdx.x == 0) {
        stats[2] = *tile_end;
        stats[3] = *item_end;
    }
}

__global__ void k_iota(int32_t *p, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = int32_t(i);
}

__global__ void k_zero_i32(int32_t *p, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <typename T> inline unsigned nblk(T n, int per)
{
    return unsigned((int64_t(n) + per - 1) / per);
}

// items per CSR row -> exclusive offsets (n + 1)
hipError_t launch_items(int64_t n, const int64_t *off, int per, DevBuf &cnt, DevBuf &ioff,
                        DevBuf &scan_tmp, hipStream_t s)
{
    if (cnt.cap < sizeof(int32_t) * size_t(n)) return hipErrorInvalidValue;
    if (n > 0) k_item_count<<<nblk(n, kThreads), kThreads, 0, s>>>(n, off, per, cnt.as<int32_t>());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_counts(cnt, ioff, n, scan_tmp, s);
}

// The Gaussians in their tile order, what the interval test needs: its
// limits (g_sorted: the projected means are already in that order).
hipError_t gauss_limits(ngd_cull *c, int64_t k, int P, bool g_sorted, hipStream_t s)
{
    k_gauss_limits<<<dim3(nblk(k, kThreads), unsigned(P)), kThreads, 0, s>>>(
        k, c->gperm.as<int32_t>(), c->g_mr.as<float>(), g_sorted ? c->g_mr_s.as<float>() : nullptr,
        c->g_thr.as<float>(), c->g_ub.as<float>(), c->g_lb.as<float>());
    return hipGetLastError();
}

// The Gaussians in their tile order, what the forward needs: records and the
// boxes of its per-wave test.
hipError_t gauss_records(ngd_cull *c, const ngd_mixture *mix, int64_t k, int R, hipStream_t s)
{
    k_rec_gather<<<nblk(k, kWave), kThreads, 0, s>>>(
        k, R, box_stride(c->n), c->gperm.as<int32_t>(), mix->rec.as<float>(),
        c->gbox_u.as<float>(), c->grec.as<float>(), c->gbox.as<float>());
    return hipGetLastError();
}

template <int N>
hipError_t front_body_n(ngd_cull *c, const ngd_mixture *mix, const float *queries,
                        hipStream_t s, bool &side_open)
{
    const int P = c->params.n_proj;
    const int64_t q = c->q, k = c->k;
    const int R = rec_stride(N);
    const int nbits = c->params.key_proj * c->params.key_bits;
    hipError_t e;
    // The Gaussians' projections feed only their own k-d order, which runs
    // on the second stream: with the k-d tiling (and more than one chunk of
    // Gaussians) they go there too, after the fork, so that the queries'
    // projections start at once.
    bool forked = false;
    if (c->params.tiling != 1 && k > kWave) {
        if ((e = hipEventRecord(c->ev_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(c->side, c->ev_fork, 0)) != hipSuccess) return e;
        forked = true;
    }
    if (k > 0) {
        // the forward drops a pair at exp2(-M log2(e) / 2) < tau 2^-margin:
        // its boxes' half-widths are sr sqrt(V_ii)
        const double skip = -std::log2(double(c->params.tau)) + kSkipLog2Margin;
        const double sr = std::sqrt(2.0 * std::log(2.0) * skip) * (1.0 + 0x1p-8);
        k_gauss_proj<N><<<nblk(k, kThreads), kThreads, 0, forked ? c->side : s>>>(
            k, P, mix->rec.as<float>(), R, mix->lfac.as<float>(), c->proj.as<float>(), c->kappa2,
            c->g_mr.as<float>(), c->g_thr.as<float>(), sr, c->gbox_u.as<float>());
    }
    const int64_t nparts = (q + kThreads - 1) / kThreads;
    // With the k-d tiling of the queries the projection kernel's block
    // extents are taken as keys, and their reduction is the root's extents
    // of the queries' k-d order (no pass of its own over the projections).
    const bool kd_queries = c->params.tiling == 0 && q > std::min(c->params.tile, kWave);
    const bool root_keys =
        kd_queries && c->kd_work.ext[0].cap >= sizeof(uint32_t) * 2 * size_t(P);
    if (q > 0) {
        auto go = [&](auto kern) {
            kern<<<nblk(q, kThreads), kThreads, 0, s>>>(q, P, queries, c->proj.as<float>(),
                                                        c->qr.as<float>(),
                                                        c->range_part.as<float>());
        };
        if (root_keys)
            P <= 16 ? go(k_query_proj<N, 16, true>) : go(k_query_proj<N, 32, true>);
        else
            P <= 16 ? go(k_query_proj<N, 16, false>) : go(k_query_proj<N, 32, false>);
    }
    if (root_keys)
        k_root_keys<<<dim3(unsigned(P)), kThreads, 0, s>>>(nparts, P, c->range_part.as<float>(),
                                                           c->kd_work.ext[0].as<uint32_t>());
    else
        k_range_final<<<dim3(unsigned(P)), kThreads, 0, s>>>(nparts, P, c->params.key_bits,
                                                             c->range_part.as<float>(),
                                                             c->qrange.as<float>());
    if ((e = hipGetLastError()) != hipSuccess) {
        if (forked) {   // the main stream still waits for the second one
            (void)hipEventRecord(c->ev_join, c->side);
            (void)hipStreamWaitEvent(s, c->ev_join, 0);
        }
        return e;
    }

    int which = 0;
    // the k-d order leaves the projections in order: tile bounds and the
    // ordered means read them without a gather
    const float *qr_s = nullptr;
    bool g_sorted = false, gauss_done = false;
    if (c->params.tiling != 1) {
        // k-d order of the query projections (runs of `tile`, and of 64
        // inside those; tiling 2: the caller's order, no reordering) and of
        // the projected means (runs of 64, the chunks of the interval test).  The two are independent: the Gaussians'
        // order runs on the second stream, forked before their projections
        // and joined before anything reads it.  Both are enqueued a phase (a
        // level) at a time, alternately, so that each stream has work while
        // the host enqueues the other's.
        KdRun rg, rq;
        if (forked) {   // forked above, behind the Gaussians' projections
            e = kd_start(rg, c->kd_g, c->kd_work_g, P, c->g_mr.as<float>(), k,
                         c->gperm.as<int32_t>(), c->g_mr_s.as<float>(), c->side);
            g_sorted = true;
        } else if (k > 0) {
            k_iota<<<nblk(k, kThreads), kThreads, 0, s>>>(c->gperm.as<int32_t>(), k);
        }
        if (e == hipSuccess && q > 0) {
            if (c->params.tiling == 2 || q <= std::min(c->params.tile, kWave)) {
                k_iota<<<nblk(q, kThreads), kThreads, 0, s>>>(c->perm.as<int32_t>(), q);
            } else {
                e = kd_start(rq, c->kd_q, c->kd_work, P, c->qr.as<float>(), q,
                             c->perm.as<int32_t>(), c->qr_s.as<float>(), s, root_keys);
                qr_s = c->qr_s.as<float>();
            }
        }
        while (e == hipSuccess && !(rq.done && rg.done)) {
            if (!rq.done) e = kd_step(rq);
            if (e == hipSuccess && !rg.done) e = kd_step(rg);
        }
        // the Gaussians' side goes on while the queries' order finishes:
        // first the interval test's limits (the join point), then what only
        // the forward reads -- the ordered records, the boxes and the
        // matrix-core forward's per-Gaussian coefficients -- which the main
        // stream waits for only at the end of the front half
        if (forked && e == hipSuccess) {
            e = gauss_limits(c, k, P, true, c->side);
            gauss_done = true;
        }
        if (forked) {
            const hipError_t ej = hipEventRecord(c->ev_join, c->side);
            if (e == hipSuccess) e = ej;
            if (e == hipSuccess) {
                side_open = true;
                e = gauss_records(c, mix, k, R, c->side);
                if (e == hipSuccess) e = launch_mfma_coef(N, c, c->side);
                c->coef_next = e == hipSuccess;
            }
            if (e != hipSuccess) {
                (void)hipEventRecord(c->ev_join, c->side);
                (void)hipStreamWaitEvent(s, c->ev_join, 0);
                return e;
            }
        }
        if (e != hipSuccess) return e;
    }
    // Morton: queries: keys, sort -> perm
    if (c->params.tiling == 1 && q > 0) {
        k_keys<<<nblk(q, kThreads), kThreads, 0, s>>>(q, P, c->qr.as<float>(),
                                                      c->qrange.as<float>(), c->params.key_proj,
                                                      c->params.key_bits, c->keys0.as<uint32_t>(),
                                                      c->vals0.as<int32_t>());
        e = radix_sort(q, nullptr, nbits, c->keys0, c->keys1, c->vals0, c->vals1, c->radix_hist,
                       c->radix_off, c->scan_tmp, s, &which);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(c->perm.p, which ? c->vals1.p : c->vals0.p, sizeof(int32_t) * q,
                           hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    // Morton: Gaussians: keys of the projected means, sort -> gperm
    if (c->params.tiling == 1 && k > 0) {
        k_keys<<<nblk(k, kThreads), kThreads, 0, s>>>(k, P, c->g_mr.as<float>(),
                                                      c->qrange.as<float>(), c->params.key_proj,
                                                      c->params.key_bits, c->keys0.as<uint32_t>(),
                                                      c->vals0.as<int32_t>());
        e = radix_sort(k, nullptr, nbits, c->keys0, c->keys1, c->vals0, c->vals1, c->radix_hist,
                       c->radix_off, c->scan_tmp, s, &which);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(c->gperm.p, which ? c->vals1.p : c->vals0.p, sizeof(int32_t) * k,
                           hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    // tiles
    const int PP = pad_proj(P);
    if (c->ntiles > 0) {
        const int bt = int(std::min<int64_t>(1024, (int64_t(c->params.tile) + 63) / 64 * 64));
        if (P <= 16)
            k_tile_bounds<N, 16><<<dim3(unsigned(c->ntiles)), bt, 0, s>>>(
                q, c->params.tile, P, PP, c->perm.as<int32_t>(), c->qr.as<float>(), qr_s,
                queries, c->qs.as<float>(), c->tile_lo.as<float>(), c->tile_hi.as<float>(),
                c->tbnd.as<float>(), c->tcen.as<float>());
        else
            k_tile_bounds<N, 32><<<dim3(unsigned(c->ntiles)), bt, 0, s>>>(
                q, c->params.tile, P, PP, c->perm.as<int32_t>(), c->qr.as<float>(), qr_s,
                queries, c->qs.as<float>(), c->tile_lo.as<float>(), c->tile_hi.as<float>(),
                c->tbnd.as<float>(), c->tcen.as<float>());
        const int64_t nsup = (c->ntiles + kSuperTiles - 1) / kSuperTiles;
        k_super_bounds<<<nblk(nsup * 2 * PP, kThreads), kThreads, 0, s>>>(
            c->ntiles, PP, c->tbnd.as<float>(), c->sbnd.as<float>());
    }
    // the tiles' bounds above overlap the second stream's last kernels
    if (side_open && (e = hipStreamWaitEvent(s, c->ev_join, 0)) != hipSuccess) return e;
    if (k > 0 && !gauss_done) {
        if ((e = gauss_limits(c, k, P, g_sorted, s)) != hipSuccess) return e;
        if ((e = gauss_records(c, mix, k, R, s)) != hipSuccess) return e;
    }
    k_zero_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long *>(c->stats.p), 2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (k == 0 || c->ntiles == 0) {
        // no pairs: every tile list is empty
        if (c->ntiles > 0)
            k_zero_i32<<<nblk(c->ntiles, kThreads), kThreads, 0, s>>>(c->tile_cnt.as<int32_t>(),
                                                                     c->ntiles);
        e = scan_counts(c->tile_cnt, c->tile_off, c->ntiles, c->scan_tmp, s);
        if (e != hipSuccess) return e;
        return launch_items(c->ntiles, c->tile_off.as<int64_t>(), kItemCands, c->item_cnt, c->item_off, c->scan_tmp, s);
    }
    // interval test; it also counts the candidates per (chunk segment, tile)
    const int64_t per_seg = (c->nchunks + c->nseg - 1) / c->nseg;
    k_zero_i32<<<nblk(int64_t(c->nseg) * c->ntiles, kThreads), kThreads, 0, s>>>(
        c->seg_cnt.as<int32_t>(), int64_t(c->nseg) * c->ntiles);
    // 128 tiles per wave: the boxes of a wave's range (16 KB at 16
    // projections) stay in the scalar cache while the workgroups that share
    // the range (consecutive chunks, same y) test them; 512 tiles per wave
    // measured 356 us against 301 us here (10-D, 2^20 queries, K = 2^18)
    const int tiles_per_wave = 128;
    dim3 grid(nblk(c->nchunks, kThreads / kWave), nblk(c->ntiles, tiles_per_wave));
#define NGD_CULL_TEST(PPV)                                                                   \
    k_cull_test<PPV><<<grid, kThreads, 0, s>>>(k, c->ntiles, c->tpad, P, tiles_per_wave,      \
                                               c->g_ub.as<float>(), c->g_lb.as<float>(),     \
                                               c->tbnd.as<float>(), c->sbnd.as<float>(),     \
                                               c->masks.as<uint64_t>(), per_seg,              \
                                               c->seg_cnt.as<int32_t>())
    switch (PP) {
    case 4: NGD_CULL_TEST(4); break;
    case 8: NGD_CULL_TEST(8); break;
    case 12: NGD_CULL_TEST(12); break;
    case 16: NGD_CULL_TEST(16); break;
    case 24: NGD_CULL_TEST(24); break;
    default: NGD_CULL_TEST(32); break;
    }
#undef NGD_CULL_TEST
    // per-tile counts -> offsets
    k_seg_prefix<<<nblk(c->ntiles, kThreads), kThreads, 0, s>>>(
        c->ntiles, c->nseg, c->seg_cnt.as<int32_t>(), c->tile_cnt.as<int32_t>(),
        reinterpret_cast<unsigned long long *>(c->stats.as<int64_t>() + 1));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = scan_counts(c->tile_cnt, c->tile_off, c->ntiles, c->scan_tmp, s);
    if (e != hipSuccess) return e;
    return launch_items(c->ntiles, c->tile_off.as<int64_t>(), kItemCands, c->item_cnt, c->item_off, c->scan_tmp, s);
}

template <int N>
hipError_t front_n(ngd_cull *c, const ngd_mixture *mix, const float *queries, hipStream_t s)
{
    bool side_open = false;
    hipError_t e = front_body_n<N>(c, mix, queries, s, side_open);
    if (side_open) {
        // the second stream's work past the interval test's join point ends
        // before the front half does, whatever happened in between
        hipError_t ej = hipEventRecord(c->ev_done, c->side);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(s, c->ev_done, 0);
        if (e == hipSuccess) e = ej;
    }
    return e;
}

}  // namespace

hipError_t launch_cull_build_front(ngd_cull *c, const ngd_mixture *mix, const float *queries,
                                   hipStream_t s)
{
    switch (c->n) {
#define NGD_CASE(NN) \
    case NN: return front_n<NN>(c, mix, queries, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_sizes(ngd_cull *c, hipStream_t s)
{
    k_gather_sizes<<<1, 64, 0, s>>>(c->stats.as<int64_t>(), c->tile_off.as<int64_t>() + c->ntiles,
                                    c->item_off.as<int64_t>() + c->ntiles);
    return hipGetLastError();
}

hipError_t launch_cull_build_lists(ngd_cull *c, hipStream_t s, int64_t cap_ent,
                                   int64_t cap_items)
{
    if (c->ntiles == 0) return hipSuccess;
    if (cap_items > 0)
        k_item_fill<<<nblk(c->ntiles, kThreads), kThreads, 0, s>>>(
            c->ntiles, c->item_off.as<int64_t>(), cap_items, c->item_tile.as<int32_t>());
    if (cap_ent == 0 || c->k == 0) return hipGetLastError();
    const int64_t per_seg = (c->nchunks + c->nseg - 1) / c->nseg;
    dim3 sgrid(nblk(c->ntiles, kFillTiles), unsigned(c->nseg));
    k_fill_cand<<<sgrid, kThreads, 0, s>>>(c->ntiles, c->tpad, c->nchunks, per_seg,
                                           c->masks.as<uint64_t>(), c->seg_cnt.as<int32_t>(),
                                           c->tile_off.as<int64_t>(), cap_ent,
                                           c->cand.as<int32_t>(), c->ent_tile.as<int32_t>());
    return hipGetLastError();
}

hipError_t launch_cull_transpose_full(ngd_cull *c, hipStream_t s)
{
    const int64_t k = c->k;
    hipError_t e;
    if (k > 0) k_zero_i32<<<nblk(k, kThreads), kThreads, 0, s>>>(c->g_cnt.as<int32_t>(), k);
    if (c->total > 0) {
        k_ghist<<<nblk(c->total, kThreads), kThreads, 0, s>>>(c->total, c->cand.as<int32_t>(),
                                                             c->g_cnt.as<int32_t>());
        k_ent_init<<<nblk(c->total, kThreads), kThreads, 0, s>>>(
            c->total, c->cand.as<int32_t>(), c->keys0.as<uint32_t>(), c->vals0.as<int32_t>());
        int nbits = 0;
        while ((int64_t(1) << nbits) < k) ++nbits;
        int which = 0;
        e = radix_sort(c->total, nullptr, nbits, c->keys0, c->keys1, c->vals0, c->vals1, c->radix_hist,
                       c->radix_off, c->scan_tmp, s,
                       &which);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(c->g_ent.p, which ? c->vals1.p : c->vals0.p,
                           sizeof(int32_t) * c->total, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        k_ent_gather<<<nblk(c->total, kThreads), kThreads, 0, s>>>(
            c->total, c->g_ent.as<int32_t>(), c->ent_tile.as<int32_t>(), c->g_tiles.as<int32_t>());
    }
    e = scan_counts(c->g_cnt, c->g_off, k, c->scan_tmp, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

namespace {

// ---- backward preparation -------------------------------------------------
// Entries with at least one kept query group, compacted in entry order and
// then stably sorted by Gaussian: each Gaussian's kept entries in ascending
// tile order, without transposing the (much longer) full candidate lists.
// Whether any 64-query group kept entry e (the flags of its groups, read
// together).
__device__ __forceinline__ bool entry_kept(const uint8_t *__restrict__ act, int64_t e, int groups)
{
    const uint8_t *a = act + e * groups;
    if (groups == 4) return *reinterpret_cast<const uint32_t *>(a) != 0u;   // aligned
    int any = 0;
#pragma unroll
    for (int g = 0; g < 16; ++g)   // groups <= 16 (tiles of at most 1024 queries)
        if (g < groups) any |= a[g];
    return any != 0;
}

// Kept entries per block of kThreads entries.
__global__ __launch_bounds__(kThreads) void k_eflag(int64_t total, int groups,
                                                    const uint8_t *__restrict__ act,
                                                    int32_t *__restrict__ bcnt)
{
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const bool kept = e < total && entry_kept(act, e, groups);
    const int n = __syncthreads_count(kept);
    if (threadIdx.x == 0) bcnt[blockIdx.x] = n;
}

// The kept entries in entry order: block offset (the scan of the block
// counts) plus the rank within the block; keys = sorted Gaussian, values =
// entry, and each Gaussian's count.
__global__ __launch_bounds__(kThreads) void k_ecompact(int64_t total, int groups,
                                                       const uint8_t *__restrict__ act,
                                                       const int64_t *__restrict__ boff,
                                                       const int32_t *__restrict__ cand,
                                                       uint32_t *__restrict__ keys,
                                                       int32_t *__restrict__ vals,
                                                       int32_t *__restrict__ a_cnt)
{
    __shared__ int wcnt[kThreads / kWave];
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const bool kept = e < total && entry_kept(act, e, groups);
    const uint64_t b = ballot(kept);
    const int w = int(threadIdx.x) / kWave;
    if (lane_id() == 0) wcnt[w] = __popcll(b);
    __syncthreads();
    if (!kept) return;
    int before = __popcll(b & lanemask_lt());
    for (int i = 0; i < w; ++i) before += wcnt[i];
    const int64_t o = boff[blockIdx.x] + before;
    const int32_t g = cand[e];
    keys[o] = uint32_t(g);
    vals[o] = int32_t(e);
    atomicAdd(&a_cnt[g], 1);
}

}  // namespace

hipError_t launch_backward_prepare(ngd_cull *c, hipStream_t s)
{
    const int64_t k = c->k, total = c->total;
    const int groups = (c->params.tile + kWave - 1) / kWave;
    if (k > 0) k_zero_i32<<<nblk(k, kThreads), kThreads, 0, s>>>(c->a_cnt.as<int32_t>(), k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (total > 0) {
        // kept entries counted per block of kThreads entries, the block
        // counts scanned (eflag and eoff hold the counts and the offsets),
        // then each kept entry placed at its block's offset plus its rank
        const int64_t nb = (total + kThreads - 1) / kThreads;
        k_eflag<<<unsigned(nb), kThreads, 0, s>>>(total, groups, c->act.as<uint8_t>(),
                                                  c->eflag.as<int32_t>());
        e = scan_counts(c->eflag, c->eoff, nb, c->scan_tmp, s);
        if (e != hipSuccess) return e;
        k_ecompact<<<unsigned(nb), kThreads, 0, s>>>(
            total, groups, c->act.as<uint8_t>(), c->eoff.as<int64_t>(), c->cand.as<int32_t>(),
            c->keys0.as<uint32_t>(), c->vals0.as<int32_t>(), c->a_cnt.as<int32_t>());
        int nbits = 0;
        while ((int64_t(1) << nbits) < k) ++nbits;
        int which = 0;
        // the kept-entry count stays on the device: eoff[nb]
        e = radix_sort(total, c->eoff.as<int64_t>() + nb, nbits, c->keys0, c->keys1, c->vals0,
                       c->vals1, c->radix_hist, c->radix_off, c->scan_tmp, s, &which);
        if (e != hipSuccess) return e;
        c->a_ent_buf = which;
    } else {
        c->a_ent_buf = 0;
    }
    e = scan_counts(c->a_cnt, c->a_off, k, c->scan_tmp, s);
    if (e != hipSuccess) return e;
    e = launch_items(k, c->a_off.as<int64_t>(), kItemTiles, c->gitem_cnt, c->gitem_off, c->scan_tmp, s);
    if (e != hipSuccess) return e;
    if (k > 0 && c->gitems_cap > 0)
        k_item_fill<<<nblk(k, kThreads), kThreads, 0, s>>>(k, c->gitem_off.as<int64_t>(),
                                                           c->gitems_cap,
                                                           c->gitem_g.as<int32_t>());
    return hipGetLastError();
}

bool cull_reserve_lists(ngd_cull *c)
{
    const int64_t tot = c->total > 0 ? c->total : 1;
    const int64_t groups = (c->params.tile + kWave - 1) / kWave;
    const int64_t nb = (tot + kRadixPerBlock - 1) / kRadixPerBlock;
    const int64_t kk = c->k > 0 ? c->k : 1;
    const int64_t T = c->ntiles > 0 ? c->ntiles : 1;
    const size_t nm = size_t(c->n + tri(c->n) + 3);
    bool ok = true;
    ok &= c->cand.ensure(sizeof(int32_t) * tot);
    ok &= c->ent_tile.ensure(sizeof(int32_t) * tot);
    ok &= c->g_ent.ensure(sizeof(int32_t) * tot);
    ok &= c->g_tiles.ensure(sizeof(int32_t) * tot);
    ok &= c->act.ensure(size_t(tot) * size_t(groups));
    // the backward's per-block kept counts and their offsets
    const int64_t nbe = (tot + kThreads - 1) / kThreads;
    ok &= c->eflag.ensure(sizeof(int32_t) * nbe);
    ok &= c->eoff.ensure(sizeof(int64_t) * (nbe + 1));
    ok &= c->a_cnt.ensure(sizeof(int32_t) * kk);
    ok &= c->a_off.ensure(sizeof(int64_t) * (kk + 1));
    ok &= c->keys0.ensure(sizeof(uint32_t) * tot);
    ok &= c->keys1.ensure(sizeof(uint32_t) * tot);
    ok &= c->vals0.ensure(sizeof(int32_t) * tot);
    ok &= c->vals1.ensure(sizeof(int32_t) * tot);
    ok &= c->radix_hist.ensure(sizeof(int32_t) * kRadixMaxBins * nb);
    ok &= c->radix_off.ensure(sizeof(int64_t) * (kRadixMaxBins * nb + 1));
    ok &= c->scan_tmp.ensure(scan_tmp_bytes(std::max<int64_t>({kRadixMaxBins * nb, T, kk, tot})));
    ok &= c->item_tile.ensure(sizeof(int32_t) * size_t(c->nitems > 0 ? c->nitems : 1));
    ok &= c->fpart.ensure(sizeof(float) * 3 * size_t(c->nitems) * size_t(c->params.tile));
    ok &= c->gitem_g.ensure(sizeof(int32_t) * size_t(c->gitems_cap > 0 ? c->gitems_cap : 1));
    ok &= c->gpart.ensure(sizeof(float) * nm * size_t(c->gitems_cap));
    ok &= c->gflag.ensure(sizeof(int32_t) * size_t(c->gitems_cap > 0 ? c->gitems_cap : 1));
    return ok;
}

bool cull_reserve_front(ngd_cull *c)
{
    const int P = c->params.n_proj;
    const int64_t q = c->q, k = c->k, n = c->n;
    const int64_t qq = q > 0 ? q : 1, kk = k > 0 ? k : 1;
    const int64_t T = c->ntiles > 0 ? c->ntiles : 1;
    const int64_t qk = std::max(qq, kk);
    const int64_t nb_sort = (qk + kRadixPerBlock - 1) / kRadixPerBlock;
    const int64_t nparts = (qq + kThreads - 1) / kThreads;
    const int64_t scan_n = std::max<int64_t>({kRadixMaxBins * nb_sort, T, kk});
    bool ok = true;
    ok &= c->proj.ensure(sizeof(float) * P * n);
    ok &= c->qr.ensure(sizeof(float) * P * qq);
    ok &= c->range_part.ensure(sizeof(float) * 2 * P * nparts);
    ok &= c->qrange.ensure(sizeof(float) * 3 * P);
    ok &= c->g_mr.ensure(sizeof(float) * P * kk);
    ok &= c->g_thr.ensure(sizeof(float) * P * kk);
    ok &= c->keys0.ensure(sizeof(uint32_t) * qk);
    ok &= c->keys1.ensure(sizeof(uint32_t) * qk);
    ok &= c->vals0.ensure(sizeof(int32_t) * qk);
    ok &= c->vals1.ensure(sizeof(int32_t) * qk);
    ok &= c->radix_hist.ensure(sizeof(int32_t) * kRadixMaxBins * nb_sort);
    ok &= c->radix_off.ensure(sizeof(int64_t) * (kRadixMaxBins * nb_sort + 1));
    ok &= c->perm.ensure(sizeof(int32_t) * qq);
    ok &= c->gperm.ensure(sizeof(int32_t) * kk);
    ok &= c->qs.ensure(sizeof(float) * n * qq);
    ok &= c->gs.ensure(sizeof(float) * 3 * qq);
    ok &= c->tile_lo.ensure(sizeof(float) * T * P);
    ok &= c->tile_hi.ensure(sizeof(float) * T * P);
    ok &= c->tbnd.ensure(sizeof(float) * T * 2 * pad_proj(P));
    ok &= c->tcen.ensure(sizeof(float) * T * c->n);
    ok &= c->sbnd.ensure(sizeof(float) * ((T + kSuperTiles - 1) / kSuperTiles) * 2 * pad_proj(P));
    if (c->params.tiling == 0) ok &= c->qr_s.ensure(sizeof(float) * P * qq);
    ok &= c->grec.ensure(sizeof(float) * kk * rec_stride(int(n)));
    ok &= c->mrec.ensure(kk * mfma_rec_bytes(int(n)));
    ok &= c->mrow.ensure(sizeof(float) * kk);
    ok &= c->g_mr_s.ensure(sizeof(float) * P * kk);
    ok &= c->g_ub.ensure(sizeof(float) * P * kk);
    ok &= c->gbox.ensure(sizeof(float) * kk * box_stride(int(n)));
    ok &= c->gbox_u.ensure(sizeof(float) * kk * box_stride(int(n)));
    ok &= c->g_lb.ensure(sizeof(float) * P * kk);
    ok &= c->masks.ensure(sizeof(uint64_t) * std::max<int64_t>(c->nchunks, 1) *
                          std::max<int64_t>(c->tpad, 64));
    ok &= c->seg_cnt.ensure(sizeof(int32_t) * c->nseg * T);
    ok &= c->tile_cnt.ensure(sizeof(int32_t) * T);
    ok &= c->tile_off.ensure(sizeof(int64_t) * (T + 1));
    ok &= c->g_cnt.ensure(sizeof(int32_t) * kk);
    ok &= c->g_off.ensure(sizeof(int64_t) * (kk + 1));
    ok &= c->item_cnt.ensure(sizeof(int32_t) * T);
    ok &= c->item_off.ensure(sizeof(int64_t) * (T + 1));
    ok &= c->gitem_cnt.ensure(sizeof(int32_t) * kk);
    ok &= c->gitem_off.ensure(sizeof(int64_t) * (kk + 1));
    ok &= c->scan_tmp.ensure(scan_tmp_bytes(scan_n));
    ok &= c->stats.ensure(sizeof(int64_t) * 4);
    if (c->params.tiling != 1) {
        // the queries' k-d plan only with the k-d tiling (tiling 2 keeps the
        // caller's order); the Gaussians' with both
        if (c->params.tiling == 0)
            ok &= kd_plan(c->kd_q, q, c->params.tile, std::min(c->params.tile, kWave)) &&
                  kd_reserve(c->kd_work, c->kd_q, q, P);
        ok &= kd_plan(c->kd_g, k, kWave, kWave);
        ok = ok && kd_reserve(c->kd_work_g, c->kd_g, k, P);
        if (ok && !c->side) ok = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess;
        if (ok && !c->ev_fork)
            ok = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
        if (ok && !c->ev_join)
            ok = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess;
        if (ok && !c->ev_done)
            ok = hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) == hipSuccess;
    }
    return ok;
}

}  // namespace ngd
