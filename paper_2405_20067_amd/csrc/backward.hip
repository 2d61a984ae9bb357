// Analytic backward pass (Sec. 4.1): gradients of every Gaussian's mean,
// factor, weight and colour given g = dl/df.
//
// With y = L^-1 d (d = x - m), G = exp(-|y|^2/2), s = g . c, w = alpha G s,
// z = L^-T y:
//   dl/dalpha = c . H,  dl/dc = alpha H,        H  = sum_x G g
//   dl/dm     = L^-T B1 = S^T B1,               B1 = sum_x w y
//   dl/dL     = tril(S^T B2),                   B2 = sum_x w y y^T
// (dl/dm = sum w z and dl/dL = tril(sum w z y^T) with z = S^T y.)
//
// Atomics-free, Gaussian-major: one wave owns one Gaussian and walks the
// tiles whose candidate list holds it, 64 queries per step; the wave keeps
// its per-lane partial moments in registers (B1: n, B2: n(n+1)/2, H: 3) and
// reduces them across lanes once at the end, in a fixed order.  Exp terms
// are recomputed, not stored.  Skipping uses the same two-stage certified
// bound and threshold as the forward kernel, so forward and backward sum
// over the same pairs.
#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kBwdThreads = 256;
constexpr int kWavesPerBlock = kBwdThreads / kWave;

template <int N> constexpr int first_stage_dims() { return N >= 4 ? 4 : N; }

template <int N, bool CULLED>
__global__ __launch_bounds__(kBwdThreads) void k_backward(
    int64_t k, int64_t q, int tile, const float *__restrict__ rec,
    const float *__restrict__ xq,          // culled: n x q sorted SoA; dense: q x n
    const float *__restrict__ gq,          // culled: 3 x q sorted SoA; dense: q x 3
    const int64_t *__restrict__ g_off, const int32_t *__restrict__ g_tiles,
    const int32_t *__restrict__ gperm, float skip, float *__restrict__ g_mean,
    float *__restrict__ g_factor, float *__restrict__ g_weight, float *__restrict__ g_colour)
{
    constexpr int T = N * (N + 1) / 2;
    constexpr int R = (N + T + 7 + 3) / 4 * 4;
    constexpr int N1 = CULLED ? first_stage_dims<N>() : N;
    constexpr int AL = N + T + 3, CO = N + T + 4;
    const int lane = lane_id();
    const int64_t sgi = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
    if (sgi >= k) return;
    const float *__restrict__ r = rec + uniform64(sgi) * R;
    const float alpha = r[AL], c0 = r[CO], c1 = r[CO + 1], c2 = r[CO + 2];

    float b1[N], b2[T], h0 = 0.0f, h1 = 0.0f, h2 = 0.0f;
#pragma unroll
    for (int a = 0; a < N; ++a) b1[a] = 0.0f;
#pragma unroll
    for (int e = 0; e < T; ++e) b2[e] = 0.0f;
    bool any = false;

    int64_t e0 = 0, e1 = 1;
    if constexpr (CULLED) {
        e0 = uniform64(g_off[sgi]);
        e1 = uniform64(g_off[sgi + 1]);
    }
    const int64_t span = CULLED ? tile : q;
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t base = CULLED ? int64_t(uniform(g_tiles[e])) * tile : 0;
        for (int64_t g0 = 0; g0 < span; g0 += kWave) {
            const int64_t sidx = g0 + lane;
            const int64_t p = base + sidx;
            const bool valid = (sidx < span) && (p < q);
            float x[N], d[N], y[N];
            float msq = 0.0f;
#pragma unroll
            for (int a = 0; a < N1; ++a) {
                x[a] = valid ? (CULLED ? xq[a * q + p] : xq[p * N + a]) : 0.0f;
                d[a] = x[a] - r[a];
            }
#pragma unroll
            for (int row = 0; row < N1; ++row) {
                const float *srow = r + N + row * (row + 1) / 2;
                float acc = srow[0] * d[0];
#pragma unroll
                for (int j = 1; j <= row; ++j) acc = fmaf(srow[j], d[j], acc);
                y[row] = acc;
                msq = fmaf(acc, acc, msq);
            }
            if constexpr (CULLED && N1 < N) {
                if (ballot(valid && msq <= skip) == 0) continue;
            }
#pragma unroll
            for (int a = N1; a < N; ++a) {
                x[a] = valid ? (CULLED ? xq[a * q + p] : xq[p * N + a]) : 0.0f;
                d[a] = x[a] - r[a];
            }
#pragma unroll
            for (int row = N1; row < N; ++row) {
                const float *srow = r + N + row * (row + 1) / 2;
                float acc = srow[0] * d[0];
#pragma unroll
                for (int j = 1; j <= row; ++j) acc = fmaf(srow[j], d[j], acc);
                y[row] = acc;
                msq = fmaf(acc, acc, msq);
            }
            if constexpr (CULLED) {
                if (ballot(valid && msq <= skip) == 0) continue;
            }
            any = true;
            const float G = valid ? __builtin_amdgcn_exp2f(-msq) : 0.0f;
            float g0v = 0.0f, g1v = 0.0f, g2v = 0.0f;
            if (valid) {
                if constexpr (CULLED) {
                    g0v = gq[p];
                    g1v = gq[q + p];
                    g2v = gq[2 * q + p];
                } else {
                    g0v = gq[p * 3 + 0];
                    g1v = gq[p * 3 + 1];
                    g2v = gq[p * 3 + 2];
                }
            }
            const float sdot = fmaf(g2v, c2, fmaf(g1v, c1, g0v * c0));
            const float w = alpha * G * sdot;
            h0 = fmaf(G, g0v, h0);
            h1 = fmaf(G, g1v, h1);
            h2 = fmaf(G, g2v, h2);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const float wy = w * y[a];
                b1[a] += wy;
#pragma unroll
                for (int b = 0; b <= a; ++b) b2[a * (a + 1) / 2 + b] = fmaf(wy, y[b], b2[a * (a + 1) / 2 + b]);
            }
        }
    }

    const int64_t gi = CULLED ? int64_t(gperm[sgi]) : sgi;
    if (!any) {
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < N; ++a) g_mean[gi * N + a] = 0.0f;
#pragma unroll
            for (int e = 0; e < T; ++e) g_factor[gi * T + e] = 0.0f;
            g_weight[gi] = 0.0f;
            g_colour[gi * 3 + 0] = 0.0f;
            g_colour[gi * 3 + 1] = 0.0f;
            g_colour[gi * 3 + 2] = 0.0f;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) b1[a] = wave_sum(b1[a]);
#pragma unroll
    for (int e = 0; e < T; ++e) b2[e] = wave_sum(b2[e]);
    h0 = wave_sum(h0);
    h1 = wave_sum(h1);
    h2 = wave_sum(h2);
    if (lane != 0) return;
    // S = S' / sqrt(c), y = y' / sqrt(c), c = log2(e)/2:
    //   S^T B1 = S'^T B1' / c,  S^T B2 = S'^T B2' / c^1.5
    const float inv_c = float(1.0 / kHalfLog2e);
    const float inv_c15 = float(1.0 / (kHalfLog2e * kSqrtHalfLog2e));
#pragma unroll
    for (int a = 0; a < N; ++a) {
        float acc = 0.0f;
#pragma unroll
        for (int kk = a; kk < N; ++kk) acc = fmaf(r[N + kk * (kk + 1) / 2 + a], b1[kk], acc);
        g_mean[gi * N + a] = acc * inv_c;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            float acc = 0.0f;
#pragma unroll
            for (int kk = a; kk < N; ++kk)
                acc = fmaf(r[N + kk * (kk + 1) / 2 + a], b2[kk * (kk + 1) / 2 + b], acc);
            g_factor[gi * T + a * (a + 1) / 2 + b] = acc * inv_c15;
        }
    }
    g_weight[gi] = fmaf(c2, h2, fmaf(c1, h1, c0 * h0));
    g_colour[gi * 3 + 0] = alpha * h0;
    g_colour[gi * 3 + 1] = alpha * h1;
    g_colour[gi * 3 + 2] = alpha * h2;
}

__global__ __launch_bounds__(256) void k_gather_grad(int64_t q, const int32_t *__restrict__ perm,
                                                     const float *__restrict__ grad_out,
                                                     float *__restrict__ gs)
{
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= q) return;
    const int64_t o = perm[p];
    gs[p] = grad_out[o * 3 + 0];
    gs[q + p] = grad_out[o * 3 + 1];
    gs[2 * q + p] = grad_out[o * 3 + 2];
}

template <int N>
hipError_t dense_n(const ngd_mixture *mix, const float *queries, int64_t q,
                   const float *grad_out, float *gm, float *gf, float *gw, float *gc,
                   hipStream_t s)
{
    const unsigned blocks = unsigned((mix->k + kWavesPerBlock - 1) / kWavesPerBlock);
    k_backward<N, false><<<blocks, kBwdThreads, 0, s>>>(mix->k, q, 0, mix->rec.as<float>(),
                                                       queries, grad_out, nullptr, nullptr,
                                                       nullptr, 0.0f, gm, gf, gw, gc);
    return hipGetLastError();
}

template <int N>
hipError_t culled_n(const ngd_mixture *mix, ngd_cull *c, const float *grad_out, float *gm,
                    float *gf, float *gw, float *gc, hipStream_t s)
{
    if (c->q > 0) {
        k_gather_grad<<<unsigned((c->q + 255) / 256), 256, 0, s>>>(
            c->q, c->perm.as<int32_t>(), grad_out, c->gs.as<float>());
    }
    const float skip = float(-std::log2(double(c->params.tau)) + kSkipLog2Margin);
    const unsigned blocks = unsigned((mix->k + kWavesPerBlock - 1) / kWavesPerBlock);
    k_backward<N, true><<<blocks, kBwdThreads, 0, s>>>(
        mix->k, c->q, c->params.tile, c->grec.as<float>(), c->qs.as<float>(), c->gs.as<float>(),
        c->g_off.as<int64_t>(), c->g_tiles.as<int32_t>(), c->gperm.as<int32_t>(), skip, gm, gf,
        gw, gc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward_dense(const ngd_mixture *mix, const float *queries, int64_t q,
                                 const float *grad_out, float *g_mean, float *g_factor,
                                 float *g_weight, float *g_colour, hipStream_t s)
{
    if (mix->k == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return dense_n<NN>(mix, queries, q, grad_out, g_mean, g_factor, g_weight, g_colour, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_culled(const ngd_mixture *mix, ngd_cull *c, const float *grad_out,
                                  float *g_mean, float *g_factor, float *g_weight,
                                  float *g_colour, hipStream_t s)
{
    if (mix->k == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return culled_n<NN>(mix, c, grad_out, g_mean, g_factor, g_weight, g_colour, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ngd
