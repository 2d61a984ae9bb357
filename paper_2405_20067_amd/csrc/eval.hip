// Forward evaluation of the mixture colour (Sec. 4.1, Eq. 8):
//   f(x) = sum_i exp2(-|S'_i (x - m_i)|^2) alpha_i c_i,  S' = sqrt(log2(e)/2) L^-1
//
// Layout: one lane per query, queries held in registers; the Gaussian being
// evaluated is the same for the whole wave, so its record (mean, S', alpha c)
// is read with wave-uniform loads and feeds the VALU as scalar operands.
//
// Culled kernel: one workgroup per tile (up to 256 lanes per group; larger
// tiles use several groups), looping over the tile's candidate list.  Each
// pair is evaluated in two stages: the first n1 coordinates give the
// Mahalanobis distance of the marginal over those coordinates, a lower
// bound of the full one (the leading block of L^-1 is the inverse of the
// leading block of L).  When no lane of the wave is below the skip
// threshold the rest of the pair is skipped; likewise before the exp.
// The threshold certifies G < tau * 2^-20, so a skipped pair changes f by
// less than that times alpha |c|.
//
// Dense kernel: the plain direct sum over all Gaussians, no skipping.
#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kEvalThreads = 256;

template <int N> constexpr int first_stage_dims() { return N >= 4 ? 4 : N; }

// Accumulates one Gaussian (record r, wave-uniform) into f for this lane's
// query x.  With SKIP, returns early when the wave can skip the pair.
template <int N, bool SKIP>
__device__ __forceinline__ void eval_pair(const float *__restrict__ r, const float (&x)[N],
                                          bool valid, float skip, float &f0, float &f1,
                                          float &f2)
{
    constexpr int N1 = first_stage_dims<N>();
    float d[N];
    float msq = 0.0f;
#pragma unroll
    for (int a = 0; a < N1; ++a) d[a] = x[a] - r[a];
#pragma unroll
    for (int row = 0; row < N1; ++row) {
        const float *srow = r + N + row * (row + 1) / 2;
        float y = srow[0] * d[0];
#pragma unroll
        for (int j = 1; j <= row; ++j) y = fmaf(srow[j], d[j], y);
        msq = fmaf(y, y, msq);
    }
    if constexpr (SKIP && N1 < N) {
        if (ballot(valid && msq <= skip) == 0) return;
    }
#pragma unroll
    for (int a = N1; a < N; ++a) d[a] = x[a] - r[a];
#pragma unroll
    for (int row = N1; row < N; ++row) {
        const float *srow = r + N + row * (row + 1) / 2;
        float y = srow[0] * d[0];
#pragma unroll
        for (int j = 1; j <= row; ++j) y = fmaf(srow[j], d[j], y);
        msq = fmaf(y, y, msq);
    }
    if constexpr (SKIP) {
        if (ballot(valid && msq <= skip) == 0) return;
    }
    constexpr int AC = N + N * (N + 1) / 2;
    const float g = __builtin_amdgcn_exp2f(-msq);
    f0 = fmaf(g, r[AC + 0], f0);
    f1 = fmaf(g, r[AC + 1], f1);
    f2 = fmaf(g, r[AC + 2], f2);
}

template <int N>
__global__ __launch_bounds__(kEvalThreads) void k_eval_dense(int64_t k, int64_t q,
                                                             const float *__restrict__ rec,
                                                             const float *__restrict__ queries,
                                                             float *__restrict__ out)
{
    constexpr int R = (N + N * (N + 1) / 2 + 7 + 3) / 4 * 4;
    const int64_t p = int64_t(blockIdx.x) * kEvalThreads + threadIdx.x;
    const bool valid = p < q;
    float x[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = valid ? queries[p * N + a] : 0.0f;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    for (int64_t i = 0; i < k; ++i) eval_pair<N, false>(rec + i * R, x, valid, 0.0f, f0, f1, f2);
    if (valid) {
        out[p * 3 + 0] = f0;
        out[p * 3 + 1] = f1;
        out[p * 3 + 2] = f2;
    }
}

template <int N>
__global__ __launch_bounds__(kEvalThreads) void k_eval_culled(
    int64_t q, int tile, const float *__restrict__ grec, const float *__restrict__ qs,
    const int64_t *__restrict__ tile_off, const int32_t *__restrict__ cand,
    const int32_t *__restrict__ perm, float skip, float *__restrict__ out)
{
    constexpr int R = (N + N * (N + 1) / 2 + 7 + 3) / 4 * 4;
    const int64_t t = blockIdx.x;
    const int s = int(blockIdx.y) * kEvalThreads + int(threadIdx.x);
    const int64_t p = t * tile + s;
    const bool valid = (s < tile) && (p < q);
    float x[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = valid ? qs[a * q + p] : 0.0f;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    const int64_t e0 = uniform64(tile_off[t]), e1 = uniform64(tile_off[t + 1]);
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t c = uniform(cand[e]);
        eval_pair<N, true>(grec + c * R, x, valid, skip, f0, f1, f2);
    }
    if (valid) {
        const int64_t o = perm[p];
        out[o * 3 + 0] = f0;
        out[o * 3 + 1] = f1;
        out[o * 3 + 2] = f2;
    }
}

template <int N>
hipError_t dense_n(const ngd_mixture *mix, const float *queries, int64_t q, float *out,
                   hipStream_t s)
{
    const unsigned blocks = unsigned((q + kEvalThreads - 1) / kEvalThreads);
    k_eval_dense<N><<<blocks, kEvalThreads, 0, s>>>(mix->k, q, mix->rec.as<float>(), queries, out);
    return hipGetLastError();
}

template <int N>
hipError_t culled_n(const ngd_mixture *mix, const ngd_cull *c, float *out, hipStream_t s)
{
    (void)mix;
    const int tile = c->params.tile;
    const int per = tile < kEvalThreads ? (tile + 63) / 64 * 64 : kEvalThreads;
    dim3 grid(unsigned(c->ntiles), unsigned((tile + kEvalThreads - 1) / kEvalThreads));
    // skip when exp2(-M') < tau 2^-margin, i.e. M' > log2(1/tau) + margin
    const float skip = float(-std::log2(double(c->params.tau)) + kSkipLog2Margin);
    k_eval_culled<N><<<grid, per, 0, s>>>(c->q, tile, c->grec.as<float>(), c->qs.as<float>(),
                                          c->tile_off.as<int64_t>(), c->cand.as<int32_t>(),
                                          c->perm.as<int32_t>(), skip, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval_dense(const ngd_mixture *mix, const float *queries, int64_t q, float *out,
                             hipStream_t s)
{
    if (q == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return dense_n<NN>(mix, queries, q, out, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_eval_culled(const ngd_mixture *mix, const ngd_cull *c, float *out,
                              hipStream_t s)
{
    if (c->q == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return culled_n<NN>(mix, c, out, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ngd
