// Per-Gaussian preparation in float64 (Sec. 3.1, Eq. 2): the precision
// factor S = L^-1 by triangular inversion, and the records the evaluation
// kernels read.  One thread per Gaussian; O(n^3) float64 work each, a few
// microseconds for the whole mixture.
#include "ngd_internal.hpp"

namespace ngd {
namespace {

template <int N>
__global__ __launch_bounds__(256) void k_prepare(int64_t k, const float *__restrict__ mean,
                                                 const float *__restrict__ factor,
                                                 const float *__restrict__ weight,
                                                 const float *__restrict__ colour,
                                                 float *__restrict__ rec,
                                                 float *__restrict__ lfac,
                                                 int *__restrict__ flag)
{
    constexpr int T = N * (N + 1) / 2;
    constexpr int R = (N + T + 7 + 3) / 4 * 4;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= k) return;

    double L[T];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < T; ++e) {
        const float v = factor[i * T + e];
        lfac[i * T + e] = v;
        bad |= !isfinite(v);
        L[e] = v;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) bad |= (L[a * (a + 1) / 2 + a] == 0.0);

    // S = L^-1, column by column: S_jj = 1 / L_jj,
    // S_ij = -(sum_{k=j}^{i-1} L_ik S_kj) S_ii  for i > j
    // (one float64 division per row; S_ii = 1 / L_ii).
    double S[T];
#pragma unroll
    for (int j = 0; j < N; ++j) S[j * (j + 1) / 2 + j] = 1.0 / L[j * (j + 1) / 2 + j];
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int r = j + 1; r < N; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int c = j; c < r; ++c) acc = fma(L[r * (r + 1) / 2 + c], S[c * (c + 1) / 2 + j], acc);
            S[r * (r + 1) / 2 + j] = -acc * S[r * (r + 1) / 2 + r];
        }
    }

    float *out = rec + i * R;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const float m = mean[i * N + a];
        bad |= !isfinite(m);
        out[a] = m;
    }
#pragma unroll
    for (int e = 0; e < T; ++e) out[N + e] = static_cast<float>(S[e] * kSqrtHalfLog2e);
    const float alpha = weight[i];
    bad |= !isfinite(alpha);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float c = colour[i * 3 + ch];
        bad |= !isfinite(c);
        out[N + T + ch] = alpha * c;
        out[N + T + 4 + ch] = c;
    }
    out[N + T + 3] = alpha;
#pragma unroll
    for (int e = N + T + 7; e < R; ++e) out[e] = 0.0f;
    if (bad) atomicOr(flag, 1);
}

__global__ void k_clear_flag(int *flag) { *flag = 0; }

template <int N>
hipError_t prepare_n(int64_t k, const float *mean, const float *factor, const float *weight,
                     const float *colour, float *rec, float *lfac, int *flag, hipStream_t s)
{
    const int64_t blocks = (k + 255) / 256;
    k_prepare<N><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(k, mean, factor, weight, colour,
                                                             rec, lfac, flag);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_clear_flag(int *flag, hipStream_t s)
{
    k_clear_flag<<<1, 1, 0, s>>>(flag);
    return hipGetLastError();
}

hipError_t launch_prepare(int n, int64_t k, const float *mean, const float *factor,
                          const float *weight, const float *colour, float *rec, float *lfac,
                          int *flag, hipStream_t s, bool clear_flag)
{
    hipError_t e = clear_flag ? launch_clear_flag(flag, s) : hipSuccess;
    if (e != hipSuccess || k == 0) return e;
    switch (n) {
#define NGD_CASE(NN) \
    case NN: return prepare_n<NN>(k, mean, factor, weight, colour, rec, lfac, flag, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ngd
