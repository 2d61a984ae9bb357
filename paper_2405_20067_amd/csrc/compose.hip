// Parent-child composition of the refinement (Sec. 3.3, Eq. 6-7) inside the
// library: a child j of parent p is given relative to its parent's frame by
// a lower-triangular factor U_j and an offset m_u,j,
//   L_c = L_p U_j,    m_c = L_p m_u,j + m_p,
// so that the child follows every update of its parent.  k_compose forms
// the absolute parameters of every Gaussian (parents copied, children
// composed in float64 and rounded to float32) ahead of the usual float64
// preparation; the children are then ordinary Gaussians for the cull and the
// forward.  The backward takes the gradients with respect to the absolute
// parameters and applies the chain rule of the product:
//   dU = tril(L_p^T dL_c),   dm_u = L_p^T dm_c,
//   dL_p += tril(dL_c U^T + dm_c m_u^T),   dm_p += dm_c,
// the parents' sums formed per parent over its children in ascending order
// (the parent indices are non-decreasing), without atomics.
#include "ngd_internal.hpp"

namespace ngd {
namespace {

constexpr int kThreads = 256;

template <int N> constexpr int tix(int r, int c) { return r * (r + 1) / 2 + c; }

// One thread per Gaussian.  flag bit 2: a parent index out of [0, kp) or
// smaller than its predecessor's.
template <int N>
__global__ __launch_bounds__(kThreads) void k_compose(
    int64_t k, int64_t kp, const float *__restrict__ mean, const float *__restrict__ factor,
    const int32_t *__restrict__ parent, const float *__restrict__ rel_factor,
    const float *__restrict__ rel_mean, float *__restrict__ abs_mean,
    float *__restrict__ abs_factor, int *__restrict__ flag)
{
    constexpr int T = N * (N + 1) / 2;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= k) return;
    if (i < kp) {
#pragma unroll
        for (int a = 0; a < N; ++a) abs_mean[i * N + a] = mean[i * N + a];
#pragma unroll
        for (int e = 0; e < T; ++e) abs_factor[i * T + e] = factor[i * T + e];
        return;
    }
    const int64_t j = i - kp;
    const int32_t p = parent[j];
    const bool ok = p >= 0 && p < kp && (j == 0 || parent[j - 1] <= p);
    if (!ok) {
        // reported by ngd_mixture_validate; the child becomes a unit
        // Gaussian at the origin, so that everything downstream stays finite
        atomicOr(flag, 2);
#pragma unroll
        for (int a = 0; a < N; ++a) abs_mean[i * N + a] = 0.0f;
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) abs_factor[i * T + tix<N>(r, c)] = r == c ? 1.0f : 0.0f;
        return;
    }
    double lp[T], u[T], mu[N];
#pragma unroll
    for (int e = 0; e < T; ++e) {
        lp[e] = factor[int64_t(p) * T + e];
        u[e] = rel_factor[j * T + e];
    }
#pragma unroll
    for (int a = 0; a < N; ++a) mu[a] = rel_mean[j * N + a];
    // products of float32 values are exact in float64; each sum runs in
    // ascending order of the inner index
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int q = c; q <= r; ++q) acc += lp[tix<N>(r, q)] * u[tix<N>(q, c)];
            abs_factor[i * T + tix<N>(r, c)] = float(acc);
        }
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q <= r; ++q) acc += lp[tix<N>(r, q)] * mu[q];
        abs_mean[i * N + r] = float(acc + double(mean[int64_t(p) * N + r]));
    }
}

// One thread per child: its relative gradients, and what it adds to its
// parent's (stored per child for k_parent_sum).
template <int N>
__global__ __launch_bounds__(kThreads) void k_compose_backward(
    int64_t kc, int64_t kp, const int32_t *__restrict__ parent,
    const float *__restrict__ factor_p, const float *__restrict__ rel_factor,
    const float *__restrict__ rel_mean, const float *__restrict__ g_abs_mean,
    const float *__restrict__ g_abs_factor, float *__restrict__ g_rel_factor,
    float *__restrict__ g_rel_mean, float *__restrict__ contrib)
{
    constexpr int T = N * (N + 1) / 2;
    const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= kc) return;
    const int64_t p = parent[j], c = kp + j;
    if (p < 0 || p >= kp) {   // flagged by k_compose; nothing is read out of range
        for (int e = 0; e < T; ++e) g_rel_factor[j * T + e] = 0.0f;
        for (int a = 0; a < N; ++a) g_rel_mean[j * N + a] = 0.0f;
        for (int e = 0; e < N + T; ++e) contrib[j * (N + T) + e] = 0.0f;
        return;
    }
    double lp[T], u[T], mu[N], gl[T], gm[N];
#pragma unroll
    for (int e = 0; e < T; ++e) {
        lp[e] = factor_p[p * T + e];
        u[e] = rel_factor[j * T + e];
        gl[e] = g_abs_factor[c * T + e];
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        mu[a] = rel_mean[j * N + a];
        gm[a] = g_abs_mean[c * N + a];
    }
    float *out = contrib + j * (N + T);
#pragma unroll
    for (int r = 0; r < N; ++r) {
        // dm_u = L_p^T dm_c
        double a = 0.0;
#pragma unroll
        for (int q = r; q < N; ++q) a += lp[tix<N>(q, r)] * gm[q];
        g_rel_mean[j * N + r] = float(a);
        out[r] = float(gm[r]);   // dm_p += dm_c
#pragma unroll
        for (int cc = 0; cc <= r; ++cc) {
            // dU = tril(L_p^T dL_c)
            double b = 0.0;
#pragma unroll
            for (int q = r; q < N; ++q) b += lp[tix<N>(q, r)] * gl[tix<N>(q, cc)];
            g_rel_factor[j * T + tix<N>(r, cc)] = float(b);
            // dL_p += tril(dL_c U^T + dm_c m_u^T)
            double d = gm[r] * mu[cc];
#pragma unroll
            for (int q = 0; q <= cc; ++q) d += gl[tix<N>(r, q)] * u[tix<N>(cc, q)];
            out[N + tix<N>(r, cc)] = float(d);
        }
    }
}

// One thread per parent: its own gradient plus its children's shares, the
// children found by binary search in the non-decreasing parent indices.
template <int N>
__global__ __launch_bounds__(kThreads) void k_parent_sum(
    int64_t kp, int64_t kc, const int32_t *__restrict__ parent,
    const float *__restrict__ g_abs_mean, const float *__restrict__ g_abs_factor,
    const float *__restrict__ contrib, float *__restrict__ g_mean, float *__restrict__ g_factor)
{
    constexpr int T = N * (N + 1) / 2;
    const int64_t p = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (p >= kp) return;
    int64_t lo = 0, hi = kc;   // first child with parent >= p
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (parent[mid] < p) lo = mid + 1; else hi = mid;
    }
    float gm[N], gl[T];
#pragma unroll
    for (int a = 0; a < N; ++a) gm[a] = g_abs_mean[p * N + a];
#pragma unroll
    for (int e = 0; e < T; ++e) gl[e] = g_abs_factor[p * T + e];
    for (int64_t j = lo; j < kc && parent[j] == p; ++j) {
        const float *cj = contrib + j * (N + T);
#pragma unroll
        for (int a = 0; a < N; ++a) gm[a] += cj[a];
#pragma unroll
        for (int e = 0; e < T; ++e) gl[e] += cj[N + e];
    }
#pragma unroll
    for (int a = 0; a < N; ++a) g_mean[p * N + a] = gm[a];
#pragma unroll
    for (int e = 0; e < T; ++e) g_factor[p * T + e] = gl[e];
}

template <int N>
hipError_t compose_n(int64_t k, int64_t kp, const float *mean, const float *factor,
                     const int32_t *parent, const float *rel_factor, const float *rel_mean,
                     float *abs_mean, float *abs_factor, int *flag, hipStream_t s)
{
    k_compose<N><<<unsigned((k + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        k, kp, mean, factor, parent, rel_factor, rel_mean, abs_mean, abs_factor, flag);
    return hipGetLastError();
}

template <int N>
hipError_t compose_backward_n(int64_t kp, int64_t kc, const int32_t *parent,
                              const float *factor_p, const float *rel_factor,
                              const float *rel_mean, const float *g_abs_mean,
                              const float *g_abs_factor, float *g_mean, float *g_factor,
                              float *g_rel_factor, float *g_rel_mean, float *contrib,
                              hipStream_t s)
{
    if (kc > 0)
        k_compose_backward<N><<<unsigned((kc + kThreads - 1) / kThreads), kThreads, 0, s>>>(
            kc, kp, parent, factor_p, rel_factor, rel_mean, g_abs_mean, g_abs_factor,
            g_rel_factor, g_rel_mean, contrib);
    if (kp > 0)
        k_parent_sum<N><<<unsigned((kp + kThreads - 1) / kThreads), kThreads, 0, s>>>(
            kp, kc, parent, g_abs_mean, g_abs_factor, contrib, g_mean, g_factor);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_compose(int n, int64_t k, int64_t kp, const float *mean, const float *factor,
                          const int32_t *parent, const float *rel_factor, const float *rel_mean,
                          float *abs_mean, float *abs_factor, int *flag, hipStream_t s)
{
    if (k == 0) return hipSuccess;
    switch (n) {
#define NGD_CASE(NN) \
    case NN: return compose_n<NN>(k, kp, mean, factor, parent, rel_factor, rel_mean, abs_mean, \
                                  abs_factor, flag, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_compose_backward(int n, int64_t kp, int64_t kc, const int32_t *parent,
                                   const float *factor_p, const float *rel_factor,
                                   const float *rel_mean, const float *g_abs_mean,
                                   const float *g_abs_factor, float *g_mean, float *g_factor,
                                   float *g_rel_factor, float *g_rel_mean, float *contrib,
                                   hipStream_t s)
{
    switch (n) {
#define NGD_CASE(NN) \
    case NN: return compose_backward_n<NN>(kp, kc, parent, factor_p, rel_factor, rel_mean,   \
                                           g_abs_mean, g_abs_factor, g_mean, g_factor,       \
                                           g_rel_factor, g_rel_mean, contrib, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ngd
