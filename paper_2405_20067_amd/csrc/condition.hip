// Conditioning of every Gaussian of a mixture on fixed values of its
// trailing dimensions (the paper's global conditioning, Sec. 3.2: when all
// inputs but the world position are constant over an image, the N-D
// Gaussians are conditioned on them and culled and evaluated as 3-D ones).
// With V = L L^T split into the kept dimensions 0..p-1 and the fixed ones
// p..n-1, the textbook Schur complement gives, for every x_p,
//   G_n(x_p, x_c) = exp(-M_c / 2) G_p(x_p),
//   G_p: mean  m_p + V_pc V_cc^-1 (x_c - m_c),
//        cov   V_pp - V_pc V_cc^-1 V_cp,
//   M_c = (x_c - m_c)^T V_cc^-1 (x_c - m_c),
// so the conditioned mixture (weights alpha exp(-M_c / 2), colours as they
// are) takes the same values over x_p as the N-D one at (x_p, x_c).
// Float64 throughout, one thread per Gaussian: V_cc = F F^T (Cholesky),
// w = F^-1 (x_c - m_c), Z = F^-1 V_cp, cov = V_pp - Z^T Z, mean = m_p + Z^T w,
// and the output factor is the Cholesky factor of cov.
#include "ngd_internal.hpp"

namespace ngd {
namespace {

constexpr int kThreads = 128;

struct CondArgs {
    float xc[NGD_MAX_N];
};

template <int N>
__global__ __launch_bounds__(kThreads) void k_condition(
    int64_t k, int p, CondArgs args, const float *__restrict__ rec,
    const float *__restrict__ lfac, float *__restrict__ mean_out,
    float *__restrict__ factor_out, float *__restrict__ weight_out,
    float *__restrict__ colour_out)
{
    constexpr int T = N * (N + 1) / 2;
    constexpr int R = (N + T + 7 + 3) / 4 * 4;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= k) return;
    const int nc = N - p;
    const int tp = p * (p + 1) / 2;
    double L[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) L[r][c] = c <= r ? double(lfac[i * T + r * (r + 1) / 2 + c]) : 0.0;
    const float *rc = rec + i * R;
    // V = L L^T (symmetric; the lower triangle suffices)
    double V[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q <= c; ++q) acc = fma(L[r][q], L[c][q], acc);
            V[r][c] = acc;
            V[c][r] = acc;
        }
    bool bad = false;
    // Cholesky of V_cc (rows / columns p..n-1) into F
    double F[N][N];
    for (int a = 0; a < nc; ++a) {
        for (int b = 0; b <= a; ++b) {
            double acc = V[p + a][p + b];
            for (int q = 0; q < b; ++q) acc -= F[a][q] * F[b][q];
            if (a == b) {
                bad |= !(acc > 0.0);
                F[a][a] = sqrt(acc > 0.0 ? acc : 1.0);
            } else {
                F[a][b] = acc / F[b][b];
            }
        }
    }
    // w = F^-1 (x_c - m_c), Z = F^-1 V_cp
    double w[N], Z[N][N];
    double mc = 0.0;
    for (int a = 0; a < nc; ++a) {
        double acc = double(args.xc[a]) - double(rc[p + a]);
        for (int q = 0; q < a; ++q) acc -= F[a][q] * w[q];
        w[a] = acc / F[a][a];
        mc = fma(w[a], w[a], mc);
        for (int j = 0; j < p; ++j) {
            double z = V[p + a][j];
            for (int q = 0; q < a; ++q) z -= F[a][q] * Z[q][j];
            Z[a][j] = z / F[a][a];
        }
    }
    // conditional covariance and mean
    double S[N][N];
    for (int r = 0; r < p; ++r) {
        double mu = double(rc[r]);
        for (int q = 0; q < nc; ++q) mu = fma(Z[q][r], w[q], mu);
        mean_out[i * p + r] = float(mu);
        for (int c = 0; c <= r; ++c) {
            double acc = V[r][c];
            for (int q = 0; q < nc; ++q) acc -= Z[q][r] * Z[q][c];
            S[r][c] = acc;
        }
    }
    // its Cholesky factor (positive diagonal)
    double G[N][N];
    for (int r = 0; r < p; ++r)
        for (int c = 0; c <= r; ++c) {
            double acc = S[r][c];
            for (int q = 0; q < c; ++q) acc -= G[r][q] * G[c][q];
            if (r == c) {
                bad |= !(acc > 0.0);
                G[r][r] = sqrt(acc > 0.0 ? acc : 1.0);
            } else {
                G[r][c] = acc / G[c][c];
            }
            factor_out[i * tp + r * (r + 1) / 2 + c] = float(G[r][c]);
        }
    const double alpha = double(rc[N + T + 3]);
    weight_out[i] = float(alpha * exp(-0.5 * mc));
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) colour_out[i * 3 + ch] = rc[N + T + 4 + ch];
    if (bad) {
        // a conditional covariance that is not positive in float64: the
        // output factor gets a zero diagonal, which ngd_mixture_update of the
        // conditioned mixture reports (ngd_mixture_validate: NGD_E_SINGULAR)
        for (int r = 0; r < p; ++r) factor_out[i * tp + r * (r + 1) / 2 + r] = 0.0f;
    }
}

template <int N>
hipError_t condition_n(const ngd_mixture *mix, int p, const CondArgs &a, float *mean_out,
                       float *factor_out, float *weight_out, float *colour_out, hipStream_t s)
{
    k_condition<N><<<unsigned((mix->k + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        mix->k, p, a, mix->rec.as<float>(), mix->lfac.as<float>(), mean_out, factor_out,
        weight_out, colour_out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_condition(const ngd_mixture *mix, int p, const float *xc, float *mean_out,
                            float *factor_out, float *weight_out, float *colour_out,
                            hipStream_t s)
{
    if (mix->k == 0) return hipSuccess;
    CondArgs a{};
    for (int j = 0; j < mix->n - p; ++j) a.xc[j] = xc[j];
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return condition_n<NN>(mix, p, a, mean_out, factor_out, weight_out, colour_out, s);
        NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ngd
