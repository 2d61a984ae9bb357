// Per-pair evaluation shared by the forward kernels (eval.hip,
// eval_mfma.hip): record layout, the staged rows of y = S'(x - m) with the
// certified skip checks, and the uniform record loads.
#pragma once

#include <utility>

#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {

// s_waitcnt immediate that waits for all scalar-memory (and LDS) loads only:
// vmcnt and expcnt at their maxima, lgkmcnt 0.
constexpr int kWaitScalar = 0xC07F;

template <int N> struct RecLayout {
    static constexpr int T = N * (N + 1) / 2;
    static constexpr int R = (N + T + 7 + 3) / 4 * 4;
    static constexpr int AC = N + T;
    static constexpr int PF = R < 32 ? R : 32;   // floats loaded ahead
    static constexpr int K1 = N < 3 ? N : 3;      // stage boundaries
    static constexpr int K2 = N < 6 ? N : 6;
};

// Record field e: from the prefetched block when e < PF, else from memory.
template <int N, int E>
__device__ __forceinline__ float field(const float (&blk)[RecLayout<N>::PF],
                                       const float *__restrict__ r)
{
    if constexpr (E < RecLayout<N>::PF)
        return blk[E];
    else
        return r[E];
}

// Rows [R0, R1) of y = S'(x - m), accumulated into msq; d holds x - m.
template <int N, int R0, int R1>
__device__ __forceinline__ void rows(const float (&blk)[RecLayout<N>::PF],
                                     const float *__restrict__ r, const float (&x)[N],
                                     float (&d)[N], float (&y)[N], float &msq)
{
    if constexpr (R0 < R1) {
        d[R0] = x[R0] - field<N, R0>(blk, r);
        constexpr int base = N + R0 * (R0 + 1) / 2;
        float acc = field<N, base>(blk, r) * d[0];
        [&]<int... J>(std::integer_sequence<int, J...>) {
            ((acc = fmaf(field<N, base + 1 + J>(blk, r), d[1 + J], acc)), ...);
        }(std::make_integer_sequence<int, R0>{});
        y[R0] = acc;
        msq = fmaf(acc, acc, msq);
        rows<N, R0 + 1, R1>(blk, r, x, d, y, msq);
    }
}

// Accumulates one Gaussian into f for this lane's query x.  With SKIP,
// returns early when the whole wave can drop the pair.
// Returns whether the wave kept the pair (the same for every lane).  With
// COUNT, st[0..2] count the pairs that passed the first and second checks
// and were kept (wave-uniform counters).
template <int N, bool SKIP, bool ACC = true, bool COUNT = false>
__device__ __forceinline__ bool eval_pair(const float (&blk)[RecLayout<N>::PF],
                                          const float *__restrict__ r, const float (&x)[N],
                                          bool valid, float skip, float &f0, float &f1,
                                          float &f2, uint32_t *st = nullptr)
{
    using Lay = RecLayout<N>;
    float d[N], y[N];
    float msq = 0.0f;
    rows<N, 0, Lay::K1>(blk, r, x, d, y, msq);
    if constexpr (SKIP && Lay::K1 < N) {
        if (ballot(valid && msq <= skip) == 0) return false;
    }
    if constexpr (COUNT) ++st[0];
    rows<N, Lay::K1, Lay::K2>(blk, r, x, d, y, msq);
    if constexpr (SKIP && Lay::K2 < N && Lay::K1 < Lay::K2) {
        if (ballot(valid && msq <= skip) == 0) return false;
    }
    if constexpr (COUNT) ++st[1];
    rows<N, Lay::K2, N>(blk, r, x, d, y, msq);
    if constexpr (SKIP) {
        if (ballot(valid && msq <= skip) == 0) return false;
    }
    if constexpr (COUNT) ++st[2];
    if constexpr (ACC) {
        const float g = __builtin_amdgcn_exp2f(-msq);
        f0 = fmaf(g, field<N, Lay::AC + 0>(blk, r), f0);
        f1 = fmaf(g, field<N, Lay::AC + 1>(blk, r), f1);
        f2 = fmaf(g, field<N, Lay::AC + 2>(blk, r), f2);
    }
    return true;
}

template <int N>
__device__ __forceinline__ void load_block(float (&blk)[RecLayout<N>::PF],
                                           const float *__restrict__ r)
{
#pragma unroll
    for (int e = 0; e < RecLayout<N>::PF; ++e) blk[e] = r[e];
}

}  // namespace ngd
