// Wavefront (64-lane) primitives for gfx950: DPP prefix scans, ballots and
// butterfly reductions.  Device code only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ngd {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool pred)
{
    return __builtin_amdgcn_ballot_w64(pred);
}

// Mask of the lanes below the calling lane.
__device__ __forceinline__ uint64_t lanemask_lt()
{
    return (uint64_t(1) << lane_id()) - 1;
}

// Workgroups are dispatched to the 8 XCDs of the chip in turn (workgroup b
// to XCD b mod 8), and each XCD has its own L2.  xcd_block maps the
// dispatch index b of a grid of nb workgroups to a logical index so that
// every XCD takes one contiguous range of the logical order (neighbouring
// tiles or entries, which share Gaussians, then share an L2).  A bijection
// of [0, nb).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t q = nb / kXcds, r = nb % kXcds;
    const int64_t x = b % kXcds, i = b / kXcds;
    return x * q + (x < r ? x : r) + i;
}

// DPP controls (GFX9 encoding).
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// Inclusive prefix sum over the 64 lanes of the wave (all lanes active).
// Within each row of 16 lanes a Hillis-Steele scan over row_shr 1, 2, 4, 8
// (lanes shifted in from outside the row read 0), then row_bcast 15 carries
// row 0 into row 1 and row 2 into row 3, and row_bcast 31 carries lanes
// 0..31 into rows 2 and 3.
__device__ __forceinline__ int wave_inclusive_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast31, 0xc, 0xf, false);
    return x;
}

// Value of lane 63 (the wave total after an inclusive scan).
__device__ __forceinline__ int wave_last(int x)
{
    return __builtin_amdgcn_readlane(x, 63);
}

// Sum over the wave, identical in every lane (xor butterfly: each step adds
// the same two operands in every lane pair, so the result is one value).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// Maximum over the wave of non-negative floats by DPP, the same in every
// lane: the bit patterns of non-negative floats order as unsigned integers
// as the floats do; a running max over row_shr 1, 2, 4, 8 and row_bcast 15,
// 31 (lanes shifted in read 0, the identity) leaves the total in lane 63.
template <int CTRL, int ROWS> __device__ __forceinline__ uint32_t dpp_umax(uint32_t x)
{
    const uint32_t y = uint32_t(__builtin_amdgcn_update_dpp(0, int(x), CTRL, ROWS, 0xf, false));
    return x > y ? x : y;
}

__device__ __forceinline__ float wave_max_nonneg(float v)
{
    uint32_t x = __float_as_uint(v);
    x = dpp_umax<kDppRowShr1, 0xf>(x);
    x = dpp_umax<kDppRowShr2, 0xf>(x);
    x = dpp_umax<kDppRowShr4, 0xf>(x);
    x = dpp_umax<kDppRowShr8, 0xf>(x);
    x = dpp_umax<kDppRowBcast15, 0xa>(x);
    x = dpp_umax<kDppRowBcast31, 0xc>(x);
    return __uint_as_float(uint32_t(__builtin_amdgcn_readlane(int(x), 63)));
}

// Sum over the wave by DPP (no LDS traffic), valid in lane 63 only: the
// inclusive-scan steps of wave_inclusive_scan on floats.  A fixed order, so
// bitwise reproducible.
template <int CTRL, int ROWS> __device__ __forceinline__ float dpp_add(float x)
{
    const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xf, false);
    return x + __int_as_float(y);
}

__device__ __forceinline__ float wave_sum_last(float v)
{
    v = dpp_add<kDppRowShr1, 0xf>(v);
    v = dpp_add<kDppRowShr2, 0xf>(v);
    v = dpp_add<kDppRowShr4, 0xf>(v);
    v = dpp_add<kDppRowShr8, 0xf>(v);
    v = dpp_add<kDppRowBcast15, 0xa>(v);
    v = dpp_add<kDppRowBcast31, 0xc>(v);
    return v;
}

// Sums over the wave of V values per lane (V a multiple of 4), scattered:
// a permlane swap across lane distance 32 halves the values each lane
// holds (lanes 0-31 keep the first half, 32-63 the second, each adding its
// partner's), one across distance 16 halves them again within each half,
// and a DPP running sum within each row of 16 lanes completes them.  Lane
// 16 r + 15 then holds the totals of values [r V/4, (r + 1) V/4) in
// v[0 .. V/4).  A fixed order: bitwise reproducible.
template <int V> __device__ __forceinline__ void wave_reduce_scatter(float (&v)[V])
{
    static_assert(V % 4 == 0, "values in four equal rows");
    constexpr int H = V / 2, Q = V / 4;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]),
                                                        __float_as_uint(v[i + H]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]),
                                                        __float_as_uint(v[i + Q]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        v[i] = dpp_add<kDppRowShr1, 0xf>(v[i]);
        v[i] = dpp_add<kDppRowShr2, 0xf>(v[i]);
        v[i] = dpp_add<kDppRowShr4, 0xf>(v[i]);
        v[i] = dpp_add<kDppRowShr8, 0xf>(v[i]);
    }
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, kWave));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, kWave));
    return v;
}

// Float to a key whose unsigned order is the float order (and back).
__device__ __forceinline__ uint32_t orderable(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float from_orderable(uint32_t k)
{
    return __uint_as_float((k >> 31) ? (k & 0x7fffffffu) : ~k);
}

// Min / max over the 64 lanes by DPP (no LDS traffic), valid in lane 63:
// within each row of 16 lanes a running min over row_shr 1, 2, 4, 8 (lanes
// shifted in from outside the row take the identity), then row_bcast 15
// carries rows 0 and 2 into rows 1 and 3 and row_bcast 31 carries lane 31
// into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_umin_dpp(uint32_t v)
{
    const int id = -1;   // 0xffffffff
    v = min(v, uint32_t(__builtin_amdgcn_update_dpp(id, int(v), kDppRowShr1, 0xf, 0xf, false)));
    v = min(v, uint32_t(__builtin_amdgcn_update_dpp(id, int(v), kDppRowShr2, 0xf, 0xf, false)));
    v = min(v, uint32_t(__builtin_amdgcn_update_dpp(id, int(v), kDppRowShr4, 0xf, 0xf, false)));
    v = min(v, uint32_t(__builtin_amdgcn_update_dpp(id, int(v), kDppRowShr8, 0xf, 0xf, false)));
    v = min(v, uint32_t(__builtin_amdgcn_update_dpp(id, int(v), kDppRowBcast15, 0xa, 0xf, false)));
    v = min(v, uint32_t(__builtin_amdgcn_update_dpp(id, int(v), kDppRowBcast31, 0xc, 0xf, false)));
    return v;
}

__device__ __forceinline__ uint32_t wave_umax_dpp(uint32_t v)
{
    v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kDppRowShr1, 0xf, 0xf, false)));
    v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kDppRowShr2, 0xf, 0xf, false)));
    v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kDppRowShr4, 0xf, 0xf, false)));
    v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kDppRowShr8, 0xf, 0xf, false)));
    v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kDppRowBcast15, 0xa, 0xf, false)));
    v = max(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kDppRowBcast31, 0xc, 0xf, false)));
    return v;
}

template <typename T> __device__ __forceinline__ T uniform(T v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint64_t u = static_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

}  // namespace ngd
