// Forward evaluation of the mixture colour (Sec. 4.1, Eq. 8):
//   f(x) = sum_i exp2(-|S'_i (x - m_i)|^2) alpha_i c_i,  S' = sqrt(log2(e)/2) L^-1
//
// Layout: one lane per query, queries held in registers; the Gaussian being
// evaluated is the same for the whole wave, so its record (mean, S', alpha c)
// is read with wave-uniform loads and feeds the VALU as scalar operands.  The
// first 32 floats of the next candidate's record are loaded one iteration
// ahead, so the loop does not wait on the load of the record it evaluates.
//
// Culled kernel: one workgroup per work item -- a tile's queries and at most
// kItemCands of its candidates -- so a tile with a long list is spread over
// many workgroups.  A tile with a single item writes its colours directly;
// otherwise items write partial sums that k_eval_reduce adds in item order.
//
// Each pair is evaluated in stages.  After the first 3 and 6 coordinates
// the partial sum |y_{0..k}|^2 is the Mahalanobis distance of the marginal
// over those coordinates (the leading block of L^-1 is the inverse of the
// leading block of L), a lower bound of the full distance.  When no lane of
// the wave is below the skip threshold the pair is dropped; the threshold
// certifies G < tau * 2^-20, so a dropped pair changes f by less than that
// times alpha |c|.  The same test is applied once more before the exp.
//
// Ahead of those checks each wave tests its 64 queries' bounding box against
// a per-Gaussian box built with the cull (lane = candidate, 2n float16
// bounds rounded outwards, in 16-byte loads): a Gaussian whose box misses the queries' box in some
// coordinate has every distance above the skip threshold (the marginal over
// that coordinate alone bounds it), so it is dropped before its record is
// read, and only the survivors go through the staged evaluation.
//
// Dense kernel: the plain direct sum over all Gaussians, no skipping.
#include "eval_common.hpp"
#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kEvalThreads = 256;
template <int N>
__global__ __launch_bounds__(kEvalThreads) void k_eval_dense(int64_t k, int64_t q,
                                                             const float *__restrict__ rec,
                                                             const float *__restrict__ queries,
                                                             float *__restrict__ out)
{
    using Lay = RecLayout<N>;
    const int64_t p = int64_t(blockIdx.x) * kEvalThreads + threadIdx.x;
    const bool valid = p < q;
    float x[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = valid ? queries[p * N + a] : 0.0f;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    float blk[Lay::PF], nxt[Lay::PF];
    if (k > 0) load_block<N>(nxt, rec);
    for (int64_t i = 0; i < k; ++i) {
#pragma unroll
        for (int e = 0; e < Lay::PF; ++e) blk[e] = nxt[e];
        if (i + 1 < k) load_block<N>(nxt, rec + (i + 1) * Lay::R);
        eval_pair<N, false>(blk, rec + i * Lay::R, x, valid, 0.0f, f0, f1, f2);
    }
    if (valid) {
        out[p * 3 + 0] = f0;
        out[p * 3 + 1] = f1;
        out[p * 3 + 2] = f2;
    }
}

// The same direct sum for batches too small to fill the chip one query per
// lane: a workgroup takes 64 queries (lane = query) and its 4 waves split
// the Gaussians into 4 consecutive ranges; the 4 partial sums are added in
// range order through LDS, so the result does not depend on scheduling.
constexpr int kSplit = kEvalThreads / kWave;
template <int N>
__global__ __launch_bounds__(kEvalThreads) void k_eval_dense_split(
    int64_t k, int64_t q, const float *__restrict__ rec, const float *__restrict__ queries,
    float *__restrict__ out)
{
    using Lay = RecLayout<N>;
    __shared__ float part[kSplit][3][kWave];
    const int w = int(threadIdx.x) / kWave, lane = lane_id();
    const int64_t p = int64_t(blockIdx.x) * kWave + lane;
    const bool valid = p < q;
    float x[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = valid ? queries[p * N + a] : 0.0f;
    const int64_t per = (k + kSplit - 1) / kSplit;
    const int64_t i0 = w * per, i1 = (i0 + per < k) ? i0 + per : k;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    float blk[Lay::PF], nxt[Lay::PF];
    if (i0 < i1) load_block<N>(nxt, rec + i0 * Lay::R);
    for (int64_t i = i0; i < i1; ++i) {
#pragma unroll
        for (int e = 0; e < Lay::PF; ++e) blk[e] = nxt[e];
        if (i + 1 < i1) load_block<N>(nxt, rec + (i + 1) * Lay::R);
        eval_pair<N, false>(blk, rec + i * Lay::R, x, valid, 0.0f, f0, f1, f2);
    }
    part[w][0][lane] = f0;
    part[w][1][lane] = f1;
    part[w][2][lane] = f2;
    __syncthreads();
    if (w == 0 && valid) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = part[0][ch][lane];
#pragma unroll
            for (int v = 1; v < kSplit; ++v) acc += part[v][ch][lane];
            out[p * 3 + ch] = acc;
        }
    }
}

// OUT = false: only the keep/skip flags are written (the backward pass needs
// them when no forward ran on this cull).  COUNT (with OUT = false): the
// flags are written and the stage counters of every wave are added to
// stats[0..4] = (pairs examined, passed the box test, passed check 1, passed
// check 2, kept).
template <int N, bool OUT, bool COUNT = false>
__global__ __launch_bounds__(kEvalThreads) void k_eval_items(
    int64_t q, int tile, const float *__restrict__ grec, const float *__restrict__ gbox,
    const float *__restrict__ qs,
    const int64_t *__restrict__ tile_off, const int32_t *__restrict__ cand,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ item_tile,
    const int64_t *__restrict__ item_off, float skip, float *__restrict__ out,
    float *__restrict__ part, uint8_t *__restrict__ act,
    unsigned long long *__restrict__ stats = nullptr)
{
    using Lay = RecLayout<N>;
    const int64_t it = xcd_block(blockIdx.x, gridDim.x);   // neighbouring tiles share an L2
    const int64_t t = uniform(item_tile[it]);
    const int64_t i0 = uniform64(item_off[t]);
    const int64_t nit = uniform64(item_off[t + 1]) - i0;
    const int64_t c0 = uniform64(tile_off[t]), c1 = uniform64(tile_off[t + 1]);
    const int64_t e0 = c0 + (it - i0) * kItemCands;
    const int64_t e1 = (e0 + kItemCands < c1) ? e0 + kItemCands : c1;

    const int s = int(blockIdx.y) * kEvalThreads + int(threadIdx.x);
    const int64_t p = t * tile + s;
    const bool valid = (s < tile) && (p < q);
    float x[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = valid ? qs[a * q + p] : 0.0f;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;

    // the wave's query box (empty, lo > hi, for a wave without queries),
    // broadcast into vector registers: the scalar ones hold the records
    float qlo[N], qhi[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        qlo[a] = from_orderable(uint32_t(
            __shfl(int(wave_umin_dpp(orderable(valid ? x[a] : INFINITY))), kWave - 1, kWave)));
        qhi[a] = from_orderable(uint32_t(
            __shfl(int(wave_umax_dpp(orderable(valid ? x[a] : -INFINITY))), kWave - 1, kWave)));
    }

    // Candidate indices are read 64 at a time with one vector load, and each
    // lane tests its candidate's box.  The survivors' records are fetched
    // with wave-uniform loads one survivor ahead into one of two register
    // blocks.  Uniform loads may complete out of order, so the wait for the
    // current block is placed before the next block's load is issued: the
    // wait then never covers the load still in flight.
    // keep/skip flag of each (candidate entry, 64-query group), one byte each
    const int ngroups = (tile + kWave - 1) / kWave;
    const int grp = s / kWave;
    float bufA[Lay::PF], bufB[Lay::PF];
    uint32_t st[3] = {0u, 0u, 0u};
    uint32_t boxed = 0;
    for (int64_t ch = e0; ch < e1; ch += kWave) {
        const int n = int((e1 - ch < kWave) ? e1 - ch : kWave);
        const int lane = lane_id();
        const int vidx = (lane < n) ? cand[ch + lane] : 0;
        bool near = false;
        if (lane < n) {
            constexpr int BW = (2 * N + 7) / 8;   // 16-byte words of 8 float16
            const uint4 *b = reinterpret_cast<const uint4 *>(gbox) + int64_t(vidx) * BW;
            uint32_t hw[4 * BW];
#pragma unroll
            for (int w = 0; w < BW; ++w) {
                const uint4 v = b[w];
                hw[4 * w] = v.x, hw[4 * w + 1] = v.y, hw[4 * w + 2] = v.z, hw[4 * w + 3] = v.w;
            }
            float bl[2 * N];
#pragma unroll
            for (int e = 0; e < 2 * N; ++e)
                bl[e] = float(__builtin_bit_cast(_Float16, uint16_t(hw[e / 2] >> (16 * (e & 1)))));
            bool apart = false;
#pragma unroll
            for (int a = 0; a < N; ++a) apart |= (qlo[a] > bl[N + a]) | (qhi[a] < bl[a]);
            near = !apart;
        }
        uint64_t live = ballot(near);
        if constexpr (COUNT) boxed += uint32_t(__builtin_popcountll(live));
        uint32_t kept = 0;
        if (live != 0) {
            int ja = __builtin_ctzll(live);
            live &= live - 1;
            int64_t ia = __builtin_amdgcn_readlane(vidx, ja);
            load_block<N>(bufA, grec + ia * Lay::R);
            for (;;) {
                __builtin_amdgcn_s_waitcnt(kWaitScalar);
                int jb = -1;
                int64_t ib = 0;
                if (live != 0) {
                    jb = __builtin_ctzll(live);
                    live &= live - 1;
                    ib = __builtin_amdgcn_readlane(vidx, jb);
                    load_block<N>(bufB, grec + ib * Lay::R);
                }
                if (eval_pair<N, true, OUT, COUNT>(bufA, grec + ia * Lay::R, x, valid, skip, f0,
                                                   f1, f2, st))
                    kept = (lane == ja) ? 1u : kept;
                if (jb < 0) break;
                __builtin_amdgcn_s_waitcnt(kWaitScalar);
                ja = -1;
                if (live != 0) {
                    ja = __builtin_ctzll(live);
                    live &= live - 1;
                    ia = __builtin_amdgcn_readlane(vidx, ja);
                    load_block<N>(bufA, grec + ia * Lay::R);
                }
                if (eval_pair<N, true, OUT, COUNT>(bufB, grec + ib * Lay::R, x, valid, skip, f0,
                                                   f1, f2, st))
                    kept = (lane == jb) ? 1u : kept;
                if (ja < 0) break;
            }
        }
        if (lane < n && grp < ngroups) act[(ch + lane) * ngroups + grp] = uint8_t(kept);
    }
    if constexpr (COUNT) {
        if (lane_id() == 0 && grp < ngroups) {
            // (examined, passed the box test, passed check 1, passed check 2,
            // kept)
            atomicAdd(&stats[0], static_cast<unsigned long long>(e1 - e0));
            atomicAdd(&stats[1], static_cast<unsigned long long>(boxed));
            atomicAdd(&stats[2], static_cast<unsigned long long>(st[0]));
            atomicAdd(&stats[3], static_cast<unsigned long long>(st[1]));
            atomicAdd(&stats[4], static_cast<unsigned long long>(st[2]));
        }
    }
    if constexpr (!OUT) return;
    if (!valid) return;
    if (nit == 1) {
        const int64_t o = perm[p];
        out[o * 3 + 0] = f0;
        out[o * 3 + 1] = f1;
        out[o * 3 + 2] = f2;
    } else {
        float *pp = part + it * 3 * int64_t(tile);
        pp[s] = f0;
        pp[tile + s] = f1;
        pp[2 * tile + s] = f2;
    }
}

// Tiles with no item (no candidates) get zeros; tiles with two or more items
// get the sum of their items' partials in item order.
__global__ __launch_bounds__(kEvalThreads) void k_eval_reduce(
    int64_t q, int tile, const int32_t *__restrict__ perm, const int64_t *__restrict__ item_off,
    const float *__restrict__ part, float *__restrict__ out)
{
    const int64_t t = blockIdx.x;
    const int64_t i0 = item_off[t], i1 = item_off[t + 1];
    if (i1 - i0 == 1) return;
    const int s = int(blockIdx.y) * kEvalThreads + int(threadIdx.x);
    const int64_t p = t * tile + s;
    if (s >= tile || p >= q) return;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    for (int64_t i = i0; i < i1; ++i) {
        const float *pp = part + i * 3 * int64_t(tile);
        f0 += pp[s];
        f1 += pp[tile + s];
        f2 += pp[2 * tile + s];
    }
    const int64_t o = perm[p];
    out[o * 3 + 0] = f0;
    out[o * 3 + 1] = f1;
    out[o * 3 + 2] = f2;
}

template <int N>
hipError_t dense_n(const ngd_mixture *mix, const float *queries, int64_t q, float *out,
                   hipStream_t s)
{
    // one query per lane while that gives every SIMD several waves;
    // smaller batches split the Gaussians over the waves of a workgroup
    if (q >= (int64_t(1) << 18) || mix->k < 4 * kSplit) {
        const unsigned blocks = unsigned((q + kEvalThreads - 1) / kEvalThreads);
        k_eval_dense<N><<<blocks, kEvalThreads, 0, s>>>(mix->k, q, mix->rec.as<float>(), queries,
                                                        out);
    } else {
        const unsigned blocks = unsigned((q + kWave - 1) / kWave);
        k_eval_dense_split<N><<<blocks, kEvalThreads, 0, s>>>(mix->k, q, mix->rec.as<float>(),
                                                              queries, out);
    }
    return hipGetLastError();
}

template <int N>
hipError_t culled_n(const ngd_mixture *mix, const ngd_cull *c, float *out, hipStream_t s)
{
    (void)mix;
    const int tile = c->params.tile;
    const int per = tile < kEvalThreads ? (tile + 63) / 64 * 64 : kEvalThreads;
    const unsigned gy = unsigned((tile + kEvalThreads - 1) / kEvalThreads);
    // skip when exp2(-M') < tau 2^-margin, i.e. M' > log2(1/tau) + margin
    const float skip = float(-std::log2(double(c->params.tau)) + kSkipLog2Margin);
    uint8_t *act = c->act.as<uint8_t>();
    if (c->nitems > 0) {
        if (out)
            k_eval_items<N, true><<<dim3(unsigned(c->nitems), gy), per, 0, s>>>(
                c->q, tile, c->grec.as<float>(), c->gbox.as<float>(), c->qs.as<float>(),
                c->tile_off.as<int64_t>(),
                c->cand.as<int32_t>(), c->perm.as<int32_t>(), c->item_tile.as<int32_t>(),
                c->item_off.as<int64_t>(), skip, out, c->fpart.as<float>(), act);
        else
            k_eval_items<N, false><<<dim3(unsigned(c->nitems), gy), per, 0, s>>>(
                c->q, tile, c->grec.as<float>(), c->gbox.as<float>(), c->qs.as<float>(),
                c->tile_off.as<int64_t>(),
                c->cand.as<int32_t>(), c->perm.as<int32_t>(), c->item_tile.as<int32_t>(),
                c->item_off.as<int64_t>(), skip, nullptr, c->fpart.as<float>(), act);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !out) return e;
    return launch_eval_reduce(c, out, s);
}

template <int N>
hipError_t stats_n(const ngd_cull *c, unsigned long long *stats, hipStream_t s)
{
    const int tile = c->params.tile;
    const int per = tile < kEvalThreads ? (tile + 63) / 64 * 64 : kEvalThreads;
    const unsigned gy = unsigned((tile + kEvalThreads - 1) / kEvalThreads);
    const float skip = float(-std::log2(double(c->params.tau)) + kSkipLog2Margin);
    if (c->nitems > 0)
        k_eval_items<N, false, true><<<dim3(unsigned(c->nitems), gy), per, 0, s>>>(
            c->q, tile, c->grec.as<float>(), c->gbox.as<float>(), c->qs.as<float>(),
            c->tile_off.as<int64_t>(),
            c->cand.as<int32_t>(), c->perm.as<int32_t>(), c->item_tile.as<int32_t>(),
            c->item_off.as<int64_t>(), skip, nullptr, c->fpart.as<float>(), c->act.as<uint8_t>(),
            stats);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval_reduce(const ngd_cull *c, float *out, hipStream_t s)
{
    const int tile = c->params.tile;
    const int per = tile < kEvalThreads ? (tile + 63) / 64 * 64 : kEvalThreads;
    const unsigned gy = unsigned((tile + kEvalThreads - 1) / kEvalThreads);
    k_eval_reduce<<<dim3(unsigned(c->ntiles), gy), per, 0, s>>>(
        c->q, tile, c->perm.as<int32_t>(), c->item_off.as<int64_t>(), c->fpart.as<float>(), out);
    return hipGetLastError();
}

hipError_t launch_eval_stats(const ngd_mixture *mix, const ngd_cull *c,
                             unsigned long long *stats, hipStream_t s)
{
    if (c->q == 0 || c->ntiles == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return stats_n<NN>(c, stats, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

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
    if (c->q == 0 || c->ntiles == 0) return hipSuccess;
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
