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
// Atomics-free and Gaussian-major.  Culled: the forward pass records, for
// every candidate entry (tile, Gaussian) and every 64-query group of the
// tile, whether it kept the pair group (one byte); the backward visits only
// the kept groups, so it sums over exactly the pairs the forward summed,
// recomputing y, G and the exp rather than storing them.  A work item is one
// Gaussian and at most kItemTiles of its candidate entries (the transposed
// lists); one wave evaluates the item's kept groups 64 queries at a time,
// keeps per-lane partial moments in registers (B1: n, B2: n(n+1)/2, H: 3),
// reduces them across lanes once and writes them to the item's slot.
// k_backward_finalize then adds each Gaussian's items in item order and
// applies S^T.  Dense: one wave per Gaussian over all queries.
#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kBwdThreads = 256;
constexpr int kMaxGroups = 16;   // 64-query groups of the largest tile (1024)
constexpr int64_t kBwdItemBlocks = 4096;
constexpr int kWavesPerBlock = kBwdThreads / kWave;
static_assert(kItemTiles <= kWave, "an item's tile list must fit one wave");

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
    for (int a = 0; a < N; ++a) b1[a] = wave_sum_last(b1[a]);
#pragma unroll
    for (int e = 0; e < T; ++e) b2[e] = wave_sum_last(b2[e]);
    h0 = wave_sum_last(h0);
    h1 = wave_sum_last(h1);
    h2 = wave_sum_last(h2);
    if (lane != kWave - 1) return;
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

// ---- culled: work items (Gaussian, up to kItemTiles of its tiles) ---------
template <int N> struct BwdLayout {
    static constexpr int T = N * (N + 1) / 2;
    static constexpr int R = (N + T + 7 + 3) / 4 * 4;
    static constexpr int NM = N + T + 3;             // B1 | B2 | H
    static constexpr int K1 = N < 3 ? N : 3;        // stage boundaries
    static constexpr int K2 = N < 6 ? N : 6;
};

// y rows [R0, R1) and msq for one lane; d[a] = x[a] - m[a].
template <int N, int R0, int R1>
__device__ __forceinline__ void brows(const float *__restrict__ r, const float (&x)[N],
                                      float (&d)[N], float (&y)[N], float &msq)
{
#pragma unroll
    for (int row = R0; row < R1; ++row) {
        d[row] = x[row] - r[row];
        const float *srow = r + N + row * (row + 1) / 2;
        float acc = srow[0] * d[0];
#pragma unroll
        for (int j = 1; j <= row; ++j) acc = fmaf(srow[j], d[j], acc);
        y[row] = acc;
        msq = fmaf(acc, acc, msq);
    }
}

// One work item (wave-uniform `it`).
template <int N>
__device__ __forceinline__ void backward_item(
    int64_t it, int64_t q, int tile, const float *__restrict__ grec,
    const float *__restrict__ qs, const float *__restrict__ gs,
    const int64_t *__restrict__ a_off, const int32_t *__restrict__ a_ent,
    const int32_t *__restrict__ ent_tile, const uint8_t *__restrict__ act,
    const int64_t *__restrict__ gitem_off, const int32_t *__restrict__ gitem_g,
    float *__restrict__ gpart, int32_t *__restrict__ gflag)
{
    using Lay = BwdLayout<N>;
    constexpr int T = Lay::T;
    const int lane = lane_id();
    const int64_t g = uniform(gitem_g[it]);
    const int64_t j0 = uniform64(gitem_off[g]);
    const int64_t t0 = uniform64(a_off[g]), t1 = uniform64(a_off[g + 1]);
    const int64_t e0 = t0 + (it - j0) * kItemTiles;
    const int64_t e1 = (e0 + kItemTiles < t1) ? e0 + kItemTiles : t1;
    const float *__restrict__ r = grec + g * Lay::R;
    constexpr int AL = N + T + 3, CO = N + T + 4;
    const float alpha = r[AL], c0 = r[CO], c1 = r[CO + 1], c2 = r[CO + 2];

    float b1[N], b2[T], h0 = 0.0f, h1 = 0.0f, h2 = 0.0f;
#pragma unroll
    for (int a = 0; a < N; ++a) b1[a] = 0.0f;
#pragma unroll
    for (int e = 0; e < T; ++e) b2[e] = 0.0f;

    // The item's entries, lane = entry (at most kItemTiles <= 64): the
    // entry's tile and the flags of its query groups, loaded together once
    // the entry is known; then the kept (entry, group) pairs in ascending
    // entry order, groups ascending within an entry.
    const int ngroups = (tile + kWave - 1) / kWave;
    const int nent = int(e1 - e0);
    int tl = 0;
    uint32_t fl = 0;   // bit g: group g kept
    if (lane < nent) {
        const int64_t ent = a_ent[e0 + lane];
        tl = ent_tile[ent];
        const uint8_t *af = act + ent * ngroups;
        if (ngroups == 4) {
            // one aligned 4-byte load: tiles of 193..256 queries
            const uint32_t v = *reinterpret_cast<const uint32_t *>(af);
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) fl |= uint32_t(((v >> (8 * gq)) & 0xffu) != 0) << gq;
        } else {
            // tiles of at most 1024 queries: at most 16 groups, loaded
            // together
#pragma unroll
            for (int gq = 0; gq < kMaxGroups; ++gq)
                if (gq < ngroups) fl |= uint32_t(af[gq] != 0) << gq;
        }
    }
    bool any = false;
    for (uint64_t m = ballot(fl != 0); m != 0; m = ballot(fl != 0)) {
        const int l = __ffsll(static_cast<unsigned long long>(m)) - 1;
        const uint32_t fb = __builtin_amdgcn_readlane(fl, l);
        const int gq = __builtin_ctz(fb);
        if (lane == l) fl = fb & (fb - 1);
        {
            const int64_t tt = __builtin_amdgcn_readlane(tl, l);
            const int sidx = gq * kWave + lane;
            const int64_t p = tt * tile + sidx;
            const bool valid = (sidx < tile) && (p < q);
            // every lane loads (a lane past the tile's end from the tile's
            // first query) and the invalid ones are zeroed: no branches
            const int64_t pc = valid ? p : tt * tile;
            float x[N], d[N], y[N];
#pragma unroll
            for (int a = 0; a < N; ++a) x[a] = qs[a * q + pc];
            float msq = 0.0f;
            brows<N, 0, N>(r, x, d, y, msq);
            any = true;
            const float G = valid ? __builtin_amdgcn_exp2f(-msq) : 0.0f;
            const float g0v = valid ? gs[pc] : 0.0f;
            const float g1v = valid ? gs[q + pc] : 0.0f;
            const float g2v = valid ? gs[2 * q + pc] : 0.0f;
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
                for (int b = 0; b <= a; ++b)
                    b2[a * (a + 1) / 2 + b] = fmaf(wy, y[b], b2[a * (a + 1) / 2 + b]);
            }
        }
    }
    if (!any) {
        if (lane == 0) gflag[it] = 0;
        return;
    }
    // the moments (B1 | B2 | H, padded to a multiple of 4) summed over the
    // wave; lane 16 r + 15 writes the totals of the r-th quarter
    constexpr int VP = (Lay::NM + 3) & ~3, Q = VP / 4;
    float mv[VP];
#pragma unroll
    for (int a = 0; a < N; ++a) mv[a] = b1[a];
#pragma unroll
    for (int e = 0; e < T; ++e) mv[N + e] = b2[e];
    mv[N + T + 0] = h0;
    mv[N + T + 1] = h1;
    mv[N + T + 2] = h2;
#pragma unroll
    for (int e = Lay::NM; e < VP; ++e) mv[e] = 0.0f;
    wave_reduce_scatter<VP>(mv);
    if ((lane & 15) != 15) return;
    float *out = gpart + it * Lay::NM;
    const int r0 = (lane >> 4) * Q;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (r0 + i < Lay::NM) out[r0 + i] = mv[i];
    if (lane == kWave - 1) gflag[it] = 1;
}

// The items (their number on the device) taken by the launched waves in
// turn: a wave's items lie a grid apart.
template <int N>
__global__ __launch_bounds__(kBwdThreads) void k_backward_items(
    int64_t k, int64_t q, int tile, const float *__restrict__ grec,
    const float *__restrict__ qs, const float *__restrict__ gs,
    const int64_t *__restrict__ a_off, const int32_t *__restrict__ a_ent,
    const int32_t *__restrict__ ent_tile, const uint8_t *__restrict__ act,
    const int64_t *__restrict__ gitem_off, const int32_t *__restrict__ gitem_g,
    float *__restrict__ gpart, int32_t *__restrict__ gflag)
{
    const int64_t nit = uniform64(gitem_off[k]);
    const int64_t stride = int64_t(gridDim.x) * kWavesPerBlock;
    for (int64_t it = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave; it < nit;
         it += stride)
        backward_item<N>(it, q, tile, grec, qs, gs, a_off, a_ent, ent_tile, act, gitem_off,
                         gitem_g, gpart, gflag);
}

// Per sorted Gaussian: sum its items' moments in item order, then
//   dm = S'^T B1 / c, dL = tril(S'^T B2) / c^1.5, dalpha = c . H, dc = alpha H.
template <int N>
__global__ __launch_bounds__(kBwdThreads) void k_backward_finalize(
    int64_t k, const float *__restrict__ grec, const int64_t *__restrict__ gitem_off,
    const float *__restrict__ gpart, const int32_t *__restrict__ gflag,
    const int32_t *__restrict__ gperm, float *__restrict__ g_mean,
    float *__restrict__ g_factor, float *__restrict__ g_weight, float *__restrict__ g_colour)
{
    using Lay = BwdLayout<N>;
    constexpr int T = Lay::T, NM = Lay::NM;
    const int64_t g = int64_t(blockIdx.x) * kBwdThreads + threadIdx.x;
    if (g >= k) return;
    float acc[NM];
#pragma unroll
    for (int e = 0; e < NM; ++e) acc[e] = 0.0f;
    for (int64_t i = gitem_off[g]; i < gitem_off[g + 1]; ++i) {
        if (!gflag[i]) continue;
        const float *pp = gpart + i * NM;
#pragma unroll
        for (int e = 0; e < NM; ++e) acc[e] += pp[e];
    }
    const float *r = grec + g * Lay::R;
    const int64_t gi = gperm[g];
    const float inv_c = float(1.0 / kHalfLog2e);
    const float inv_c15 = float(1.0 / (kHalfLog2e * kSqrtHalfLog2e));
#pragma unroll
    for (int a = 0; a < N; ++a) {
        float s = 0.0f;
#pragma unroll
        for (int kk = a; kk < N; ++kk) s = fmaf(r[N + kk * (kk + 1) / 2 + a], acc[kk], s);
        g_mean[gi * N + a] = s * inv_c;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            float s = 0.0f;
#pragma unroll
            for (int kk = a; kk < N; ++kk)
                s = fmaf(r[N + kk * (kk + 1) / 2 + a], acc[N + kk * (kk + 1) / 2 + b], s);
            g_factor[gi * T + a * (a + 1) / 2 + b] = s * inv_c15;
        }
    }
    const float alpha = r[N + T + 3];
    const float h0 = acc[N + T], h1 = acc[N + T + 1], h2 = acc[N + T + 2];
    g_weight[gi] = fmaf(r[N + T + 6], h2, fmaf(r[N + T + 5], h1, r[N + T + 4] * h0));
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
    hipError_t err = launch_backward_prepare(c, s);
    if (err != hipSuccess) return err;
    if (c->gitems_cap > 0) {
        // about four rounds of resident waves (4 per SIMD at this kernel's
        // register count), each taking items a grid apart: 1,024 / 2,048 /
        // 4,096 blocks measured 327-343 / 319-326 / 293-305 us at 10-D,
        // 2^20 queries (8,192 and 16,384 alike), against 346-353 us with
        // one wave per item
        const unsigned blocks = unsigned(std::min<int64_t>(
            (c->gitems_cap + kWavesPerBlock - 1) / kWavesPerBlock, kBwdItemBlocks));
        const int32_t *a_ent = c->a_ent_buf ? c->vals1.as<int32_t>() : c->vals0.as<int32_t>();
        k_backward_items<N><<<blocks, kBwdThreads, 0, s>>>(
            mix->k, c->q, c->params.tile, c->grec.as<float>(), c->qs.as<float>(),
            c->gs.as<float>(), c->a_off.as<int64_t>(), a_ent,
            c->ent_tile.as<int32_t>(), c->act.as<uint8_t>(), c->gitem_off.as<int64_t>(),
            c->gitem_g.as<int32_t>(), c->gpart.as<float>(), c->gflag.as<int32_t>());
    }
    const unsigned fb = unsigned((mix->k + kBwdThreads - 1) / kBwdThreads);
    k_backward_finalize<N><<<fb, kBwdThreads, 0, s>>>(
        mix->k, c->grec.as<float>(), c->gitem_off.as<int64_t>(), c->gpart.as<float>(),
        c->gflag.as<int32_t>(), c->gperm.as<int32_t>(), gm, gf, gw, gc);
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
