// Culled forward with a matrix-core filter: the Mahalanobis distance of
// every (query, candidate) pair of a tile as one BF16 MFMA contraction
// of quadratic query features against per-Gaussian quadratic coefficients.
//
// The quadratic form (Sec. 3.1, Eq. 1-2, in exp2 units, S' = sqrt(log2(e)/2)
// L^-1, P' = S'^T S'):
//   M'(x) = |S'(x - m)|^2
//         = sum_{i<=j} C_ij x'_i x'_j + sum_i b'_i x'_i + a',
//   x' = x - c, m' = m - c, C_ii = P'_ii, C_ij = 2 P'_ij (i < j),
//   b' = -2 S'^T (S' m'),  a' = |S' m'|^2,
// with c the centre of the tile's query box, so that the features stay
// small and the expanded form does not cancel away its own accuracy.  The
// feature vector (1, x', x'_i x'_j) has 1 + N + N(N+1)/2 entries (66 at
// N = 10), laid out as one k-step of 16 for the constant and linear terms
// and ceil(N(N+1)/2 / 16) k-steps for the quadratic ones.
//
// Precision: features and coefficients are split into bf16 pairs
// v = hi + lo + r, |r| <= 2^-16 |v|, and the contraction takes the three
// products hi*hi + hi*lo + lo*hi with fp32 accumulation
// (v_mfma_f32_32x32x16_bf16).  Its error against the exact form is below
// 2^-13 * sum_k |F_k| |C_k| (a generous bound: split and omitted lo*lo terms
// give about 3 * 2^-16, accumulation of at most 3 * 96 exact products about
// 2^-16).  Over a 64-query group with h_i = max |x'_i| that sum is at most
//   R' |h|^2 + |b'|_1 max h + |a'|,   R' = max row sum of |S'|^T |S'|,
// and the fp32 rounding of b' adds at most 2^-18 R' |m'|_1 max h.  A
// candidate is skipped for the whole group only when the smallest M' of the
// group minus that bound exceeds the skip threshold log2(1/tau) + 20, the
// same certificate the fp32 kernel applies (G < tau 2^-20).  Every
// candidate that is not skipped is evaluated exactly as in the fp32 kernel
// (the same staged code, lane = query), so the colours carry fp32 accuracy;
// they differ from the fp32 kernel's only by pairs below the certificate.
//
// Once per cull build: the quadratic coefficients of every ordered Gaussian
// (float64 P', then bf16 hi / lo) and for every candidate entry (tile,
// Gaussian) the centred constant and linear coefficients and bound terms --
// one thread per entry; the centre of every tile's query box comes with the
// cull's tile bounds.
// Filter kernel, one workgroup per tile (up to 256 queries in 4 waves):
// per wave the query features as MFMA A fragments (rows = queries, 2 blocks
// of 32); the entries' B fragments staged in LDS in double-buffered chunks of
// 64 (the next chunk loaded straight into LDS while the current one is
// computed); per block of
// 32 entries 3 x KS x 2 MFMAs and the certified group test; the (entry,
// group) flag records whether the pair may contribute.  The
// float32 items kernel then evaluates only the flagged pairs (eval.hip).
#include <cmath>
#include <type_traits>

#include "eval_common.hpp"
#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMThreads = 256;
constexpr int kCh = 64;       // entries staged in LDS at a time (one per lane)
static_assert(kCh == kWave, "a wave loads the indices of one chunk");
constexpr float kGammaQ = 1.0f / 8192.0f;     // 2^-13
constexpr float kGammaB = 1.0f / 262144.0f;   // 2^-18

template <int N> struct Feat {
    static constexpr int T = N * (N + 1) / 2;
    static constexpr int KQ = (T + 15) / 16;   // quadratic k-steps
    static constexpr int KS = 1 + KQ;          // plus constant and linear
    static_assert(N + 1 <= 16, "constant and linear terms fill one k-step");
};

// Quadratic slot q -> (i, j), i <= j, the upper triangle by rows.
template <int N> struct QuadTable {
    int i[Feat<N>::KQ * 16];
    int j[Feat<N>::KQ * 16];
    constexpr QuadTable() : i(), j()
    {
        int q = 0;
        for (int a = 0; a < N; ++a)
            for (int b = a; b < N; ++b) {
                i[q] = a;
                j[q] = b;
                ++q;
            }
        for (; q < Feat<N>::KQ * 16; ++q) {
            i[q] = -1;
            j[q] = -1;
        }
    }
};
template <int N> inline constexpr QuadTable<N> kQuad{};

__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo)
{
    hi = __bf16(v);
    lo = __bf16(v - float(hi));
}

// Per ordered Gaussian: the quadratic coefficients as bf16 hi / lo pairs in
// B-fragment order -- for quadratic k-step ks and half h, 8 hi then 8 lo --
// and R' = max row sum of |S'|^T |S'|.  P' is formed in float64.
template <int N>
__global__ __launch_bounds__(256) void k_mfma_coef(int64_t k, const float *__restrict__ grec,
                                                   __bf16 *__restrict__ mrec,
                                                   float *__restrict__ rrow)
{
    using Fe = Feat<N>;
    constexpr int R = RecLayout<N>::R;
    const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (s >= k) return;
    const float *r = grec + s * R + N;   // S' packed lower by rows
    double S[Fe::T];
#pragma unroll
    for (int e = 0; e < Fe::T; ++e) S[e] = double(r[e]);
    auto sidx = [](int row, int col) { return row * (row + 1) / 2 + col; };
    __bf16 *o = mrec + s * (Fe::KQ * 32);
#pragma unroll
    for (int q = 0; q < Fe::KQ * 16; ++q) {
        float cf = 0.0f;
        if (kQuad<N>.i[q] >= 0) {
            const int a = kQuad<N>.i[q], b = kQuad<N>.j[q];   // a <= b
            double p = 0.0;
#pragma unroll
            for (int row = 0; row < N; ++row)
                if (row >= b) p += S[sidx(row, a)] * S[sidx(row, b)];
            cf = float(a == b ? p : 2.0 * p);
        }
        __bf16 hi, lo;
        split_bf16(cf, hi, lo);
        const int ks = q / 16, h = (q % 16) / 8, e = q % 8;
        o[(ks * 2 + h) * 16 + e] = hi;
        o[(ks * 2 + h) * 16 + 8 + e] = lo;
    }
    double best = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        double rs = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
#pragma unroll
            for (int row = 0; row < N; ++row) {
                if (row >= a && row >= b) rs += fabs(S[sidx(row, a)]) * fabs(S[sidx(row, b)]);
            }
        }
        best = rs > best ? rs : best;
    }
    rrow[s] = float(best) * (1.0f + 1.0f / 1048576.0f);
}

// Per candidate entry (tile, Gaussian): the centred constant and linear
// coefficients a' = |S'm'|^2, b' = -2 S'^T (S'm'), m' = m - c_tile, as the
// k-step-0 B fragments (per half: 8 bf16 hi, 8 bf16 lo), and the bound terms
// (|a'|, |b'|_1, |m'|_1, R').
template <int N>
__global__ __launch_bounds__(256) void k_mfma_entry(int64_t total,
                                                    const int32_t *__restrict__ cand,
                                                    const int32_t *__restrict__ ent_tile,
                                                    const float *__restrict__ grec,
                                                    const float *__restrict__ rrow,
                                                    const float *__restrict__ tcen,
                                                    bf16x8 *__restrict__ eb0,
                                                    float4 *__restrict__ ebnd)
{
    constexpr int R = RecLayout<N>::R;
    // the record's mean and factor: NV float4s, staged per wave in LDS by
    // 16-byte global-to-LDS loads in rounds of 64 consecutive slots (each
    // round reads whole stretches of records), at an odd stride per entry
    // so that the lanes' reads meet no bank conflicts
    constexpr int NV = (N + RecLayout<N>::T + 3) / 4;
    constexpr int kSt = NV | 1;
    __shared__ float4 s_rec[256 / kWave][kWave * kSt];
    const int w = int(threadIdx.x) / kWave, lane = lane_id();
    // consecutive blocks (neighbouring tiles' entries, which share
    // Gaussians) on one XCD, so that they share its L2
    const int64_t ew = xcd_block(blockIdx.x, gridDim.x) * 256 + w * kWave;   // the wave's first entry
    if (ew >= total) return;                                    // uniform over the wave
    const int nw = int(total - ew < kWave ? total - ew : kWave);
    const int64_t e = ew + lane;
    const int spl = lane < nw ? cand[e] : 0;
#pragma unroll
    for (int i = 0; i < kSt; ++i) {
        const int sl = i * kWave + lane;
        const int j = sl / kSt, v = sl - j * kSt;
        const int spj = __shfl(spl, j, kWave);
        if (v < NV && j < nw)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(grec + int64_t(spj) * R + 4 * v),
                (__attribute__((address_space(3))) void *)(&s_rec[w][i * kWave]), 16, 0, 0);
    }
    // the wave reads only what its own loads wrote
    __builtin_amdgcn_s_waitcnt(0);
    if (lane >= nw) return;
    const int sp = spl;
    float r[NV * 4];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const float4 u = s_rec[w][lane * kSt + v];
        r[4 * v + 0] = u.x;
        r[4 * v + 1] = u.y;
        r[4 * v + 2] = u.z;
        r[4 * v + 3] = u.w;
    }
    const float *c = tcen + int64_t(ent_tile[e]) * N;
    float mp[N], y[N], b[N];
    float m1 = 0.0f;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        mp[a] = r[a] - c[a];
        m1 += fabsf(mp[a]);
    }
    float a0 = 0.0f;
#pragma unroll
    for (int row = 0; row < N; ++row) {
        float acc = 0.0f;
#pragma unroll
        for (int col = 0; col <= row; ++col)
            acc = fmaf(r[N + row * (row + 1) / 2 + col], mp[col], acc);
        y[row] = acc;
        a0 = fmaf(acc, acc, a0);
    }
    float b1 = 0.0f;
#pragma unroll
    for (int col = 0; col < N; ++col) {
        float acc = 0.0f;
#pragma unroll
        for (int row = col; row < N; ++row)
            acc = fmaf(r[N + row * (row + 1) / 2 + col], y[row], acc);
        b[col] = -2.0f * acc;
        b1 += fabsf(b[col]);
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        bf16x8 vhi, vlo;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int slot = 8 * hh + k;
            const float v = slot == 0 ? a0 : (slot <= N ? b[slot - 1] : 0.0f);
            __bf16 hi, lo;
            split_bf16(v, hi, lo);
            vhi[k] = hi;
            vlo[k] = lo;
        }
        eb0[e * 4 + hh * 2 + 0] = vhi;
        eb0[e * 4 + hh * 2 + 1] = vlo;
    }
    ebnd[e] = make_float4(fabsf(a0), b1, m1, rrow[sp]);
}

// OUT: the colours are accumulated and written (caller order); otherwise
// only the (entry, group) flags.  COUNT (with OUT = false): the counters
// stats[0..4] = (examined, not skipped by the matrix filter, passed check 1,
// passed check 2, kept) are added.
template <int N, bool OUT, bool COUNT>
__global__ __launch_bounds__(kMThreads, 3) void k_mfma_filter(
    int64_t q, int tile, const bf16x8 *__restrict__ mrec, const bf16x8 *__restrict__ eb0,
    const float4 *__restrict__ ebnd, const float *__restrict__ tcen,
    const float *__restrict__ qs, const float *__restrict__ grec,
    const int64_t *__restrict__ tile_off, const int32_t *__restrict__ cand,
    const int32_t *__restrict__ perm, float skip, uint8_t *__restrict__ act,
    float *__restrict__ out, unsigned long long *__restrict__ stats)
{
    using Fe = Feat<N>;
    using Lay = RecLayout<N>;
    constexpr int KS = Fe::KS, KQ = Fe::KQ;
    // Per buffer, three regions of 16-byte slots, each entry's units padded
    // to an odd stride so that 8 and 16 consecutive entries fall on distinct
    // bank groups: the k-step-0 units (half * 2 + {hi, lo}) of the entries,
    // their quadratic units ((k-step - 1) * 2 + half) * 2 + {hi, lo}, and
    // their bound terms |a'|, |b'|_1, |m'|_1, R' (consecutive).
    constexpr int kMU = KQ * 4;                  // quadratic units per entry
    constexpr int kStA = 5, kStB = kMU + 1;      // entry strides
    constexpr int kOffB = kCh * kStA, kOffC = kOffB + kCh * kStB;
    constexpr int kBufSlots = kOffC + kCh;
    __shared__ bf16x8 s_lds[2][kBufSlots];

    // one workgroup per tile (and part of a tile of more than 256 queries):
    // the query features are formed once for all of the tile's candidates
    // neighbouring tiles, which share candidates, on one XCD (one L2)
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int64_t e0 = uniform64(tile_off[t]), e1 = uniform64(tile_off[t + 1]);

    const int lane = lane_id(), w = int(threadIdx.x) / kWave, h = lane / 32;
    const int s = int(blockIdx.y) * kMThreads + int(threadIdx.x);
    const int64_t p = t * tile + s;
    const bool valid = (s < tile) && (p < q);
    float cen[N];
#pragma unroll
    for (int a = 0; a < N; ++a) cen[a] = tcen[t * N + a];

    // The coordinates this lane needs, loaded first and all together (from
    // a valid row, the tile's first, where a row is past the tile's end):
    // its own query's (the wave's half-widths) and its row of each of the
    // two A row blocks.
    float xo[N], xb[2][N];
    bool vrow[2];
    {
        const int64_t pc = valid ? p : t * tile;
#pragma unroll
        for (int a = 0; a < N; ++a) xo[a] = qs[a * q + pc];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int sr = w * kWave + int(blockIdx.y) * kMThreads + rb * 32 + (lane % 32);
            const int64_t pr = t * tile + sr;
            vrow[rb] = (sr < tile) && (pr < q);
            const int64_t prc = vrow[rb] ? pr : t * tile;
#pragma unroll
            for (int a = 0; a < N; ++a) xb[rb][a] = qs[a * q + prc];
        }
    }
    // this wave's half-widths about the centre
    float h2 = 0.0f, hm = 0.0f;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const float ha = wave_max_nonneg(valid ? fabsf(xo[a] - cen[a]) : 0.0f);
        h2 = fmaf(ha, ha, h2);
        hm = fmaxf(hm, ha);
    }
    h2 *= 1.0f + 1.0f / 1048576.0f;

    // A fragments: rows are the wave's queries (two blocks of 32).  Every
    // lane forms all 16 features of each k-step for its row (indices known
    // at compile time), then keeps the half h = lane / 32 it holds.
    bf16x8 ahi[2][KS], alo[2][KS];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const bool vr = vrow[rb];
        float xr[N];
#pragma unroll
        for (int a = 0; a < N; ++a) xr[a] = vr ? xb[rb][a] - cen[a] : 0.0f;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            float f[16];
#pragma unroll
            for (int slot = 0; slot < 16; ++slot) {
                f[slot] = 0.0f;
                if (ks == 0) {
                    if (slot == 0)
                        f[slot] = vr ? 1.0f : 0.0f;
                    else if (slot <= N)
                        f[slot] = xr[slot - 1];
                } else {
                    const int qq = (ks - 1) * 16 + slot;
                    if (kQuad<N>.i[qq] >= 0) f[slot] = xr[kQuad<N>.i[qq]] * xr[kQuad<N>.j[qq]];
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = h ? f[8 + e] : f[e];
                __bf16 hi, lo;
                split_bf16(v, hi, lo);
                ahi[rb][ks][e] = hi;
                alo[rb][ks][e] = lo;
            }
        }
    }
    // all 64 queries of the group valid: no row masking in the group test;
    // none valid (past the tile's end): the wave only loads and meets
    const bool full = ballot(valid) == ~uint64_t(0);
    const bool live = ballot(valid) != 0;
    uint32_t rowvalid = 0;   // bit rb * 16 + r: accumulator element r of row block rb
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r / 4) + 4 * h + (r % 4);
            const int sq = w * kWave + int(blockIdx.y) * kMThreads + rb * 32 + row;
            if (sq < tile && t * tile + sq < q) rowvalid |= 1u << (rb * 16 + r);
        }
    }

    const int ngroups = (tile + kWave - 1) / kWave;
    const int grp = s / kWave;
    unsigned long long n_exam = 0, n_pass = 0;

    // Chunks of kCh entries staged in LDS, double-buffered: the workgroup
    // issues the loads of chunk c + 1 straight into LDS (global_load_lds,
    // 16 bytes per lane, lane l of a wave to slot M0 + l) while it computes
    // chunk c, then waits for them and meets at one barrier.
    // The workgroup is always kMThreads threads (waves whose rows are all
    // past the tile's end only load and meet).  Each region is loaded in
    // rounds of kMThreads slots, a wave's 64 lanes on 64 consecutive slots;
    // a lane on a padding slot or an entry past the list's end loads
    // nothing.
    auto load_region = [&](auto region, int buf, int64_t ch, int nch, int cv) {
        constexpr int R = decltype(region)::value;
        constexpr int off = R == 0 ? 0 : (R == 1 ? kOffB : kOffC);
        constexpr int len = R == 0 ? kCh * kStA : (R == 1 ? kCh * kStB : kCh);
        constexpr int st = R == 0 ? kStA : (R == 1 ? kStB : 1);
        constexpr int units = R == 0 ? 4 : (R == 1 ? kMU : 1);
#pragma unroll
        for (int k = 0; k < (len + kMThreads - 1) / kMThreads; ++k) {
            const int wbase = k * kMThreads + w * kWave;   // this wave's first slot
            if (wbase >= len) break;                       // uniform over the wave
            const int sl = wbase + lane;
            const int j = sl / st, u = sl - j * st;
            // a wave-uniform base and a 32-bit lane offset (in 16-byte units)
            const bf16x8 *base;
            uint32_t o;
            if constexpr (R == 0) {
                base = eb0 + ch * 4;
                o = uint32_t(j * 4 + u);
            } else if constexpr (R == 1) {
                base = mrec;
                o = uint32_t(__shfl(cv, j & (kWave - 1), kWave)) * kMU + uint32_t(u);
            } else {
                base = reinterpret_cast<const bf16x8 *>(ebnd + ch);
                o = uint32_t(j);
            }
            const bf16x8 *src = base + o;
            if (sl < len && u < units && j < nch)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(src),
                    (__attribute__((address_space(3))) void *)(&s_lds[buf][off + wbase]), 16, 0,
                    0);
        }
    };
    auto load_chunk = [&](int buf, int64_t ch, int cv) {
        const int nch = int((e1 - ch < kCh) ? e1 - ch : kCh);   // entries present
        load_region(std::integral_constant<int, 0>{}, buf, ch, nch, cv);
        load_region(std::integral_constant<int, 1>{}, buf, ch, nch, cv);
        load_region(std::integral_constant<int, 2>{}, buf, ch, nch, cv);
    };
    auto cand_of = [&](int64_t ch) { return (ch + lane < e1) ? cand[ch + lane] : 0; };
    if (e0 < e1) load_chunk(0, e0, cand_of(e0));
    int cv_next = cand_of(e0 + kCh);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    uint32_t st[3] = {0u, 0u, 0u};
    int buf = 0;
    for (int64_t ch = e0; ch < e1; ch += kCh) {
        const bool more = ch + kCh < e1;
        if (more) load_chunk(buf ^ 1, ch + kCh, cv_next);
        const int cv_after = cand_of(ch + 2 * kCh);
        const int n = int((e1 - ch < kCh) ? e1 - ch : kCh);
        if constexpr (COUNT) {
            // a group past the tile's end counts its pairs as examined, as
            // the float32 kernel does
            if (!live) n_exam += uint64_t(n);
        }
        for (int cb = 0; live && cb < n; cb += 32) {
            const int jl = cb + (lane % 32);
            const bool jv = jl < n;
            const int jc = jv ? jl : cb;   // idle lanes: a valid row, column ignored
            bf16x8 bhi[KS], blo[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int sl = ks == 0 ? jc * kStA + h * 2
                                       : kOffB + jc * kStB + ((ks - 1) * 2 + h) * 2;
                bhi[ks] = s_lds[buf][sl];
                blo[ks] = s_lds[buf][sl + 1];
            }
            const bf16x8 bdv = s_lds[buf][kOffC + jc];
            const float4 bd = *reinterpret_cast<const float4 *>(&bdv);
            f32x16 acc0 = {}, acc1 = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[0][ks], bhi[ks], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[1][ks], bhi[ks], acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][ks], blo[ks], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][ks], blo[ks], acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][ks], bhi[ks], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][ks], bhi[ks], acc1, 0, 0, 0);
            }
            // certified group test of the entry in this lane's column: the
            // smallest M' over the group's rows, as a signed-integer minimum
            // of the float bits -- exact among non-negative values, and any
            // negative value (rounding below 0) stays negative, which keeps
            // the candidate, as it must
            int mi = 0x7f800000;   // +inf
            if (full) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    mi = min(mi, min(__float_as_int(acc0[r]), __float_as_int(acc1[r])));
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if (rowvalid & (1u << r)) mi = min(mi, __float_as_int(acc0[r]));
                    if (rowvalid & (1u << (16 + r))) mi = min(mi, __float_as_int(acc1[r]));
                }
            }
            const float mn = __int_as_float(mi);
            const float bound =
                kGammaQ * (bd.w * h2 + bd.y * hm + bd.x) + kGammaB * bd.w * bd.z * hm;
            const bool pass = jv && !(mn - bound > skip);
            const uint64_t bal = ballot(pass);
            if constexpr (COUNT) {
                n_exam += uint64_t(n - cb < 32 ? n - cb : 32);
                n_pass += uint64_t(__popc(uint32_t(bal) | uint32_t(bal >> 32)));
            }
            if (lane < 32 && jv && grp < ngroups)
                act[(ch + jl) * ngroups + grp] =
                    uint8_t(((bal >> lane) | (bal >> (lane + 32))) & 1u);
        }
        // the next chunk in LDS, and every wave done with this one
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        buf ^= 1;
        cv_next = cv_after;
    }
    // The pairs the filter kept are evaluated in float32 by the staged code
    // of the float32 kernel (lane = its own query), in ascending entry order
    // per group, each record fetched with wave-uniform loads one pair ahead;
    // the flag becomes the kept decision.  The flags read are this wave's
    // own (written above, complete after the last wait).
    if (live && grp < ngroups) {
        float x[N];
        {
            // the row index made opaque here, so that the compiler does not
            // keep its N addresses live through the loop above
            int pc = int(valid ? s : 0);
            asm volatile("" : "+v"(pc));
            const float *qp = qs + t * tile + pc;
#pragma unroll
            for (int a = 0; a < N; ++a) x[a] = qp[a * q];
        }
        float bufA[Lay::PF], bufB[Lay::PF];
        for (int64_t ch = e0; ch < e1; ch += kWave) {
            const int n = int((e1 - ch < kWave) ? e1 - ch : kWave);
            uint8_t *fl = act + (ch + lane) * ngroups + grp;
            uint64_t todo = ballot(lane < n && *fl != 0);
            if (todo == 0) continue;
            const int vidx = (lane < n) ? cand[ch + lane] : 0;
            uint32_t kept = 0;
            int ja = __builtin_ctzll(todo);
            todo &= todo - 1;
            load_block<N>(bufA, grec + int64_t(__builtin_amdgcn_readlane(vidx, ja)) * Lay::R);
            while (ja >= 0) {
                const int64_t ia = __builtin_amdgcn_readlane(vidx, ja);
                const int jb = todo ? __builtin_ctzll(todo) : -1;
                __builtin_amdgcn_s_waitcnt(kWaitScalar);
                if (jb >= 0) {
                    todo &= todo - 1;
                    load_block<N>(bufB,
                                  grec + int64_t(__builtin_amdgcn_readlane(vidx, jb)) * Lay::R);
                }
                if (eval_pair<N, true, OUT, COUNT>(bufA, grec + ia * Lay::R, x, valid, skip, f0,
                                                   f1, f2, st))
                    kept = (lane == ja) ? 1u : kept;
#pragma unroll
                for (int e = 0; e < Lay::PF; ++e) bufA[e] = bufB[e];
                ja = jb;
            }
            if (lane < n) *fl = uint8_t(kept);
        }
    }
    if constexpr (COUNT) {
        if (lane == 0 && grp < ngroups) {
            atomicAdd(&stats[0], n_exam);
            atomicAdd(&stats[1], n_pass);
            atomicAdd(&stats[2], static_cast<unsigned long long>(st[0]));
            atomicAdd(&stats[3], static_cast<unsigned long long>(st[1]));
            atomicAdd(&stats[4], static_cast<unsigned long long>(st[2]));
        }
    }
    if constexpr (OUT) {
        if (valid) {
            const int64_t o = perm[p];
            out[o * 3 + 0] = f0;
            out[o * 3 + 1] = f1;
            out[o * 3 + 2] = f2;
        }
    }
}

template <int N>
hipError_t mfma_prepare_n(ngd_cull *c, hipStream_t s)
{
    hipError_t e;
    if (c->mrec_seq != c->build_seq) {
        // once per cull build: per-Gaussian quadratic coefficients (unless
        // the build launched them beside its own work) and the per-entry
        // centred coefficients (the tile centres come with the cull's tile
        // bounds)
        if (c->coef_seq != c->build_seq && c->k > 0)
            k_mfma_coef<N><<<unsigned((c->k + 255) / 256), 256, 0, s>>>(
                c->k, c->grec.as<float>(), c->mrec.as<__bf16>(), c->mrow.as<float>());
        if (c->total > 0)
            k_mfma_entry<N><<<unsigned((c->total + 255) / 256), 256, 0, s>>>(
                c->total, c->cand.as<int32_t>(), c->ent_tile.as<int32_t>(), c->grec.as<float>(),
                c->mrow.as<float>(), c->tcen.as<float>(), c->eb0.as<bf16x8>(),
                c->ebnd.as<float4>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        c->mrec_seq = c->build_seq;
    }
    return hipSuccess;
}

template <int N>
hipError_t mfma_n(ngd_cull *c, float *out, unsigned long long *stats, hipStream_t s)
{
    const int tile = c->params.tile;
    const unsigned gy = unsigned((tile + kMThreads - 1) / kMThreads);
    const float skip = float(-std::log2(double(c->params.tau)) + kSkipLog2Margin);
    hipError_t e = mfma_prepare_n<N>(c, s);
    if (e != hipSuccess) return e;
    if (c->ntiles > 0) {
        // every tile's workgroup writes its queries' colours (zeros for a
        // tile with no candidates)
        const dim3 grid(unsigned(c->ntiles), gy);
        auto go = [&](auto kern, float *o, unsigned long long *st) {
            kern<<<grid, kMThreads, 0, s>>>(c->q, tile, c->mrec.as<bf16x8>(), c->eb0.as<bf16x8>(),
                                            c->ebnd.as<float4>(), c->tcen.as<float>(),
                                            c->qs.as<float>(), c->grec.as<float>(),
                                            c->tile_off.as<int64_t>(), c->cand.as<int32_t>(),
                                            c->perm.as<int32_t>(), skip, c->act.as<uint8_t>(), o,
                                            st);
        };
        if (stats)
            go(k_mfma_filter<N, false, true>, nullptr, stats);
        else if (out)
            go(k_mfma_filter<N, true, false>, out, nullptr);
        else
            go(k_mfma_filter<N, false, false>, nullptr, nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t mfma_rec_bytes(int n)
{
    const int t = n * (n + 1) / 2;
    return size_t((t + 15) / 16) * 32 * sizeof(uint16_t);
}

size_t mfma_entry_bytes() { return 4 * sizeof(bf16x8) + sizeof(float4); }

hipError_t launch_mfma_coef(int n, ngd_cull *c, hipStream_t s)
{
    if (c->k == 0) return hipSuccess;
    switch (n) {
#define NGD_CASE(NN)                                                                           \
    case NN:                                                                                   \
        k_mfma_coef<NN><<<unsigned((c->k + 255) / 256), 256, 0, s>>>(                          \
            c->k, c->grec.as<float>(), c->mrec.as<__bf16>(), c->mrow.as<float>());             \
        return hipGetLastError();
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mfma_prepare(const ngd_mixture *mix, ngd_cull *c, hipStream_t s)
{
    if (c->q == 0 || c->ntiles == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return mfma_prepare_n<NN>(c, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_eval_mfma(const ngd_mixture *mix, ngd_cull *c, float *out,
                            unsigned long long *stats, hipStream_t s)
{
    if (c->q == 0 || c->ntiles == 0) return hipSuccess;
    switch (mix->n) {
#define NGD_CASE(NN) \
    case NN: return mfma_n<NN>(c, out, stats, s);
        NGD_CASE(1) NGD_CASE(2) NGD_CASE(3) NGD_CASE(4) NGD_CASE(5) NGD_CASE(6)
        NGD_CASE(7) NGD_CASE(8) NGD_CASE(9) NGD_CASE(10) NGD_CASE(11) NGD_CASE(12)
#undef NGD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ngd
