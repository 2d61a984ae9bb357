// k-d ordering of points in projection space, the tiling of the cull.
//
// Definition (shared with the CPU re-implementation): a run of n points is
// cut in units of u = leaf while n > leaf, else of u = sub (sub <= leaf);
// it needs T = ceil(n/u) units, and its first ceil(T/2)*u points in the
// order (value on the split projection, then position in the run) go left
// and the rest right, each side keeping its relative order.  The split
// projection is the one of largest extent (max - min) over the run, the
// first such on ties.  Runs of at most `sub` points are leaves; the runs of
// at most `leaf` points (tiles) are those of a split with sub = leaf, the
// finer splits only reorder inside them.  Because every split is an exact
// rank split on a stable order, run boundaries depend only on
// (n, leaf, sub), and the host lays them out level by level.
//
// Upper levels (nodes of more than kLocalMax points) run one level at a
// time over all of the level's nodes, each node cut into slices (one
// workgroup each), in five launches:
//   hist 0   per slice of kHistSlice points: the node's split projection
//            (largest extent, from the node's min / max accumulated by the
//            previous level's scatter; for the root by a pass over its
//            slices), then the histogram of the first radix digit (11, 11,
//            10 bits of the order-preserving key), added into the node's
//            round-0 histogram
//   hist 1,2 per slice: the bin of the previous round's histogram that holds
//            the rank n_left (every workgroup of the node finds the same; the
//            node's first records it), then the histogram of the next digit
//            among the points that match the digits found so far
//   count    per slice of kSlice points: the last digit's bin, which
//            completes the pivot key (the first point that goes right); the
//            points below / equal to it
//   scatter  per slice: offsets from the node's earlier slices' counts,
//            stable ranks by workgroup prefix sums in position order; index
//            and projection values move to the next buffer, the children's
//            min / max are accumulated for the next split, and the node's
//            histograms are cleared for the next level
// Nodes of at most kLocalMax points finish their whole subtree in one
// workgroup each (k_kd_local): the order and the sort keys stay in LDS, and
// every level of the subtree is one bitonic sort of (run, key, position)
// over blocks of the smallest power-of-two length that holds every run.
#include <algorithm>
#include <map>
#include <vector>

#include "ngd_internal.hpp"
#include "wave.hpp"

namespace ngd {
namespace {

constexpr int kThreads = 256;
constexpr int kSlice = 1024;        // points per scatter / count workgroup
constexpr int kHistSlice = 4096;    // points per histogram workgroup
constexpr int kBins = 2048;
constexpr int kShift[3] = {21, 10, 0};
constexpr int kWidth[3] = {11, 11, 10};

constexpr int kHistThreads = 512;

constexpr int kLocalMax = 1024;    // points per subtree workgroup (<= 4096: 12-bit positions)
constexpr unsigned kWideLocalBlocks = 512;   // subtrees for the 512-thread variant
// Min / max key slots come in kExtRep planes of max_nodes x P x 2: a
// workgroup merges into plane (blockIdx.x mod kExtRep), so that the atomics
// of the many workgroups of one node (all of them, at the root) spread over
// as many cache lines; readers reduce the planes.
constexpr int kExtRep = 16;
constexpr int kRootPer = 4;        // points per thread of the root's extents
constexpr int kLocalRuns = 128;     // runs per subtree (8-bit run ids)
constexpr int kLocalSplit = 64;     // runs split at one level of a subtree

// node table row: start, size, n_left (-1: leaf), first slice, end slice,
// first child's index in the next level (-1: none), first histogram slice,
// end histogram slice
constexpr int kNodeCols = 8;
// slice table row: start, length, node
constexpr int kSliceCols = 3;

// The plane of min / max key slots a workgroup merges into.
__device__ __forceinline__ uint32_t *ext_plane(uint32_t *ext, int64_t max_nodes, int P)
{
    return ext + int64_t(blockIdx.x % kExtRep) * max_nodes * 2 * P;
}

// Clears the histograms; resets the root's min / max key slots (P
// projections) of planes first_plane.. to their identities.
__global__ __launch_bounds__(kThreads) void k_kd_zero(int32_t *__restrict__ p, int64_t n,
                                                      uint32_t *__restrict__ ext, int P,
                                                      int64_t max_nodes, int first_plane)
{
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) p[i] = 0;
    if (i >= int64_t(P) * first_plane && i < int64_t(P) * kExtRep) {
        uint32_t *e = ext + (i / P) * max_nodes * 2 * P + 2 * (i % P);
        e[0] = 0xffffffffu;
        e[1] = 0u;
    }
}

// Workgroup min / max of per-thread keys for projections j < P, merged into
// ext[(node * P + j) * 2 + {0, 1}] by atomics (order-independent).
template <int PMAX>
__device__ void block_merge_ext(const uint32_t (&kmin)[PMAX], const uint32_t (&kmax)[PMAX],
                                int P, uint32_t *ext, int64_t node)
{
    __shared__ uint32_t smin[kThreads / kWave][PMAX], smax[kThreads / kWave][PMAX];
    const int w = threadIdx.x / kWave;
    // wave minima / maxima by DPP (no LDS traffic), totals in lane 63
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
        if (j < P) {
            const uint32_t a = wave_umin_dpp(kmin[j]), b = wave_umax_dpp(kmax[j]);
            if (lane_id() == kWave - 1) {
                smin[w][j] = a;
                smax[w][j] = b;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < P) {
        const int j = threadIdx.x;
        uint32_t a = 0xffffffffu, b = 0u;
#pragma unroll
        for (int i = 0; i < kThreads / kWave; ++i) {
            a = min(a, smin[i][j]);
            b = max(b, smax[i][j]);
        }
        if (a != 0xffffffffu) atomicMin(&ext[(node * P + j) * 2 + 0], a);
        if (b != 0u) atomicMax(&ext[(node * P + j) * 2 + 1], b);
    }
    __syncthreads();
}

// The root's min / max: kRootPer points per thread, all P of their loads
// in flight together.
template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_kd_root_ext(int64_t n, int P,
                                                          const float *__restrict__ vin,
                                                          uint32_t *__restrict__ ext,
                                                          int64_t max_nodes)
{
    uint32_t kmin[PMAX], kmax[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
        kmin[j] = 0xffffffffu;
        kmax[j] = 0u;
    }
    const int64_t i0 = int64_t(blockIdx.x) * kThreads * kRootPer + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kRootPer; ++u) {
        const int64_t i = i0 + int64_t(u) * kThreads;
        if (i < n) {
#pragma unroll
            for (int j = 0; j < PMAX; ++j) {
                if (j < P) {
                    const uint32_t key = orderable(vin[int64_t(j) * n + i]);
                    kmin[j] = min(kmin[j], key);
                    kmax[j] = max(kmax[j], key);
                }
            }
        }
    }
    block_merge_ext<PMAX>(kmin, kmax, P, ext_plane(ext, max_nodes, P), 0);
}

// Block exclusive scan of one count per thread (THREADS threads).  Every
// caller scans counts of points of one node, whose wave sums stay below
// 2^31 (the point count is): the wave scan runs in 32 bits by DPP, the
// workgroup's combination in 64.
template <int THREADS = kThreads>
__device__ int64_t block_exscan(int64_t v, int64_t *total)
{
    __shared__ int64_t wt[THREADS / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int64_t inc = wave_inclusive_scan(int(v));
    if (lane == kWave - 1) wt[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < THREADS / kWave; ++i) {
        before += (i < w) ? wt[i] : 0;
        all += wt[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// One round of the radix selection, by a whole workgroup: the bin of the
// node's histogram h (2^width bins, of the points matching `pre`) that holds
// rank r; returns the extended prefix and the rank inside that bin.
template <int THREADS>
__device__ void block_select(const int32_t *__restrict__ h, int width, uint32_t pre, int64_t r,
                             uint32_t *out_pre, int64_t *out_rank)
{
    __shared__ uint32_t s_pre;
    __shared__ int64_t s_rank;
    constexpr int kMaxPer = kBins / THREADS;
    const int per = (1 << width) / THREADS;
    int32_t cnt[kMaxPer];
    int64_t mine = 0;
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
        cnt[i] = i < per ? h[threadIdx.x * per + i] : 0;
        mine += cnt[i];
    }
    int64_t tot;
    int64_t cum = block_exscan<THREADS>(mine, &tot);
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
        if (i < per && r >= cum && r < cum + cnt[i]) {
            s_pre = (pre << width) | uint32_t(threadIdx.x * per + i);
            s_rank = r - cum;
        }
        cum += cnt[i];
    }
    __syncthreads();
    *out_pre = s_pre;
    *out_rank = s_rank;
}

// Per slice of kHistSlice points, one round of the radix selection of the
// node's pivot.  Round 0 first picks the node's split projection (its
// first slice records it and resets the children's min / max slots);
// rounds 1 and 2 first finish the previous round (its first slice records
// the prefix and rank).  The histogram of the round's digit among the
// points that match the prefix is added into the node's histogram of the
// round (integer atomics: the sum does not depend on their order).
// sel_pre / sel_rank: 3 x max_nodes, the state after rounds 0, 1, 2.
__global__ __launch_bounds__(kHistThreads) void k_kd_hist(
    const int64_t *__restrict__ nodes, const int64_t *__restrict__ slices, int64_t node0,
    int64_t hslice0, int64_t max_nodes, int64_t n, int P, int round,
    const float *__restrict__ vin, const uint32_t *__restrict__ ext,
    uint32_t *__restrict__ ext_next, int32_t *__restrict__ dim, uint32_t *__restrict__ sel_pre,
    int64_t *__restrict__ sel_rank, int32_t *__restrict__ hist)
{
    __shared__ int h[kBins];
    __shared__ float s_ext[32];
    __shared__ int s_dim;
    const int64_t sl = blockIdx.x;
    const int64_t s0 = slices[sl * kSliceCols + 0], len = slices[sl * kSliceCols + 1];
    const int64_t nd = slices[sl * kSliceCols + 2] - node0;
    const int64_t *row = nodes + nd * kNodeCols;
    const int64_t nleft = row[2];
    const bool first = sl + hslice0 == row[6];
    if (nleft < 0) {   // a leaf (uniform over the workgroup)
        if (round == 0 && first && threadIdx.x == 0) dim[nd] = -1;
        return;
    }
    // the slice's keys of projection d, loaded before the previous round's
    // selection so that the two latencies overlap
    constexpr int kPer = kHistSlice / kHistThreads;
    uint32_t keys[kPer];
    auto load_keys = [&](int d) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t i = threadIdx.x + int64_t(u) * kHistThreads;
            keys[u] = i < len ? orderable(vin[int64_t(d) * n + s0 + i]) : 0u;
        }
    };
    uint32_t pre = 0u;
    int d;
    if (round == 0) {
        // the projection of largest extent, the first on ties
        if (int(threadIdx.x) < P) {
            const int j = threadIdx.x;
            uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll 4
            for (int e = 0; e < kExtRep; ++e) {
                const uint32_t *x = ext + int64_t(e) * max_nodes * 2 * P + (nd * P + j) * 2;
                lo = min(lo, x[0]);
                hi = max(hi, x[1]);
            }
            s_ext[j] = from_orderable(hi) - from_orderable(lo);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int best = 0;
            for (int j = 1; j < P; ++j)
                if (s_ext[j] > s_ext[best]) best = j;
            s_dim = best;
        }
        __syncthreads();
        d = s_dim;
        load_keys(d);
        if (first) {
            if (threadIdx.x == 0) dim[nd] = d;
            const int64_t ch = row[5];
            if (ext_next && ch >= 0) {   // both children's slots, every plane
                for (int t = threadIdx.x; t < 2 * P * kExtRep; t += kHistThreads) {
                    uint32_t *x = ext_next + int64_t(t / (2 * P)) * max_nodes * 2 * P +
                                  (ch * P + t % (2 * P)) * 2;
                    x[0] = 0xffffffffu;
                    x[1] = 0u;
                }
            }
        }
    } else {
        d = dim[nd];
        load_keys(d);
        const uint32_t p0 = round == 1 ? 0u : sel_pre[nd];
        const int64_t r0 = round == 1 ? nleft : sel_rank[nd];
        int64_t r1;
        block_select<kHistThreads>(hist + ((round - 1) * max_nodes + nd) * kBins,
                                   kWidth[round - 1], p0, r0, &pre, &r1);
        if (first && threadIdx.x == 0) {
            sel_pre[(round - 1) * max_nodes + nd] = pre;
            sel_rank[(round - 1) * max_nodes + nd] = r1;
        }
    }
    for (int b = threadIdx.x; b < kBins; b += kHistThreads) h[b] = 0;
    __syncthreads();
    const int shift = kShift[round], width = kWidth[round];
    const uint32_t mask = (1u << width) - 1u;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t key = keys[u];
        const bool valid = threadIdx.x + int64_t(u) * kHistThreads < len;
        const bool match = (round == 0) || ((key >> (shift + width)) == pre);
        if (valid && match) atomicAdd(&h[(key >> shift) & mask], 1);
    }
    __syncthreads();
    int32_t *nh = hist + (round * max_nodes + nd) * kBins;
    for (int b = threadIdx.x; b < kBins; b += kHistThreads)
        if (h[b]) atomicAdd(&nh[b], h[b]);
}

// Per slice of kSlice points: the last round of the selection (the node's
// first slice records the pivot key and the number of pivot-equal points
// that go left), then the slice's points below and equal to the pivot.
__global__ __launch_bounds__(kThreads) void k_kd_count(
    const int64_t *__restrict__ nodes, const int64_t *__restrict__ slices, int64_t node0,
    int64_t slice0, int64_t max_nodes, int64_t n, const float *__restrict__ vin,
    const int32_t *__restrict__ dim, uint32_t *__restrict__ sel_pre,
    int64_t *__restrict__ sel_rank, const int32_t *__restrict__ hist, int64_t *__restrict__ cnt)
{
    const int64_t sl = blockIdx.x;
    const int64_t s0 = slices[sl * kSliceCols + 0], len = slices[sl * kSliceCols + 1];
    const int64_t nd = slices[sl * kSliceCols + 2] - node0;
    const int d = dim[nd];
    int64_t less = 0, eq = 0;
    if (d >= 0) {   // uniform
        // the slice's keys first: their loads overlap the selection
        constexpr int kPer = kSlice / kThreads;
        uint32_t keys[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t i = threadIdx.x + int64_t(u) * kThreads;
            keys[u] = i < len ? orderable(vin[int64_t(d) * n + s0 + i]) : 0u;
        }
        uint32_t pivot;
        int64_t r;
        block_select<kThreads>(hist + (2 * max_nodes + nd) * kBins, kWidth[2],
                               sel_pre[max_nodes + nd], sel_rank[max_nodes + nd], &pivot, &r);
        if (sl + slice0 == nodes[nd * kNodeCols + 3] && threadIdx.x == 0) {
            sel_pre[2 * max_nodes + nd] = pivot;
            sel_rank[2 * max_nodes + nd] = r;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const bool valid = threadIdx.x + int64_t(u) * kThreads < len;
            less += valid && keys[u] < pivot;
            eq += valid && keys[u] == pivot;
        }
    }
    int64_t tl, te;
    block_exscan(less, &tl);
    block_exscan(eq, &te);
    if (threadIdx.x == 0) {
        cnt[sl * 2 + 0] = tl;
        cnt[sl * 2 + 1] = te;
    }
}

// Block-wide exclusive prefix count of a flag (position order), with total.
__device__ __forceinline__ int block_flag_scan(bool f, int *total)
{
    __shared__ int wc[kThreads / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const uint64_t b = ballot(f);
    const int before_lane = __popcll(b & lanemask_lt());
    if (lane == 0) wc[w] = __popcll(b);
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kThreads / kWave; ++i) {
        before += (i < w) ? wc[i] : 0;
        all += wc[i];
    }
    __syncthreads();
    *total = all;
    return before + before_lane;
}

template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_kd_scatter(
    const int64_t *__restrict__ nodes, const int64_t *__restrict__ slices, int64_t node0,
    int64_t slice0, int64_t n, int P, const int32_t *__restrict__ idx_in,
    const float *__restrict__ vin, const int32_t *__restrict__ dim,
    const uint32_t *__restrict__ prefix, const int64_t *__restrict__ rank,
    const int64_t *__restrict__ cnt, int32_t *__restrict__ idx_out, float *__restrict__ vout,
    uint32_t *__restrict__ ext_next, int32_t *__restrict__ hist, int64_t max_nodes)
{
    const int64_t sl = blockIdx.x;
    const int64_t s0 = slices[sl * kSliceCols + 0], len = slices[sl * kSliceCols + 1];
    const int64_t nd = slices[sl * kSliceCols + 2] - node0;
    const int64_t *row = nodes + nd * kNodeCols;
    const int64_t start = row[0], size = row[1], nleft = row[2];
    const int d = dim[nd];
    if (d < 0) {   // a leaf: its points stay where they are
        for (int64_t i = threadIdx.x; i < len; i += kThreads) {
            const int64_t pos = s0 + i;
            idx_out[pos] = idx_in ? idx_in[pos] : int32_t(pos);
#pragma unroll
            for (int j = 0; j < PMAX; ++j)
                if (j < P) vout[int64_t(j) * n + pos] = vin[int64_t(j) * n + pos];
        }
        return;
    }
    const int64_t sb = row[3] - slice0;   // the node's first slice
    if (sl == sb) {   // the node's histograms, clean for the next level
        for (int r = 0; r < 3; ++r)
            for (int b = threadIdx.x; b < kBins; b += kThreads)
                hist[(r * max_nodes + nd) * kBins + b] = 0;
    }
    // points below the pivot, and equal to it, in the node's earlier slices
    int64_t l_mine = 0, e_mine = 0;
    for (int64_t s = sb + threadIdx.x; s < sl; s += kThreads) {
        l_mine += cnt[s * 2 + 0];
        e_mine += cnt[s * 2 + 1];
    }
    int64_t l_before, e_before;
    block_exscan(l_mine, &l_before);
    block_exscan(e_mine, &e_before);
    const uint32_t pivot = prefix[nd];
    const int64_t need = rank[nd];   // pivot-equal points that go left
    const int64_t lo = l_before + (need < e_before ? need : e_before);
    const int64_t ro = (s0 - start) - lo;
    const int64_t ch = row[5];
    const bool track = ext_next != nullptr && ch >= 0;
    uint32_t lmin[PMAX], lmax[PMAX], rmin[PMAX], rmax[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
        lmin[j] = rmin[j] = 0xffffffffu;
        lmax[j] = rmax[j] = 0u;
    }
    int64_t run_eq = 0, run_left = 0;
    for (int64_t base = 0; base < len; base += kThreads) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < len;
        const int64_t pos = s0 + i;
        // the point's values first, so their loads overlap the scans
        float v[PMAX];
#pragma unroll
        for (int j = 0; j < PMAX; ++j) v[j] = (valid && j < P) ? vin[int64_t(j) * n + pos] : 0.0f;
        const int32_t id = valid ? (idx_in ? idx_in[pos] : int32_t(pos)) : 0;
        const uint32_t key = valid ? orderable(vin[int64_t(d) * n + pos]) : 0xffffffffu;
        const bool is_less = valid && key < pivot;
        const bool is_eq = valid && key == pivot;
        int teq, tleft;
        const int64_t eq_rank = e_before + run_eq + block_flag_scan(is_eq, &teq);
        const bool left = is_less || (is_eq && eq_rank < need);
        const int64_t left_rank = run_left + block_flag_scan(left, &tleft);
        const int64_t dest = left ? start + lo + left_rank : start + nleft + ro + (i - left_rank);
        run_eq += teq;
        run_left += tleft;
        // every destination lies in the node's own run (the counts agree);
        // the test only guards the buffers should they ever not
        if (valid && dest >= start && dest < start + size) {
            idx_out[dest] = id;
#pragma unroll
            for (int j = 0; j < PMAX; ++j) {
                if (j < P) {
                    vout[int64_t(j) * n + dest] = v[j];
                    if (track) {
                        const uint32_t k = orderable(v[j]);
                        if (left) {
                            lmin[j] = min(lmin[j], k);
                            lmax[j] = max(lmax[j], k);
                        } else {
                            rmin[j] = min(rmin[j], k);
                            rmax[j] = max(rmax[j], k);
                        }
                    }
                }
            }
        }
    }
    if (track) {   // uniform
        uint32_t *plane = ext_plane(ext_next, max_nodes, P);
        block_merge_ext<PMAX>(lmin, lmax, P, plane, ch);
        block_merge_ext<PMAX>(rmin, rmax, P, plane, ch + 1);
    }
}

// ---- subtrees of at most kLocalMax points, one workgroup each -------------

template <int THREADS>
__device__ int local_exscan(int v, int *total)
{
    __shared__ int wt[THREADS / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) wt[w] = inc;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < THREADS / kWave; ++i) {
        before += (i < w) ? wt[i] : 0;
        all += wt[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <int PMAX, int kLocalThreads>
__global__ __launch_bounds__(kLocalThreads) void k_kd_local(
    const int64_t *__restrict__ nodes, int64_t n, int P, int leaf, int sub,
    const int32_t *__restrict__ idx_in, const float *__restrict__ vin,
    int32_t *__restrict__ idx_out, float *__restrict__ vout)
{
    __shared__ uint16_t ord[2][kLocalMax];
    __shared__ uint16_t lpre[kLocalMax];
    __shared__ uint8_t flag[kLocalMax];
    __shared__ uint8_t run_of[kLocalMax];
    __shared__ int rs[kLocalRuns], rl[kLocalRuns], rn[kLocalRuns], rd[kLocalRuns], rsi[kLocalRuns];
    __shared__ int split_list[kLocalSplit];
    // min / max slots of the splitting runs; during the sort (after the
    // split projections are chosen) the same memory exchanges keys between
    // waves
    __shared__ uint32_t ext_buf[2][kLocalSplit][PMAX];
    static_assert(sizeof(ext_buf) >= kLocalMax * sizeof(uint64_t), "key exchange fits");
    auto &emin = ext_buf[0];
    auto &emax = ext_buf[1];
    uint64_t *keys = reinterpret_cast<uint64_t *>(&ext_buf[0][0][0]);
    __shared__ int nruns_s, nsplit_s, sortlen_s;

    const int64_t *row = nodes + int64_t(blockIdx.x) * kNodeCols;
    const int64_t start = row[0];
    const int m = int(row[1]);   // <= kLocalMax, with at most kLocalRuns leaves (host plan)
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    constexpr int kWaves = kLocalThreads / kWave;
    int m2 = 1;
    while (m2 < m) m2 <<= 1;
    constexpr int kPer = kLocalMax / kLocalThreads;   // positions per thread
    constexpr int kSpan = kPer * kWave;   // elements per wave
    static_assert(kPer * kLocalThreads == kLocalMax, "elements: lane, register, wave bits");

    for (int i = tid; i < m; i += kLocalThreads) {
        ord[0][i] = uint16_t(i);
        run_of[i] = 0;
    }
    if (tid == 0) {
        rs[0] = 0;
        rl[0] = m;
        nruns_s = 1;
    }
    __syncthreads();
    int cur = 0;
    while (true) {
        // runs that split at this level, and where
        if (tid == 0) {
            int ns = 0;
            for (int b = 0; b < nruns_s; ++b) {
                const int len = rl[b];
                if (len > sub && ns < kLocalSplit) {
                    const int u = len > leaf ? leaf : sub;
                    const int T = (len + u - 1) / u;
                    rn[b] = ((T + 1) / 2) * u;
                    rsi[b] = ns;
                    split_list[ns++] = b;
                } else {
                    rn[b] = -1;
                    rsi[b] = -1;
                }
            }
            nsplit_s = ns;
            // every run inside one aligned block of L positions (L a power
            // of two): sorting each block sorts every run
            int maxlen = 1;
            for (int b = 0; b < nruns_s; ++b) maxlen = rl[b] > maxlen ? rl[b] : maxlen;
            int L = 1;
            while (L < maxlen) L <<= 1;
            for (int b = 0; b < nruns_s; ++b)
                if (rs[b] / L != (rs[b] + rl[b] - 1) / L) L = m2;
            sortlen_s = L < m2 ? L : m2;
        }
        __syncthreads();
        const int nsplit = nsplit_s;
        if (nsplit == 0) break;
        // extent of every projection over every splitting run.  Each wave
        // covers kSpan consecutive positions, each lane kPer consecutive ones
        // of them: when every lane's positions lie in one splitting run (or
        // past the end), which holds for runs aligned to kPer, the lane first
        // reduces its own positions in registers; otherwise the wave takes
        // its span 64 positions at a time.  Then one DPP min / max per run
        // present in the wave and projection, merged by LDS atomics.
        for (int t = tid; t < nsplit * PMAX; t += kLocalThreads) {
            emin[t / PMAX][t % PMAX] = 0xffffffffu;
            emax[t / PMAX][t % PMAX] = 0u;
        }
        __syncthreads();
        {
            auto merge = [&](int si, const uint32_t (&lo)[PMAX], const uint32_t (&hi)[PMAX]) {
                uint64_t todo = ballot(si >= 0);
                while (todo) {
                    const int src = __ffsll((unsigned long long)todo) - 1;
                    const int cur_si = __builtin_amdgcn_readlane(si, src);
                    const bool mine = si == cur_si;
                    todo &= ~ballot(mine);
#pragma unroll
                    for (int j = 0; j < PMAX; ++j) {
                        if (j < P) {
                            const uint32_t a = wave_umin_dpp(mine ? lo[j] : 0xffffffffu);
                            const uint32_t c = wave_umax_dpp(mine ? hi[j] : 0u);
                            if (lane == kWave - 1) {
                                atomicMin(&emin[cur_si][j], a);
                                atomicMax(&emax[cur_si][j], c);
                            }
                        }
                    }
                }
            };
            const int p0 = w * kSpan + lane * kPer;
            int sl[kPer];
            int lr = -1;
            bool same = true;
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                sl[u] = p0 + u < m ? rsi[run_of[p0 + u]] : -1;
                if (sl[u] >= 0) {
                    if (lr < 0) lr = sl[u];
                    else if (sl[u] != lr) same = false;
                }
            }
            if (ballot(!same) == 0) {
                uint32_t lo[PMAX], hi[PMAX];
#pragma unroll
                for (int j = 0; j < PMAX; ++j) {
                    lo[j] = 0xffffffffu;
                    hi[j] = 0u;
                }
                // all of the lane's loads issued together (positions outside
                // a splitting run read a valid point and are left out)
                int ou[kPer];
                bool in[kPer];
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    in[u] = p0 + u < m && sl[u] >= 0;
                    ou[u] = in[u] ? ord[cur][p0 + u] : 0;
                }
                // four projections per round: the workgroup's gathers then
                // stay within 4 x 4 KB of the subtree's values at a time,
                // which the L2 keeps while every lane reads them
#pragma unroll
                for (int j0 = 0; j0 < PMAX; j0 += 4) {
                    float v[4][kPer];
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                        for (int u = 0; u < kPer; ++u)
                            v[jj][u] = j0 + jj < P ? vin[int64_t(j0 + jj) * n + start + ou[u]] : 0.0f;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int j = j0 + jj;
                        if (j >= P) continue;
#pragma unroll
                        for (int u = 0; u < kPer; ++u) {
                            if (!in[u]) continue;
                            const uint32_t k = orderable(v[jj][u]);
                            lo[j] = min(lo[j], k);
                            hi[j] = max(hi[j], k);
                        }
                    }
                    // each round's loads complete before the next round's
                    // are issued
                    __builtin_amdgcn_s_waitcnt(0);
                }
                merge(lr, lo, hi);
            } else {
#pragma unroll 1
                for (int u = 0; u < kPer; ++u) {
                    const int i = w * kSpan + u * kWave + lane;
                    const int si = i < m ? rsi[run_of[i]] : -1;
                    uint32_t kv[PMAX];
#pragma unroll
                    for (int j = 0; j < PMAX; ++j)
                        kv[j] = (j < P && si >= 0)
                                    ? orderable(vin[int64_t(j) * n + start + ord[cur][i]])
                                    : 0u;
                    merge(si, kv, kv);
                }
            }
        }
        __syncthreads();
        for (int si = tid; si < nsplit; si += kLocalThreads) {
            int best = 0;
            float best_ext = 0.0f;
            for (int j = 0; j < P; ++j) {
                const float e = from_orderable(emax[si][j]) - from_orderable(emin[si][j]);
                if (j == 0 || e > best_ext) {
                    best = j;
                    best_ext = e;
                }
            }
            rd[split_list[si]] = best;
        }
        __syncthreads();
        // sort keys (run, key on the run's split projection, position); runs
        // that do not split sort by (run, position), i.e. stay in place.
        // Element e = w * kSpan + r * 64 + lane is register r of that lane.
        uint64_t kr[kPer];
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int i = w * kSpan + r * kWave + lane;
            uint64_t key = ~uint64_t(0);
            if (i < m) {
                const int b = run_of[i];
                key = (uint64_t(b) << 44) | uint64_t(i);
                if (rn[b] >= 0) {
                    const float v = vin[int64_t(rd[b]) * n + start + ord[cur][i]];
                    key |= uint64_t(orderable(v)) << 12;
                }
            }
            kr[r] = key;
        }
        // bitonic sort of every aligned block of L keys, ascending (the last
        // merge of a block sorts it up whatever its position); elements past
        // m2 hold the largest key and stay in their own blocks.  Partners at
        // distance j < 64 are lanes of the wave, at j < kSpan registers of
        // the thread, further off other waves (through LDS).
        const int L = sortlen_s;
        for (int k = 2; k <= L; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (j >= kSpan) {   // uniform
#pragma unroll
                    for (int r = 0; r < kPer; ++r) keys[w * kSpan + r * kWave + lane] = kr[r];
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < kPer; ++r) {
                        const int e = w * kSpan + r * kWave + lane;
                        const uint64_t o = keys[e ^ j];
                        const bool up = k == L || (e & k) == 0;
                        const bool keep_min = ((e & j) == 0) == up;
                        kr[r] = keep_min ? (kr[r] < o ? kr[r] : o) : (kr[r] > o ? kr[r] : o);
                    }
                    __syncthreads();
                } else if (j >= kWave) {
                    const int rj = j / kWave;
#pragma unroll
                    for (int r = 0; r < kPer; ++r) {
                        if (r & rj) continue;
                        const int e = w * kSpan + r * kWave + lane;
                        const bool up = k == L || (e & k) == 0;
                        const uint64_t a = kr[r], c = kr[r | rj];
                        if ((a > c) == up) {
                            kr[r] = c;
                            kr[r | rj] = a;
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < kPer; ++r) {
                        const int e = w * kSpan + r * kWave + lane;
                        const uint64_t o = __shfl_xor(kr[r], j, kWave);
                        const bool up = k == L || (e & k) == 0;
                        const bool keep_min = ((e & j) == 0) == up;
                        kr[r] = keep_min ? (kr[r] < o ? kr[r] : o) : (kr[r] > o ? kr[r] : o);
                    }
                }
            }
        }
        // left flags by old position: sorted rank inside the run < n_left
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int rank = w * kSpan + r * kWave + lane;
            if (rank >= m) continue;
            const uint64_t key = kr[r];
            const int i = int(key & 0xfffu), b = int(key >> 44);
            flag[i] = (rn[b] >= 0 && rank - rs[b] < rn[b]) ? 1 : 0;
        }
        __syncthreads();
        {
            int c[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * tid + q;
                c[q] = i < m ? flag[i] : 0;
                sum += c[q];
            }
            int tot;
            int run = local_exscan<kLocalThreads>(sum, &tot);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * tid + q;
                if (i < m) lpre[i] = uint16_t(run);
                run += c[q];
            }
        }
        __syncthreads();
        // stable partition of every splitting run
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int i = tid + q * kLocalThreads;
            if (i >= m) break;
            const int b = run_of[i];
            int np = i;
            if (rn[b] >= 0) {
                const int s = rs[b];
                const int lb = int(lpre[i]) - int(lpre[s]);
                np = flag[i] ? s + lb : s + rn[b] + (i - s - lb);
            }
            ord[cur ^ 1][np] = ord[cur][i];
        }
        __syncthreads();
        cur ^= 1;
        // next level's runs, in order of their starts
        if (tid == 0) {
            const int nr = nruns_s;
            int out = nr + nsplit;   // every splitting run becomes two
            for (int b = nr - 1; b >= 0; --b) {
                if (rn[b] >= 0) {
                    out -= 2;
                    const int s = rs[b], len = rl[b], nl = rn[b];
                    rs[out + 1] = s + nl;
                    rl[out + 1] = len - nl;
                    rs[out] = s;
                    rl[out] = nl;
                } else {
                    out -= 1;
                    rs[out] = rs[b];
                    rl[out] = rl[b];
                }
            }
            nruns_s = nr + nsplit;
        }
        __syncthreads();
        for (int b = w; b < nruns_s; b += kWaves)
            for (int i = rs[b] + lane; i < rs[b] + rl[b]; i += kWave) run_of[i] = uint8_t(b);
        __syncthreads();
    }
    // the subtree's points in their final order; the values move four
    // projections at a time, as the extents read them
    int64_t of[kPer];
    bool pin[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int p = tid + q * kLocalThreads;
        pin[q] = p < m;
        of[q] = start + (pin[q] ? ord[cur][p] : 0);
        if (pin[q]) idx_out[start + p] = idx_in ? idx_in[of[q]] : int32_t(of[q]);
    }
    if (vout) {
#pragma unroll
        for (int j0 = 0; j0 < PMAX; j0 += 4) {
            float v[4][kPer];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int q = 0; q < kPer; ++q)
                    v[jj][q] = j0 + jj < P ? vin[int64_t(j0 + jj) * n + of[q]] : 0.0f;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int q = 0; q < kPer; ++q)
                    if (j0 + jj < P && pin[q])
                        vout[int64_t(j0 + jj) * n + start + tid + q * kLocalThreads] = v[jj][q];
        }
    }
}

inline unsigned nb(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// Leaves of a run of `size` points (the split rule above).
int64_t count_leaves(int64_t size, int leaf, int sub, std::map<int64_t, int64_t> &memo)
{
    if (size <= sub) return 1;
    auto it = memo.find(size);
    if (it != memo.end()) return it->second;
    const int64_t u = size > leaf ? leaf : sub;
    const int64_t T = (size + u - 1) / u, nl = ((T + 1) / 2) * u;
    const int64_t r = count_leaves(nl, leaf, sub, memo) + count_leaves(size - nl, leaf, sub, memo);
    memo[size] = r;
    return r;
}

}  // namespace

bool kd_plan(KdPlan &pl, int64_t n, int leaf, int sub)
{
    if (pl.n == n && pl.leaf == leaf && pl.sub == sub) return true;
    pl.n = n;
    pl.leaf = leaf;
    pl.sub = sub;
    pl.levels.clear();
    pl.local = KdLevel{};
    pl.has_local = false;
    std::vector<int64_t> nodes, slices;
    std::vector<std::pair<int64_t, int64_t>> cur;
    if (n > 0) cur.push_back({0, n});
    int64_t max_nodes = 0, max_slices = 0;
    std::map<int64_t, int64_t> memo;
    while (true) {
        bool any = false;
        int64_t biggest = 0, most_leaves = 0;
        for (auto &nd : cur) {
            any |= nd.second > sub;
            biggest = std::max(biggest, nd.second);
            if (nd.second <= kLocalMax)
                most_leaves = std::max(most_leaves, count_leaves(nd.second, leaf, sub, memo));
        }
        if (!any) break;
        if (biggest <= kLocalMax && most_leaves <= kLocalRuns) {
            // the rest of every subtree in one workgroup each
            pl.local.node0 = int64_t(nodes.size()) / kNodeCols;
            for (auto &nd : cur)
                nodes.insert(nodes.end(), {nd.first, nd.second, -1, 0, 0, -1, 0, 0});
            pl.local.node1 = int64_t(nodes.size()) / kNodeCols;
            pl.has_local = true;
            break;
        }
        KdLevel lv;
        lv.node0 = int64_t(nodes.size()) / kNodeCols;
        lv.slice0 = int64_t(slices.size()) / kSliceCols;
        std::vector<std::pair<int64_t, int64_t>> next;
        for (auto &nd : cur) {
            const int64_t st = nd.first, sz = nd.second;
            const int64_t node_id = int64_t(nodes.size()) / kNodeCols;
            int64_t nl = -1, child = -1;
            if (sz > sub) {
                const int64_t u = sz > leaf ? leaf : sub;
                const int64_t T = (sz + u - 1) / u;
                nl = ((T + 1) / 2) * u;
                child = int64_t(next.size());
                next.push_back({st, nl});
                next.push_back({st + nl, sz - nl});
            } else {
                next.push_back({st, sz});
            }
            const int64_t sb = int64_t(slices.size()) / kSliceCols;
            for (int64_t s = st; s < st + sz; s += kSlice) {
                slices.push_back(s);
                slices.push_back(std::min<int64_t>(kSlice, st + sz - s));
                slices.push_back(node_id);
            }
            const int64_t se = int64_t(slices.size()) / kSliceCols;
            nodes.insert(nodes.end(), {st, sz, nl, sb, se, child, 0, 0});
        }
        lv.node1 = int64_t(nodes.size()) / kNodeCols;
        lv.slice1 = int64_t(slices.size()) / kSliceCols;
        // the histogram slices of the level's nodes, after its slices
        lv.hslice0 = lv.slice1;
        for (int64_t nd = lv.node0; nd < lv.node1; ++nd) {
            const int64_t st = nodes[nd * kNodeCols + 0], sz = nodes[nd * kNodeCols + 1];
            nodes[nd * kNodeCols + 6] = int64_t(slices.size()) / kSliceCols;
            for (int64_t s = st; s < st + sz; s += kHistSlice) {
                slices.push_back(s);
                slices.push_back(std::min<int64_t>(kHistSlice, st + sz - s));
                slices.push_back(nd);
            }
            nodes[nd * kNodeCols + 7] = int64_t(slices.size()) / kSliceCols;
        }
        lv.hslice1 = int64_t(slices.size()) / kSliceCols;
        max_nodes = std::max(max_nodes, lv.node1 - lv.node0);
        max_slices = std::max(max_slices, lv.slice1 - lv.slice0);
        pl.levels.push_back(lv);
        cur.swap(next);
    }
    // the last upper level's children are not upper-level nodes: no slots
    if (!pl.levels.empty()) {
        const KdLevel &last = pl.levels.back();
        for (int64_t i = last.node0; i < last.node1; ++i) nodes[i * kNodeCols + 5] = -1;
    }
    pl.max_nodes = max_nodes;
    pl.max_slices = max_slices;
    if (!pl.node_tab.ensure(sizeof(int64_t) * std::max<size_t>(nodes.size(), 1)) ||
        !pl.slice_tab.ensure(sizeof(int64_t) * std::max<size_t>(slices.size(), 1))) {
        pl.n = -1;
        return false;
    }
    if ((!nodes.empty() && hipMemcpy(pl.node_tab.p, nodes.data(), sizeof(int64_t) * nodes.size(),
                                     hipMemcpyHostToDevice) != hipSuccess) ||
        (!slices.empty() && hipMemcpy(pl.slice_tab.p, slices.data(),
                                      sizeof(int64_t) * slices.size(),
                                      hipMemcpyHostToDevice) != hipSuccess)) {
        pl.n = -1;
        return false;
    }
    return true;
}

bool kd_reserve(KdWork &w, const KdPlan &pl, int64_t n, int P)
{
    const int64_t nn = std::max<int64_t>(n, 1);
    const int64_t ms = std::max<int64_t>(pl.max_slices, 1), mn = std::max<int64_t>(pl.max_nodes, 1);
    bool ok = true;
    ok &= w.idx[0].ensure(sizeof(int32_t) * nn);
    ok &= w.idx[1].ensure(sizeof(int32_t) * nn);
    ok &= w.val[0].ensure(sizeof(float) * P * nn);
    ok &= w.val[1].ensure(sizeof(float) * P * nn);
    ok &= w.ext[0].ensure(sizeof(uint32_t) * 2 * P * mn * kExtRep);
    ok &= w.ext[1].ensure(sizeof(uint32_t) * 2 * P * mn * kExtRep);
    ok &= w.hist.ensure(sizeof(int32_t) * 3 * kBins * mn);
    ok &= w.cnt.ensure(sizeof(int64_t) * 2 * ms);
    ok &= w.dim.ensure(sizeof(int32_t) * mn);
    ok &= w.prefix.ensure(sizeof(uint32_t) * 3 * mn);
    ok &= w.rank.ensure(sizeof(int64_t) * 3 * mn);
    return ok;
}

hipError_t kd_start(KdRun &r, const KdPlan &pl, KdWork &w, int P, const float *vals, int64_t n,
                    int32_t *perm, float *vals_sorted, hipStream_t s, bool root_given)
{
    r = KdRun{};
    r.root_given = root_given;
    r.pl = &pl;
    r.w = &w;
    r.P = P;
    r.vals = vals;
    r.n = n;
    r.perm = perm;
    r.vals_sorted = vals_sorted;
    r.s = s;
    r.vin = vals;
    r.done = n == 0;
    if (n == 0) return hipSuccess;
    const int64_t mn = std::max<int64_t>(pl.max_nodes, 1), ms = std::max<int64_t>(pl.max_slices, 1);
    if (pl.n != n || (pl.levels.empty() && !pl.has_local) || P < 1 || P > 32 ||
        w.idx[0].cap < sizeof(int32_t) * size_t(n) || w.idx[1].cap < sizeof(int32_t) * size_t(n) ||
        w.val[0].cap < sizeof(float) * P * size_t(n) ||
        w.val[1].cap < sizeof(float) * P * size_t(n) ||
        w.ext[0].cap < sizeof(uint32_t) * 2 * P * size_t(mn) * kExtRep ||
        w.ext[1].cap < sizeof(uint32_t) * 2 * P * size_t(mn) * kExtRep ||
        w.hist.cap < sizeof(int32_t) * 3 * kBins * size_t(mn) ||
        w.cnt.cap < sizeof(int64_t) * 2 * size_t(ms) || w.dim.cap < sizeof(int32_t) * size_t(mn) ||
        w.prefix.cap < sizeof(uint32_t) * 3 * size_t(mn) ||
        w.rank.cap < sizeof(int64_t) * 3 * size_t(mn)) {
        r.done = true;
        return hipErrorInvalidValue;
    }
    return hipSuccess;
}

hipError_t kd_step(KdRun &r)
{
    if (r.done) return hipSuccess;
    const KdPlan &pl = *r.pl;
    KdWork &w = *r.w;
    const int P = r.P;
    const int64_t n = r.n;
    const hipStream_t s = r.s;
    const int64_t mn = std::max<int64_t>(pl.max_nodes, 1);
    const int64_t *nodes = pl.node_tab.as<int64_t>();
    const int64_t *slices = pl.slice_tab.as<int64_t>();
    int32_t *hist = w.hist.as<int32_t>();
    int32_t *dim = w.dim.as<int32_t>();
    uint32_t *prefix = w.prefix.as<uint32_t>();
    int64_t *rank = w.rank.as<int64_t>();
    int64_t *cnt = w.cnt.as<int64_t>();
    const size_t nlev = pl.levels.size();
    const size_t phase = r.phase++;
    if (phase == 0) {   // the root's extents
        if (nlev == 0) return hipSuccess;
        k_kd_zero<<<nb(3 * kBins * mn, kThreads), kThreads, 0, s>>>(
            hist, 3 * kBins * mn, w.ext[0].as<uint32_t>(), P, mn, r.root_given ? 1 : 0);
        if (r.root_given) return hipGetLastError();
        const unsigned nr = nb(n, kThreads * kRootPer);
        if (P <= 16)
            k_kd_root_ext<16><<<nr, kThreads, 0, s>>>(n, P, r.vals, w.ext[0].as<uint32_t>(), mn);
        else
            k_kd_root_ext<32><<<nr, kThreads, 0, s>>>(n, P, r.vals, w.ext[0].as<uint32_t>(), mn);
        return hipGetLastError();
    }
    if (phase <= nlev) {   // upper level phase - 1
        const size_t li = phase - 1;
        const KdLevel &lv = pl.levels[li];
        const int64_t ns = lv.slice1 - lv.slice0;
        const int64_t *nt = nodes + lv.node0 * kNodeCols;
        const int64_t *st = slices + lv.slice0 * kSliceCols;
        uint32_t *ext = w.ext[li & 1].as<uint32_t>();
        uint32_t *ext_next = (li + 1 < nlev) ? w.ext[(li + 1) & 1].as<uint32_t>() : nullptr;
        const int64_t *hst = slices + lv.hslice0 * kSliceCols;
        const unsigned nhs = unsigned(lv.hslice1 - lv.hslice0);
        for (int rd = 0; rd < 3; ++rd)
            k_kd_hist<<<nhs, kHistThreads, 0, s>>>(nt, hst, lv.node0, lv.hslice0, mn, n, P, rd,
                                                   r.vin, ext, ext_next, dim, prefix, rank, hist);
        k_kd_count<<<unsigned(ns), kThreads, 0, s>>>(nt, st, lv.node0, lv.slice0, mn, n, r.vin,
                                                     dim, prefix, rank, hist, cnt);
        int32_t *idx_out = w.idx[r.cur].as<int32_t>();
        float *vout = w.val[r.cur].as<float>();
        if (P <= 16)
            k_kd_scatter<16><<<unsigned(ns), kThreads, 0, s>>>(
                nt, st, lv.node0, lv.slice0, n, P, r.idx_in, r.vin, dim, prefix + 2 * mn,
                rank + 2 * mn, cnt, idx_out, vout, ext_next, hist, mn);
        else
            k_kd_scatter<32><<<unsigned(ns), kThreads, 0, s>>>(
                nt, st, lv.node0, lv.slice0, n, P, r.idx_in, r.vin, dim, prefix + 2 * mn,
                rank + 2 * mn, cnt, idx_out, vout, ext_next, hist, mn);
        r.idx_in = idx_out;
        r.vin = vout;
        r.cur ^= 1;
        return hipGetLastError();
    }
    // the subtrees, or the order out as it stands
    r.done = true;
    if (pl.has_local) {
        const int64_t *nt = nodes + pl.local.node0 * kNodeCols;
        const unsigned nl = unsigned(pl.local.node1 - pl.local.node0);
        // 512 threads per subtree when every subtree's workgroup is resident
        // at once with them (three per CU), else 256 (seven per CU)
        auto go = [&](auto kern, int threads) {
            kern<<<nl, threads, 0, s>>>(nt, n, P, pl.leaf, pl.sub, r.idx_in, r.vin, r.perm,
                                        r.vals_sorted);
        };
        const bool wide = nl <= kWideLocalBlocks;
        if (P <= 16)
            wide ? go(k_kd_local<16, 512>, 512) : go(k_kd_local<16, 256>, 256);
        else
            wide ? go(k_kd_local<32, 512>, 512) : go(k_kd_local<32, 256>, 256);
        return hipGetLastError();
    }
    hipError_t e =
        hipMemcpyAsync(r.perm, r.idx_in, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && r.vals_sorted)
        e = hipMemcpyAsync(r.vals_sorted, r.vin, sizeof(float) * P * n, hipMemcpyDeviceToDevice,
                           s);
    return e;
}

hipError_t kd_order(const KdPlan &pl, KdWork &w, int P, const float *vals, int64_t n,
                    int32_t *perm, float *vals_sorted, hipStream_t s)
{
    KdRun r;
    hipError_t e = kd_start(r, pl, w, P, vals, n, perm, vals_sorted, s);
    while (e == hipSuccess && !r.done) e = kd_step(r);
    return e;
}

}  // namespace ngd
