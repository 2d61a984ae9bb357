// Internal declarations shared by the host side of libngd and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/ngd.h"

namespace ngd {

// 0.5 * log2(e): exp(-M/2) == exp2(-M * kHalfLog2e).  The precision factor
// is stored pre-scaled by sqrt(kHalfLog2e) so the kernels call exp2 directly.
constexpr double kHalfLog2e = 0.72134752044448170368;
constexpr double kSqrtHalfLog2e = 0.84932180028801904272;

// Pairs whose Gaussian value is certified below tau * 2^-kSkipLog2Margin
// are skipped inside the evaluation kernels (see ngd_eval).
constexpr double kSkipLog2Margin = 20.0;

// Work items: the forward splits each tile's candidate list into items of
// at most kItemCands candidates; the backward splits each Gaussian's tile
// list into items of at most kItemTiles tiles.  Items are independent
// workgroups / waves; their partial sums are combined in a fixed order.
constexpr int kItemCands = 512;
constexpr int kItemTiles = 32;

inline int tri(int n) { return n * (n + 1) / 2; }

// Per-Gaussian record read by the evaluation kernels, one row of `stride`
// floats: m (n) | S' = sqrt(kHalfLog2e) L^-1 packed lower by rows (tri) |
// alpha*c (3) | alpha (1) | c (3) | padding to a multiple of 4.
inline int rec_stride(int n) { return (n + tri(n) + 7 + 3) / 4 * 4; }
// 4-byte words per Gaussian of the forward's box: n lows, then n highs, as
// float16, padded to a multiple of 16 bytes
inline int box_stride(int n) { return (2 * n + 7) / 8 * 4; }

// Device allocation through the configurable allocator; reports the
// matching release function (NULL: hipFree) and its context.
void *dev_alloc(size_t bytes, void (**free_fn)(void *, void *), void **ctx);

// A grow-only device buffer, released with the allocator that made it.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    void (*free_fn)(void *, void *) = nullptr;
    void *ctx = nullptr;
    // Returns false on allocation failure (old contents are not kept).
    bool ensure(size_t bytes);
    void release();
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// k-d ordering (kd.hip): per-level node and slice tables of the upper
// levels, and the nodes whose subtrees finish in one workgroup each; laid
// out on the host from (n, leaf, sub) alone and kept while they stay the same.
struct KdLevel {
    int64_t node0 = 0, node1 = 0, slice0 = 0, slice1 = 0, hslice0 = 0, hslice1 = 0;
};
struct KdPlan {
    int64_t n = -1;
    int leaf = 0, sub = 0;
    std::vector<KdLevel> levels;   // upper levels
    bool has_local = false;
    KdLevel local;                 // node rows of the subtree workgroups
    int64_t max_nodes = 0, max_slices = 0;
    DevBuf node_tab;    // rows: start, size, n_left (-1 leaf), slice begin / end, child,
                        // histogram slice begin / end
    DevBuf slice_tab;   // rows: start, length, node
};
struct KdWork {
    DevBuf idx[2], val[2], ext[2];
    DevBuf hist, cnt, dim, prefix, rank;
};
bool kd_plan(KdPlan &pl, int64_t n, int leaf, int sub);
bool kd_reserve(KdWork &w, const KdPlan &pl, int64_t n, int P);
// Orders n points with P <= 32 projections (vals: P x n, point order) and
// writes the order (position -> point) to perm and, when vals_sorted is not
// null, the projections in that order (P x n).  Needs a plan with at least
// one split (n > sub).
hipError_t kd_order(const KdPlan &pl, KdWork &w, int P, const float *vals, int64_t n,
                    int32_t *perm, float *vals_sorted, hipStream_t s);
// The same, enqueued phase by phase (the root, each upper level, the
// subtrees), so that two orders on two streams can be enqueued alternately:
// kd_start checks the buffers, each kd_step enqueues one phase until done.
struct KdRun {
    const KdPlan *pl = nullptr;
    KdWork *w = nullptr;
    int P = 0;
    const float *vals = nullptr;
    int64_t n = 0;
    int32_t *perm = nullptr;
    float *vals_sorted = nullptr;
    hipStream_t s = nullptr;
    size_t phase = 0;
    const int32_t *idx_in = nullptr;   // null: the identity order
    const float *vin = nullptr;
    int cur = 0;
    bool done = true;
    // the root's min / max keys are already in plane 0 of w.ext[0] (slots
    // 2j and 2j + 1 of projection j), written by the caller ahead of the run
    bool root_given = false;
};
hipError_t kd_start(KdRun &r, const KdPlan &pl, KdWork &w, int P, const float *vals, int64_t n,
                    int32_t *perm, float *vals_sorted, hipStream_t s, bool root_given = false);
hipError_t kd_step(KdRun &r);

}  // namespace ngd

struct ngd_mixture {
    int n = 0;
    int64_t k = 0;
    int64_t version = 0;
    int device = 0;
    ngd::DevBuf rec;     // k x rec_stride(n) float
    ngd::DevBuf lfac;    // k x tri(n) float: copy of L for the cull
    ngd::DevBuf flag;    // int: bit 1 a bad factor or parameter, bit 2 a bad parent index
    // parent-child composition (ngd_mixture_update_composed): kp parents,
    // then k - kp children; kp < 0 when the last update was a plain one
    int64_t kp = -1;
    ngd::DevBuf comp_parent, comp_u, comp_mu;   // copies: kc int32, kc x tri, kc x n
    ngd::DevBuf abs_mean, abs_factor;           // k x n, k x tri: absolute parameters
    ngd::DevBuf g_abs;                          // k x (n + tri): backward scratch
    ngd::DevBuf contrib;                        // kc x (n + tri): children's shares
};

struct ngd_cull {
    // identity of what it was built for
    const ngd_mixture *mix = nullptr;
    int64_t mix_version = -1;
    const float *queries = nullptr;
    int64_t q = 0;
    int n = 0;
    int64_t k = 0;
    ngd_cull_params params{};
    float kappa2 = 0.f;
    int64_t ntiles = 0;
    int64_t total = 0;
    int64_t max_per_tile = 0;
    int64_t nitems = 0;        // forward work items
    int64_t gitems_cap = 0;    // upper bound of backward work items
    int64_t nchunks = 0;       // ceil(k / 64)
    int64_t tpad = 0;          // ntiles rounded up to 64
    int nseg = 0;              // chunk segments used by the list build
    // device buffers
    ngd::DevBuf proj;          // n_proj x n float
    ngd::DevBuf qr;            // n_proj x q float (caller order)
    ngd::DevBuf range_part;    // per-block min/max partials
    ngd::DevBuf qrange;        // n_proj lo | n_proj hi | n_proj scale (float)
    ngd::DevBuf g_mr, g_thr;   // n_proj x k float (caller order)
    ngd::DevBuf keys0, keys1, vals0, vals1;   // radix sort ping-pong
    ngd::DevBuf radix_hist;    // 256 x nblocks int32
    ngd::DevBuf radix_off;     // 256 x nblocks + 1 int64
    ngd::DevBuf perm;          // q int32
    ngd::DevBuf gperm;         // k int32
    ngd::DevBuf qs;            // n x q float: sorted queries, by dimension
    ngd::DevBuf gs;            // 3 x q float: sorted upstream gradient
    ngd::DevBuf tile_lo, tile_hi;   // ntiles x n_proj float
    // per tile / super-tile box: pad_proj(n_proj) lows, then as many highs
    // (padding -inf / +inf)
    ngd::DevBuf tbnd;               // ntiles x 2 pad_proj(n_proj) float
    ngd::DevBuf sbnd;               // ceil(ntiles / kSuperTiles) x 2 pad_proj(n_proj) float
    ngd::DevBuf qr_s;               // n_proj x q float, tile order (k-d tiling)
    ngd::DevBuf grec;          // k x rec_stride float, sorted Gaussians
    ngd::DevBuf g_mr_s;             // n_proj x k float, sorted Gaussians
    ngd::DevBuf g_ub, g_lb;         // n_proj x k float, sorted: the interval test's limits
    ngd::DevBuf gbox_u, gbox;       // k x box_stride(n) words, caller's order and
                                    // sorted: per coordinate, the range outside which
                                    // the forward keeps no query
    ngd::DevBuf masks;         // nchunks x tpad uint64
    ngd::DevBuf seg_cnt;       // nseg x ntiles int32 (counts, then prefixes)
    ngd::DevBuf tile_cnt;      // ntiles int32
    ngd::DevBuf tile_off;      // ntiles + 1 int64
    ngd::DevBuf cand;          // total int32
    ngd::DevBuf g_cnt;         // k int32
    ngd::DevBuf g_off;         // k + 1 int64
    ngd::DevBuf g_tiles;       // total int32: tile of each transposed entry
    ngd::DevBuf g_ent;         // total int32: candidate entry of each transposed entry
    ngd::DevBuf ent_tile;      // total int32: tile of each candidate entry
    ngd::DevBuf act;           // total x groups uint8: forward kept (entry, group)
    mutable int64_t act_version = -1;  // mixture version the flags belong to
    bool transposed = false;   // g_off / g_tiles hold the full transposed lists
    // backward: the entries with a kept group, grouped by Gaussian
    ngd::DevBuf eflag;         // ceil(total / 256) int32: kept entries per block
    ngd::DevBuf eoff;          // ceil(total / 256) + 1 int64: their offsets
    ngd::DevBuf a_cnt;         // k int32
    ngd::DevBuf a_off;         // k + 1 int64
    int a_ent_buf = 0;         // which sort buffer (vals0 / vals1) holds them
    ngd::DevBuf item_cnt;      // ntiles int32: forward items per tile
    ngd::DevBuf item_off;      // ntiles + 1 int64
    ngd::DevBuf item_tile;     // nitems int32
    ngd::DevBuf fpart;         // nitems x 3 x tile float: forward partial sums
    ngd::DevBuf gitem_cnt;     // k int32: backward items per Gaussian
    ngd::DevBuf gitem_off;     // k + 1 int64
    ngd::DevBuf gitem_g;       // gitems_cap int32: sorted Gaussian of each item
    ngd::DevBuf gpart;         // gitems_cap x (n + tri + 3) float: moments
    ngd::DevBuf gflag;         // gitems_cap int32: item had contributing pairs
    ngd::DevBuf scan_tmp;      // scan block sums
    ngd::DevBuf stats;         // 4 int64: -, max per tile, total, items
    int64_t *stats_host = nullptr;  // pinned: max per tile, total, items
    ngd::KdPlan kd_q, kd_g;    // k-d tiling plans of the queries and the Gaussians
    ngd::KdWork kd_work;       // query k-d work
    ngd::KdWork kd_work_g;     // Gaussian k-d work (runs concurrently, on `side`)
    hipStream_t side = nullptr;          // default-priority, non-blocking
    // fork; the interval test's join (the Gaussians' limits); the end of the
    // second stream's work (the forward's per-Gaussian data)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_done = nullptr;
    hipEvent_t ev_sizes = nullptr;   // the list sizes have reached the host
    // matrix-core forward: quadratic coefficients of the ordered Gaussians
    ngd::DevBuf mrec;          // k x mfma_rec_bytes(n): bf16 hi / lo pairs
    ngd::DevBuf mrow;          // k float: bound factor R'
    ngd::DevBuf tcen;          // ntiles x n float: centre of each tile's query box
    ngd::DevBuf eb0;           // total x 64 B: centred constant / linear terms, bf16
    ngd::DevBuf ebnd;          // total x 4 float: bound terms of each entry
    int64_t build_seq = 0;     // builds of this handle
    int64_t mrec_seq = -1;     // build the per-entry records belong to
    int64_t coef_seq = -1;     // build the per-Gaussian coefficients (mrec, mrow) belong to
    bool coef_next = false;    // the build in progress has launched them
};

namespace ngd {

// ---- launchers (each returns the hipError_t of its launches) ----------
// clear_flag: the mixture's flag is cleared first (false: a composition
// kernel ahead of it has already cleared it and may have set bit 2).
hipError_t launch_prepare(int n, int64_t k, const float *mean, const float *factor,
                          const float *weight, const float *colour, float *rec,
                          float *lfac, int *flag, hipStream_t s, bool clear_flag = true);
hipError_t launch_clear_flag(int *flag, hipStream_t s);
// compose.hip: absolute parameters of parents and children (Eq. 6-7), and
// the chain rule of the composition in the backward.
hipError_t launch_compose(int n, int64_t k, int64_t kp, const float *mean, const float *factor,
                          const int32_t *parent, const float *rel_factor, const float *rel_mean,
                          float *abs_mean, float *abs_factor, int *flag, hipStream_t s);
// condition.hip: every Gaussian conditioned on x_c (host, n - p values) of
// its trailing dimensions; p-dimensional outputs.
hipError_t launch_condition(const ngd_mixture *mix, int p, const float *xc, float *mean_out,
                            float *factor_out, float *weight_out, float *colour_out,
                            hipStream_t s);
hipError_t launch_compose_backward(int n, int64_t kp, int64_t kc, const int32_t *parent,
                                   const float *factor_p, const float *rel_factor,
                                   const float *rel_mean, const float *g_abs_mean,
                                   const float *g_abs_factor, float *g_mean, float *g_factor,
                                   float *g_rel_factor, float *g_rel_mean, float *contrib,
                                   hipStream_t s);

hipError_t launch_cull_build_front(ngd_cull *c, const ngd_mixture *mix,
                                   const float *queries, hipStream_t s);
// stats[1..3] = longest list, total, items (device) for one copy to the host.
hipError_t launch_gather_sizes(ngd_cull *c, hipStream_t s);
// The lists of a built front: entries below cap_ent and items below
// cap_items are written (the buffers' capacities, or the exact sizes).
hipError_t launch_cull_build_lists(ngd_cull *c, hipStream_t s, int64_t cap_ent,
                                   int64_t cap_items);
// Gaussian -> tile lists of all candidates (g_off, g_tiles); built on
// demand for ngd_cull_export.
hipError_t launch_cull_transpose_full(ngd_cull *c, hipStream_t s);

hipError_t launch_eval_dense(const ngd_mixture *mix, const float *queries, int64_t q,
                             float *out, hipStream_t s);
// Counting run of the culled forward (flags written, no colours): adds
// (pairs examined, passed check 1, passed check 2, kept) to stats[0..3].
hipError_t launch_eval_stats(const ngd_mixture *mix, const ngd_cull *c,
                             unsigned long long *stats, hipStream_t s);
// Culled forward; with out == nullptr only the keep/skip flags are written.
hipError_t launch_eval_reduce(const ngd_cull *c, float *out, hipStream_t s);
// Culled forward with the BF16 MFMA filter (eval_mfma.hip).  out: colours;
// out == nullptr: keep/skip flags only; stats != nullptr: counting mode,
// stats[0..4] = (group-candidate pairs examined, not skipped by the matrix
// filter, passed check 1, passed check 2, kept).  Builds the coefficient
// records (c->mrec, c->mrow, reserved by the caller) once per cull build.
// The matrix-core coefficient records of the current cull build (once per
// build; launch_eval_mfma builds them itself when they are missing).
hipError_t launch_mfma_prepare(const ngd_mixture *mix, ngd_cull *c, hipStream_t s);
hipError_t launch_eval_mfma(const ngd_mixture *mix, ngd_cull *c, float *out,
                            unsigned long long *stats, hipStream_t s);
size_t mfma_rec_bytes(int n);
// The per-Gaussian coefficients of the matrix-core forward (c->mrec, c->mrow)
// from the cull's ordered records c->grec, on stream s.
hipError_t launch_mfma_coef(int n, ngd_cull *c, hipStream_t s);
size_t mfma_entry_bytes();
hipError_t launch_eval_culled(const ngd_mixture *mix, const ngd_cull *c, float *out,
                              hipStream_t s);
hipError_t launch_backward_dense(const ngd_mixture *mix, const float *queries, int64_t q,
                                 const float *grad_out, float *g_mean, float *g_factor,
                                 float *g_weight, float *g_colour, hipStream_t s);
hipError_t launch_backward_culled(const ngd_mixture *mix, ngd_cull *c,
                                  const float *grad_out, float *g_mean, float *g_factor,
                                  float *g_weight, float *g_colour, hipStream_t s);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);
// Groups the entries with a kept query group by Gaussian (a_cnt, a_off, the
// sorted entries in vals0/vals1) and builds the backward work items.
hipError_t launch_backward_prepare(ngd_cull *c, hipStream_t s);
// Mean squared error over q x 3 and its gradient; rel_eps > 0: each error
// weighted by 1 / (|f| + rel_eps)^2, the weight held constant.
hipError_t launch_l2_loss(const float *f, const float *target, int64_t q, float *loss,
                          float *grad, float *partials, int nparts, hipStream_t s,
                          float rel_eps = 0.0f);

// Stable LSD radix sort of (key, value) pairs by the low nbits of the keys,
// kRadixPerBlock keys per block.  n is the count, or an upper bound when
// n_dev (a device count) is given.  Buffers: keys/vals ping-pong of n,
// hist kRadixMaxBins x blocks int32, off kRadixMaxBins x blocks + 1 int64,
// scan_tmp for a scan of kRadixMaxBins x blocks.  *which tells which
// ping-pong buffer holds the result.
constexpr int kRadixPerBlock = 4096;
constexpr int kRadixMaxBins = 1024;   // digits of up to 10 bits
// Tiles per super-tile of the interval test (a k-d node of 16 tiles): a
// chunk of Gaussians outside a super-tile's bounds is outside each of its
// tiles' bounds.
constexpr int kSuperTiles = 16;
// Projections per box in the interval test: n_proj rounded up to 4 (to 8
// above 16).
inline int pad_proj(int p) { return p <= 16 ? (p + 3) & ~3 : (p + 7) & ~7; }
// Every buffer's capacity is checked on the host first (hipErrorInvalidValue
// when one is too small).
hipError_t radix_sort(int64_t n, const int64_t *n_dev, int nbits, DevBuf &k0, DevBuf &k1,
                      DevBuf &v0, DevBuf &v1, DevBuf &hist, DevBuf &off, DevBuf &scan_tmp,
                      hipStream_t s, int *which);

// Exclusive scan of `n` int32 counts into n + 1 int64 offsets (out[n] is
// the total).  `tmp` must hold scan_tmp_bytes(n) bytes.
// The capacities of in (n int32), out (n + 1 int64) and tmp are checked on
// the host first (hipErrorInvalidValue when one is too small).
size_t scan_tmp_bytes(int64_t n);
hipError_t scan_counts(const DevBuf &in, DevBuf &out, int64_t n, DevBuf &tmp, hipStream_t s);

// Sizes the cull's buffers need before the lists are built, and after the
// number of candidates is known.
bool cull_reserve_front(ngd_cull *c);
bool cull_reserve_lists(ngd_cull *c);

}  // namespace ngd
