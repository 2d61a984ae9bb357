/*
 * libngd -- evaluation and differentiation of N-dimensional Gaussian
 * mixtures with random-projection tile culling, on AMD Instinct MI355X
 * (gfx950).
 *
 * The method is that of Diolatzis et al., "N-Dimensional Gaussians for
 * Fitting of High Dimensional Functions" (SIGGRAPH 2024):
 *   Sec. 3.1, Eq. 1   G(x - m) = exp(-1/2 (x-m)^T V^-1 (x-m))   (unnormalised)
 *   Sec. 3.1, Eq. 2   V = L L^T, L lower triangular, optimised directly
 *   Sec. 4.1, Eq. 8   f(x) = sum_i G_i(x - m_i) alpha_i c_i     (RGB)
 *   Sec. 3.2, Eq. 3-5 cull Gaussian i for a tile of queries when, on some
 *                     random unit vector r, the tile's projected extent lies
 *                     outside [m_r - kappa sigma_r, m_r + kappa sigma_r],
 *                     sigma_r^2 = r^T V r
 *   Sec. 4.1          gradients of all parameters computed analytically
 *
 * Conventions for every call:
 *   - Returns NGD_OK (0) or a negative NGD_E_* code; ngd_last_error() gives a
 *     message for the calling thread.  No C++ exception crosses this ABI.
 *   - Array arguments named "device" are device pointers (hipMalloc'ed or
 *     from a framework allocator); "host" arguments are host pointers.  All
 *     device arrays are float32 (or the integer type shown), C-contiguous,
 *     4-byte aligned, and owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).  All
 *     device work is enqueued on it; the caller keeps its buffers alive until
 *     that work has finished.  Calls documented as "synchronises" wait for
 *     the stream before returning.
 *   - Outputs are overwritten, never accumulated into.
 *   - Handles are not thread-safe; one handle, one thread at a time.
 *   - Arguments are validated on the host before any device work; an invalid
 *     call changes nothing.
 */
#ifndef NGD_H
#define NGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NGD_OK 0
#define NGD_E_INVAL (-1)    /* NULL pointer, size out of range, bad parameter */
#define NGD_E_SINGULAR (-2) /* a factor has a zero or non-finite diagonal entry,
                               or a parameter is not finite (ngd_mixture_validate) */
#define NGD_E_HIP (-3)      /* HIP runtime error; message holds HIP's string */
#define NGD_E_NOMEM (-4)    /* device or host allocation failed */
#define NGD_E_STALE (-5)    /* cull built for another mixture version, another
                               query buffer or another query count */

#define NGD_MAX_N 12        /* dimensions supported: 1 .. NGD_MAX_N */
#define NGD_MAX_PROJ 32     /* projection vectors: 1 .. NGD_MAX_PROJ */

/* Arithmetic of ngd_eval / ngd_eval_backward (culled only for BF16_MFMA). */
#define NGD_FP32 0          /* float32 direct evaluation, staged certified skip */
#define NGD_BF16_MFMA 1     /* the (query group, candidate) skip decided by a
                               BF16 matrix-core contraction of quadratic query
                               features (1, x', x'_i x'_j; x' centred on the
                               work item's query box) against per-Gaussian
                               quadratic coefficients, each split into bf16
                               hi + lo with the products hi*hi + hi*lo + lo*hi
                               accumulated in float32 (Sec. 3.1, Eq. 1-2
                               expanded).  A candidate is skipped for a group
                               only when the contraction minus a certified
                               error bound puts every query of the group past
                               the skip threshold; every other candidate is
                               evaluated exactly as with NGD_FP32, so colours
                               keep float32 accuracy. */

typedef struct ngd_mixture ngd_mixture;
typedef struct ngd_cull ngd_cull;

/* Parameters of the tile cull (Sec. 3.2). */
typedef struct {
    int n_proj;     /* number of random projection vectors, 1..NGD_MAX_PROJ (16) */
    float tau;      /* value threshold in (0, 1): a culled (tile, Gaussian) pair
                       has G <= tau at every query of the tile.  The interval
                       half-width is kappa sigma_r with kappa^2 = 2 ln(1/tau)
                       (tau = exp(-4.5) gives the paper's 3 sigma). (1e-4) */
    int tile;       /* queries per tile: 256 (the paper's 16 x 16 pixel tile) */
    int key_proj;   /* tiling 1: projections in the locality key, 0..n_proj (16) */
    int key_bits;   /* tiling 1: bits per key projection; key_proj*key_bits <= 32 (2) */
    int tiling;     /* how tiles are formed from queries without an image (0):
                       0  k-d: recursive exact-rank splits of the queries on the
                          projection of largest extent, down to runs of `tile`;
                          Gaussians ordered the same way in runs of 64
                       1  Morton: stable sort on key_proj projections quantised
                          to key_bits each, bits interleaved
                       2  given order: tile t is queries [t*tile, (t+1)*tile)
                          as the caller laid them out -- for queries of an
                          image arranged tile by tile (the paper's 16 x 16
                          pixel tiles, Sec. 3.2); Gaussians as with 0 */
} ngd_cull_params;

/* Message for the last failing call on this thread ("" if none). */
const char *ngd_last_error(void);

/* Library version: major*10000 + minor*100 + patch. */
int ngd_version(void);

/* Default cull parameters (values in parentheses above).  `p` host. */
int ngd_cull_params_default(ngd_cull_params *p);

/* Replaces the device allocator used for library-owned workspaces (default
 * hipMalloc / hipFree).  alloc(bytes, ctx) returns a device pointer aligned
 * to 256 bytes (as hipMalloc's are), or NULL; free(ptr, ctx) releases it.  A
 * pointer that is not so aligned is released at once and the call that
 * needed it fails with NGD_E_NOMEM.  Both NULL restores the default.
 * Affects allocations made after the call; memory is always released with
 * the allocator that made it. */
int ngd_set_allocator(void *(*alloc_fn)(size_t bytes, void *ctx),
                      void (*free_fn)(void *ptr, void *ctx), void *ctx);

/* ---- mixture --------------------------------------------------------- */

/* Creates a mixture of k Gaussians in n dimensions (1 <= n <= NGD_MAX_N,
 * 0 <= k < 2^31) and allocates its derived-data workspace on the current
 * device.  *out receives the handle. */
int ngd_mixture_create(int n, int64_t k, ngd_mixture **out);

/* Loads parameters (Sec. 3.1, Eq. 2; Sec. 4.1) and derives, in float64 on
 * the device, S = L^-1 for every Gaussian (the precision factor,
 * V^-1 = S^T S) plus the per-Gaussian records the kernels read.  Inputs are
 * activated values:
 *   mean   device, k x n
 *   factor device, k x n(n+1)/2: L packed lower triangle by rows,
 *          element (i, j), j <= i, at i(i+1)/2 + j; any nonzero diagonal
 *   weight device, k       (alpha: brightness, or opacity)
 *   colour device, k x 3   (c: RGB)
 * Copies what it needs; the inputs may be freed once the stream reaches
 * this point.  Bumps the mixture version (culls built before go stale).
 * A zero or non-finite diagonal entry sets a device flag that
 * ngd_mixture_validate reports; this call itself does not synchronise. */
int ngd_mixture_update(ngd_mixture *mix, const float *mean, const float *factor,
                       const float *weight, const float *colour, void *stream);

/* Synchronises; NGD_E_SINGULAR if the last update saw a zero or non-finite
 * factor diagonal or a non-finite parameter; NGD_E_INVAL if the last
 * composed update saw a parent index outside [0, kp) or out of order. */
int ngd_mixture_validate(const ngd_mixture *mix, void *stream);

/* Parent-child composition of the refinement (Sec. 3.3, Eq. 6-7) done by the
 * library: Gaussians 0 .. kp-1 are parents, given absolutely; Gaussians
 * kp + j (j < kc = k - kp) are children, each given in its parent's frame by
 * a lower-triangular factor U_j and an offset m_u,j:
 *   L = L_parent[j] U_j,   m = L_parent[j] m_u,j + m_parent[j].
 *   mean       device kp x n        (parents)
 *   factor     device kp x n(n+1)/2 (parents, packed like ngd_mixture_update)
 *   weight     device k             (parents, then children)
 *   colour     device k x 3         (parents, then children)
 *   parent     device kc int32, non-decreasing, each in [0, kp)
 *   rel_factor device kc x n(n+1)/2 (U, packed the same way)
 *   rel_mean   device kc x n        (m_u)
 * The children's factor and mean are formed in float64 (exact products of
 * the float32 inputs, sums in ascending order) and rounded to float32; from
 * there every Gaussian is prepared as by ngd_mixture_update and the cull and
 * evaluation see no difference between parents and children.  The relative
 * parameters are copied (the backward uses the copies).  A parent index
 * outside [0, kp) or smaller than its predecessor's is reported by
 * ngd_mixture_validate (NGD_E_INVAL); that child is then a unit Gaussian
 * at the origin (finite, so nothing downstream faults).  kp outside [0, k], kc > 0 with kp = 0, NULL or misaligned arrays:
 * NGD_E_INVAL before any device work.  Bumps the version.  Does not
 * synchronise. */
int ngd_mixture_update_composed(ngd_mixture *mix, int64_t kp, const float *mean,
                                const float *factor, const float *weight, const float *colour,
                                const int32_t *parent, const float *rel_factor,
                                const float *rel_mean, void *stream);

/* Number of dimensions / Gaussians / current version. */
int ngd_mixture_info(const ngd_mixture *mix, int *n, int64_t *k, int64_t *version);

/* Frees the handle (NULL is a no-op).  Synchronises the device. */
int ngd_mixture_destroy(ngd_mixture *mix);

/* ---- cull ------------------------------------------------------------ */

/* Builds (or, when *inout is non-NULL, rebuilds in place, reusing its
 * memory) the cull structure for `queries` against the mixture's current
 * version (Sec. 3.2, Eq. 3-5):
 *   queries device, q x n (the buffer later passed to ngd_eval)
 *   proj    host, p->n_proj x n: the random projection vectors r_j (any
 *           length; Eq. 5 does not depend on it).  Copied.
 * Steps on the device: query and mean projections (Eq. 3), projected
 * variances in float64 (Eq. 4), a locality order of queries and Gaussians
 * (p->tiling), tiles of p->tile consecutive ordered queries with
 * their projected bounds, the (tile, Gaussian) interval test (Eq. 5), the
 * per-tile candidate lists (CSR, ascending) and their transpose.
 * Synchronises once, to read the number of candidates (the list kernels
 * are already enqueued then; they complete in stream order).  q = 0 or
 * k = 0 gives an empty structure. */
int ngd_cull_build(const ngd_mixture *mix, const float *queries, int64_t q,
                   const ngd_cull_params *p, const float *proj, void *stream,
                   ngd_cull **inout);

/* Sizes of a built cull (host outputs, any may be NULL): total candidates,
 * the longest tile list, and the number of tiles. */
int ngd_cull_stats(const ngd_cull *cull, int64_t *total, int64_t *max_per_tile,
                   int64_t *ntiles);

/* Copies the cull to host arrays (any may be NULL; synchronises):
 *   perm     q        sorted query position -> caller's query index
 *   gperm    k        sorted Gaussian position -> caller's Gaussian index
 *   tile_off ntiles+1 offsets into cand (int64)
 *   cand     total    candidates per tile, as sorted Gaussian positions,
 *                     ascending within a tile
 *   g_off    k+1      offsets into g_tiles, by sorted Gaussian position
 *   g_tiles  total    tiles of each sorted Gaussian, ascending
 *   tile_lo, tile_hi  ntiles x n_proj projected bounds of each tile */
int ngd_cull_export(const ngd_cull *cull, int32_t *perm, int32_t *gperm,
                    int64_t *tile_off, int32_t *cand, int64_t *g_off, int32_t *g_tiles,
                    float *tile_lo, float *tile_hi);

/* Frees the handle (NULL is a no-op).  Synchronises the device. */
int ngd_cull_destroy(ngd_cull *cull);

/* ---- evaluation -------------------------------------------------------- */

/* Mixture colour f(x) = sum_i G_i(x - m_i) alpha_i c_i (Sec. 4.1, Eq. 8).
 *   cull     NULL: dense direct sum over all Gaussians, no culling.
 *            Otherwise a cull built for this mixture version, this
 *            `queries` pointer and this q (NGD_E_STALE if not): the sum over
 *            each tile's candidates, where pairs whose Gaussian value is
 *            certified below tau * 2^-20 are skipped without evaluation.
 *   queries  device, q x n
 *   out      device, q x 3, in the caller's query order
 *   precision NGD_FP32, or NGD_BF16_MFMA (needs a cull; its first use on a
 *            cull build derives the per-Gaussian coefficients, k x 260 bytes
 *            at n = 10, in library memory)
 * Does not synchronise. */
int ngd_eval(const ngd_mixture *mix, const ngd_cull *cull, const float *queries,
             int64_t q, int precision, float *out, void *stream);

/* Builds, ahead of ngd_eval, what a forward of `precision` derives once per
 * cull build: for NGD_BF16_MFMA the per-entry centred terms of the
 * matrix-core forward of Eq. 1-2 expanded (and the per-Gaussian quadratic
 * coefficients, which ngd_cull_build itself launches beside its own work when
 * it orders the Gaussians on its second stream; the tiles' centres come with
 * the cull's tile bounds); nothing for NGD_FP32.  ngd_eval builds them itself
 * when they are missing, so this call only moves that work out of the first
 * forward (for instance to time the forward kernel alone).
 *   mix, cull, queries, q as for ngd_eval (a cull is required).
 * Returns NGD_E_INVAL for a NULL handle or an unknown precision,
 * NGD_E_STALE for a cull of another mixture version or queries.
 * Does not synchronise. */
int ngd_eval_prepare(const ngd_mixture *mix, const ngd_cull *cull, const float *queries,
                     int64_t q, int precision, void *stream);

/* Work counters of the culled forward, for measurement (synchronises).
 * Runs the forward kernel of `precision` on the same cull in a counting mode
 * (no colours written) and returns in counts (host, 5 x int64): the
 * (64-query group, candidate) pairs examined, those not skipped by the
 * first filter (the matrix-core one with NGD_BF16_MFMA; with NGD_FP32 the
 * test of the group's bounding box against each Gaussian's per-coordinate
 * box of half-widths sqrt(2 ln2 skip V_ii), skip the forward's threshold),
 * those that then passed the first and the second Mahalanobis-bound check
 * (marginals over the first 3 and 6 coordinates), and those kept (evaluated
 * with exp and accumulated).
 * `cull` and `queries`/q as for ngd_eval. */
int ngd_eval_stats(const ngd_mixture *mix, const ngd_cull *cull, const float *queries,
                   int64_t q, int precision, int64_t *counts, void *stream);

/* Gradients of a loss l given grad_out = dl/df (device, q x 3), with respect
 * to every Gaussian's mean, factor, weight and colour (the analytic
 * gradients of Sec. 4.1; no query gradient):
 *   dl/dalpha_i = sum_x G_i s,  dl/dc_i = alpha_i sum_x G_i g,
 *   dl/dm_i = sum_x w z,        dl/dL_i = tril(sum_x w z y^T),
 * with g = grad_out(x), s = g . c_i, w = alpha_i G_i s, y = L_i^-1 (x - m_i),
 * z = L_i^-T y.  With a cull the sums run over the same pairs as ngd_eval's.
 * Outputs (device, overwritten, caller's Gaussian order): g_mean k x n,
 * g_factor k x n(n+1)/2 (packed like the factor), g_weight k, g_colour k x 3.
 * Each Gaussian's sums are formed by one wave in a fixed order: no atomics,
 * bitwise reproducible.  `cull` may be NULL (dense).  With a cull the sums
 * run over the pairs the last ngd_eval on this cull and mixture version kept,
 * whatever its precision; without one, the keep decisions are taken first
 * with `precision`.  The gradient arithmetic is float32 in both cases.  Does
 * not synchronise. */
int ngd_eval_backward(const ngd_mixture *mix, const ngd_cull *cull,
                      const float *queries, int64_t q, const float *grad_out,
                      int precision, float *g_mean, float *g_factor, float *g_weight,
                      float *g_colour, void *stream);

/* Conditions every Gaussian on fixed values of its trailing dimensions (the
 * paper's global conditioning, Sec. 3.2: with every input but the position
 * constant over an image, the N-D Gaussians are conditioned on them and
 * then culled and evaluated as p-D ones).  With V = L L^T split into the
 * kept dimensions 0..p-1 and the fixed ones p..n-1 (textbook Schur
 * complement):
 *   mean'   = m_p + V_pc V_cc^-1 (x_c - m_c)
 *   factor' = Cholesky factor (positive diagonal) of V_pp - V_pc V_cc^-1 V_cp
 *   weight' = alpha exp(-(x_c - m_c)^T V_cc^-1 (x_c - m_c) / 2),  colour' = c
 * so that the p-D mixture of these parameters takes, at every x_p, the value
 * of the N-D mixture at (x_p, x_c).  Float64 arithmetic, one thread per
 * Gaussian, from the parameters of the last update.
 *   p          kept dimensions, 1 .. n-1
 *   xc         HOST, n - p finite values of dimensions p .. n-1 (copied)
 *   outputs    device: mean_out k x p, factor_out k x p(p+1)/2 (packed like
 *              ngd_mixture_update), weight_out k, colour_out k x 3 --
 *              the arguments of ngd_mixture_update for a p-D mixture.
 * A conditional covariance that is not positive in float64 gets a zero
 * diagonal, which that update reports through ngd_mixture_validate.
 * Invalid p, NULL / non-finite xc, NULL or misaligned outputs: NGD_E_INVAL;
 * no update yet: NGD_E_STALE.  Does not synchronise. */
int ngd_mixture_condition(const ngd_mixture *mix, int p, const float *xc, float *mean_out,
                          float *factor_out, float *weight_out, float *colour_out, void *stream);

/* ngd_eval_backward for a mixture whose last update was
 * ngd_mixture_update_composed (else NGD_E_INVAL), with the gradients carried
 * through the composition (Sec. 3.3, Eq. 6-7) by the chain rule of the
 * product, for every child j of parent p:
 *   dU_j = tril(L_p^T dL_c),   dm_u,j = L_p^T dm_c,
 *   dL_p += tril(dL_c U_j^T + dm_c m_u,j^T),   dm_p += dm_c,
 * where dL_c, dm_c are the gradients with respect to the child's absolute
 * factor and mean.  Outputs (device, overwritten): g_mean kp x n and
 * g_factor kp x n(n+1)/2 (the parents' own terms plus their children's, the
 * children summed in index order), g_weight k and g_colour k x 3 (every
 * Gaussian), g_rel_factor kc x n(n+1)/2 and g_rel_mean kc x n.  Float64
 * chain arithmetic, no atomics: bitwise reproducible.  Other arguments and
 * errors as ngd_eval_backward.  Does not synchronise. */
int ngd_eval_backward_composed(const ngd_mixture *mix, const ngd_cull *cull,
                               const float *queries, int64_t q, const float *grad_out,
                               int precision, float *g_mean, float *g_factor, float *g_weight,
                               float *g_colour, float *g_rel_factor, float *g_rel_mean,
                               void *stream);

/* Mean squared error and its gradient, the loss of the 10-D fitting
 * workload (Sec. 4.1 fits colours with an L2-type loss):
 *   loss = 1/(3q) sum (f - target)^2,  grad = 2 (f - target) / (3q)
 * f, target, grad device q x 3; loss device, one float.  Deterministic
 * two-level reduction.  Does not synchronise. */
int ngd_l2_loss(const float *f, const float *target, int64_t q, float *loss,
                float *grad, void *stream);

/* Largest q the allocation-free loss accepts (its scratch does not grow
 * with q: 1024 float64 partial sums, 8 KiB per device). */
#define NGD_NOALLOC_MAX_Q 2147483647LL

/* ngd_l2_loss without any allocation, for callers that cannot allocate
 * device memory while they run: code under HIP graph capture, tight serving
 * or training loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels, partition and result (bit for bit) as ngd_l2_loss.  Its partial
 * sums live in a static device array of 8 KiB, one per GPU, held until the
 * process ends; its device address is looked up once per device on the
 * first call with that device current (hipGetSymbolAddress).  Every call on
 * one GPU shares that array: calls that overlap on one GPU (two streams, two
 * threads) race and may return wrong sums.  Each partial is written before
 * it is read, so nothing is cleared between calls.  q outside
 * [0, NGD_NOALLOC_MAX_Q] or NULL / misaligned arrays: NGD_E_INVAL before any
 * device work.  No hipMalloc, hipFree or allocating library call.  Does not
 * synchronise. */
int ngd_l2_loss_noalloc(const float *f, const float *target, int64_t q, float *loss,
                        float *grad, void *stream);

/* Relative squared error, the loss the paper trains with (Sec. 4.1 names a
 * relative L2 loss after Noise2Noise): each error is divided by the squared
 * prediction scale, which is held constant for the gradient,
 *   w = 1 / (|f| + eps)^2,
 *   loss = 1/(3q) sum w (f - target)^2,  grad = 2 w (f - target) / (3q).
 * (|f| makes the weight finite for any prediction; for f >= 0 it is the
 * Noise2Noise form, whose eps is 0.01.)  f, target, grad device q x 3; loss
 * device, one float.  eps must be finite and > 0, else NGD_E_INVAL.  Same
 * reduction and errors as ngd_l2_loss.  Does not synchronise. */
int ngd_rel_l2_loss(const float *f, const float *target, int64_t q, float eps,
                    float *loss, float *grad, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NGD_H */
