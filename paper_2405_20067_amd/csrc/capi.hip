// C-ABI of libngd: argument validation, handles, workspaces and error
// reporting around the kernels.  Every check runs on the host before any
// device work, so an invalid call has no effect.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "ngd_internal.hpp"

namespace ngd {
namespace {

thread_local std::string g_err;

struct Allocator {
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(NGD_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

inline hipStream_t S(void *stream) { return static_cast<hipStream_t>(stream); }

bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

}  // namespace

void *dev_alloc(size_t bytes, void (**free_fn)(void *, void *), void **ctx)
{
    Allocator a;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
    }
    *free_fn = a.free_fn;
    *ctx = a.ctx;
    if (a.alloc_fn) return a.alloc_fn(bytes, a.ctx);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

bool DevBuf::ensure(size_t bytes)
{
    if (bytes == 0) bytes = 4;
    if (bytes <= cap) return true;
    release();
    // grow with headroom so repeated rebuilds settle quickly
    const size_t want = bytes + bytes / 8;
    p = dev_alloc(want, &free_fn, &ctx);
    if (!p) return false;
    cap = want;
    // the kernels read workspaces with 16-byte vector loads
    if ((reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
        release();
        return false;
    }
    return true;
}

void DevBuf::release()
{
    if (p) {
        if (free_fn)
            free_fn(p, ctx);
        else
            (void)hipFree(p);
    }
    p = nullptr;
    cap = 0;
    free_fn = nullptr;
    ctx = nullptr;
}

}  // namespace ngd

using namespace ngd;

namespace {
// The shared body of the two losses (rel_eps 0: the plain one).
int l2_loss_impl(const char *who, const float *f, const float *target, int64_t q, float *loss,
                 float *grad, float rel_eps, void *stream)
{
    if (q < 0 || q >= (int64_t(1) << 31))
        return fail(NGD_E_INVAL, "%s: q=%lld outside [0, 2^31)", who, (long long)q);
    if (!loss || (q > 0 && (!f || !target || !grad)))
        return fail(NGD_E_INVAL, "%s: NULL array", who);
    if (!aligned4(f) || !aligned4(target) || !aligned4(grad) || !aligned4(loss))
        return fail(NGD_E_INVAL, "%s: arrays must be 4-byte aligned", who);
    // per-device partial-sum workspace, kept for the life of the process
    constexpr int kParts = 1024;
    static std::mutex mu;
    static DevBuf parts[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (dev < 0 || dev >= 64) return fail(NGD_E_INVAL, "%s: device %d", who, dev);
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!parts[dev].ensure(sizeof(double) * kParts))
            return fail(NGD_E_NOMEM, "%s: workspace allocation failed", who);
    }
    e = launch_l2_loss(f, target, q, loss, grad, parts[dev].as<float>(), kParts, S(stream),
                       rel_eps);
    if (e != hipSuccess) return hip_fail(e, who);
    return NGD_OK;
}
// Partial sums of the allocation-free loss: one array per device, held
// until the process ends.  Host code never passes this name to a kernel or
// a copy (on the host it is only a stand-in for the symbol); it uses the
// device address hipGetSymbolAddress returns for the current device.
constexpr int kStaticParts = 1024;
static __device__ __align__(256) double scratch[kStaticParts];

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
int static_scratch(const char *who, double **out)
{
    static std::mutex mu;
    static double *addr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (dev < 0 || dev >= 64) return fail(NGD_E_INVAL, "%s: device %d", who, dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, who);
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return NGD_OK;
}
}  // namespace

extern "C" {

const char *ngd_last_error(void) { return g_err.c_str(); }

int ngd_version(void) { return 1 * 10000 + 0 * 100 + 0; }

int ngd_cull_params_default(ngd_cull_params *p)
{
    if (!p) return fail(NGD_E_INVAL, "ngd_cull_params_default: p is NULL");
    p->n_proj = 16;
    p->tau = 1e-4f;
    p->tile = 256;
    p->key_proj = 16;
    p->key_bits = 2;
    p->tiling = 0;
    return NGD_OK;
}

int ngd_set_allocator(void *(*alloc_fn)(size_t, void *), void (*free_fn)(void *, void *),
                      void *ctx)
{
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
        return fail(NGD_E_INVAL, "ngd_set_allocator: give both functions or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc_fn = alloc_fn;
    g_alloc.free_fn = free_fn;
    g_alloc.ctx = alloc_fn ? ctx : nullptr;
    return NGD_OK;
}

int ngd_mixture_create(int n, int64_t k, ngd_mixture **out)
{
    if (!out) return fail(NGD_E_INVAL, "ngd_mixture_create: out is NULL");
    *out = nullptr;
    if (n < 1 || n > NGD_MAX_N)
        return fail(NGD_E_INVAL, "ngd_mixture_create: n=%d outside [1, %d]", n, NGD_MAX_N);
    if (k < 0 || k >= (int64_t(1) << 31))
        return fail(NGD_E_INVAL, "ngd_mixture_create: k=%lld outside [0, 2^31)", (long long)k);
    ngd_mixture *m = new (std::nothrow) ngd_mixture();
    if (!m) return fail(NGD_E_NOMEM, "ngd_mixture_create: host allocation failed");
    m->n = n;
    m->k = k;
    const size_t kk = size_t(k > 0 ? k : 1);
    if (!m->rec.ensure(sizeof(float) * kk * rec_stride(n)) ||
        !m->lfac.ensure(sizeof(float) * kk * tri(n)) || !m->flag.ensure(sizeof(int))) {
        m->rec.release();
        m->lfac.release();
        m->flag.release();
        delete m;
        return fail(NGD_E_NOMEM, "ngd_mixture_create: device allocation of %zu bytes failed",
                    sizeof(float) * kk * (rec_stride(n) + tri(n)));
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) m->device = dev;
    (void)hipGetLastError();
    *out = m;
    return NGD_OK;
}

int ngd_mixture_update(ngd_mixture *mix, const float *mean, const float *factor,
                       const float *weight, const float *colour, void *stream)
{
    if (!mix) return fail(NGD_E_INVAL, "ngd_mixture_update: mixture is NULL");
    if (mix->k > 0 && (!mean || !factor || !weight || !colour))
        return fail(NGD_E_INVAL, "ngd_mixture_update: NULL parameter array");
    if (!aligned4(mean) || !aligned4(factor) || !aligned4(weight) || !aligned4(colour))
        return fail(NGD_E_INVAL, "ngd_mixture_update: arrays must be 4-byte aligned");
    hipError_t e = launch_prepare(mix->n, mix->k, mean, factor, weight, colour,
                                  mix->rec.as<float>(), mix->lfac.as<float>(),
                                  mix->flag.as<int>(), S(stream));
    if (e != hipSuccess) return hip_fail(e, "ngd_mixture_update");
    mix->kp = -1;
    ++mix->version;
    return NGD_OK;
}

int ngd_mixture_validate(const ngd_mixture *mix, void *stream)
{
    if (!mix) return fail(NGD_E_INVAL, "ngd_mixture_validate: mixture is NULL");
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, mix->flag.p, sizeof(int), hipMemcpyDeviceToHost,
                                  S(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
    if (e != hipSuccess) return hip_fail(e, "ngd_mixture_validate");
    if (flag & 2)
        return fail(NGD_E_INVAL,
                    "ngd_mixture_validate: a parent index is outside [0, kp) or smaller than "
                    "the one before it");
    if (flag)
        return fail(NGD_E_SINGULAR,
                    "ngd_mixture_validate: a factor has a zero or non-finite diagonal entry, "
                    "or a parameter is not finite");
    return NGD_OK;
}

int ngd_mixture_update_composed(ngd_mixture *mix, int64_t kp, const float *mean,
                                const float *factor, const float *weight, const float *colour,
                                const int32_t *parent, const float *rel_factor,
                                const float *rel_mean, void *stream)
{
    const char *who = "ngd_mixture_update_composed";
    if (!mix) return fail(NGD_E_INVAL, "%s: mixture is NULL", who);
    const int64_t k = mix->k;
    if (kp < 0 || kp > k)
        return fail(NGD_E_INVAL, "%s: kp=%lld outside [0, k=%lld]", who, (long long)kp,
                    (long long)k);
    const int64_t kc = k - kp;
    if (kc > 0 && kp == 0) return fail(NGD_E_INVAL, "%s: children without parents", who);
    if ((kp > 0 && (!mean || !factor)) || (k > 0 && (!weight || !colour)) ||
        (kc > 0 && (!parent || !rel_factor || !rel_mean)))
        return fail(NGD_E_INVAL, "%s: NULL parameter array", who);
    if (!aligned4(mean) || !aligned4(factor) || !aligned4(weight) || !aligned4(colour) ||
        !aligned4(parent) || !aligned4(rel_factor) || !aligned4(rel_mean))
        return fail(NGD_E_INVAL, "%s: arrays must be 4-byte aligned", who);
    const int n = mix->n, t = tri(n);
    const size_t kk = size_t(k > 0 ? k : 1), cc = size_t(kc > 0 ? kc : 1);
    if (!mix->abs_mean.ensure(sizeof(float) * kk * n) ||
        !mix->abs_factor.ensure(sizeof(float) * kk * t) ||
        !mix->comp_parent.ensure(sizeof(int32_t) * cc) ||
        !mix->comp_u.ensure(sizeof(float) * cc * t) || !mix->comp_mu.ensure(sizeof(float) * cc * n))
        return fail(NGD_E_NOMEM, "%s: device allocation failed", who);
    hipError_t e = hipSuccess;
    // the backward applies the chain rule with the same relative parameters
    if (kc > 0) {
        e = hipMemcpyAsync(mix->comp_parent.p, parent, sizeof(int32_t) * kc,
                           hipMemcpyDeviceToDevice, S(stream));
        if (e == hipSuccess)
            e = hipMemcpyAsync(mix->comp_u.p, rel_factor, sizeof(float) * kc * t,
                               hipMemcpyDeviceToDevice, S(stream));
        if (e == hipSuccess)
            e = hipMemcpyAsync(mix->comp_mu.p, rel_mean, sizeof(float) * kc * n,
                               hipMemcpyDeviceToDevice, S(stream));
    }
    if (e == hipSuccess) e = launch_clear_flag(mix->flag.as<int>(), S(stream));
    if (e == hipSuccess)
        e = launch_compose(n, k, kp, mean, factor, mix->comp_parent.as<int32_t>(),
                           mix->comp_u.as<float>(), mix->comp_mu.as<float>(),
                           mix->abs_mean.as<float>(), mix->abs_factor.as<float>(),
                           mix->flag.as<int>(), S(stream));
    if (e == hipSuccess)
        e = launch_prepare(n, k, mix->abs_mean.as<float>(), mix->abs_factor.as<float>(), weight,
                           colour, mix->rec.as<float>(), mix->lfac.as<float>(),
                           mix->flag.as<int>(), S(stream), false);
    if (e != hipSuccess) return hip_fail(e, who);
    mix->kp = kp;
    ++mix->version;
    return NGD_OK;
}

int ngd_mixture_info(const ngd_mixture *mix, int *n, int64_t *k, int64_t *version)
{
    if (!mix) return fail(NGD_E_INVAL, "ngd_mixture_info: mixture is NULL");
    if (n) *n = mix->n;
    if (k) *k = mix->k;
    if (version) *version = mix->version;
    return NGD_OK;
}

int ngd_mixture_destroy(ngd_mixture *mix)
{
    if (!mix) return NGD_OK;
    (void)hipDeviceSynchronize();
    DevBuf *bufs[] = {&mix->rec,    &mix->lfac,       &mix->flag,  &mix->comp_parent,
                      &mix->comp_u, &mix->comp_mu,    &mix->abs_mean, &mix->abs_factor,
                      &mix->g_abs,  &mix->contrib};
    for (DevBuf *b : bufs) b->release();
    delete mix;
    return NGD_OK;
}

static void cull_release(ngd_cull *c)
{
    DevBuf *bufs[] = {&c->proj,    &c->qr,       &c->range_part, &c->qrange,  &c->g_mr,
                      &c->g_thr,   &c->keys0,    &c->keys1,      &c->vals0,   &c->vals1,
                      &c->radix_hist, &c->radix_off, &c->perm,   &c->gperm,   &c->qs,
                      &c->gs,      &c->tile_lo,  &c->tile_hi, &c->tbnd,   &c->sbnd,   &c->qr_s,    &c->grec,    &c->g_mr_s,
                      &c->g_ub, &c->g_lb, &c->masks,    &c->seg_cnt,    &c->tile_cnt, &c->tile_off,
                      &c->cand,    &c->g_cnt,    &c->g_off,      &c->g_tiles, &c->scan_tmp,
                      &c->stats,   &c->item_cnt, &c->item_off,   &c->item_tile, &c->fpart,
                      &c->gitem_cnt, &c->gitem_off, &c->gitem_g, &c->gpart,   &c->gflag,
                      &c->g_ent,   &c->ent_tile, &c->act,       &c->eflag,   &c->eoff,
                      &c->a_cnt,   &c->a_off,    &c->gbox_u,     &c->gbox,
                      &c->kd_q.node_tab, &c->kd_q.slice_tab, &c->kd_g.node_tab,
                      &c->kd_g.slice_tab, &c->kd_work.idx[0], &c->kd_work.idx[1],
                      &c->kd_work.val[0], &c->kd_work.val[1], &c->kd_work.ext[0],
                      &c->kd_work.ext[1], &c->kd_work.hist, &c->kd_work.cnt,
                      &c->kd_work.dim,
                      &c->kd_work.prefix, &c->kd_work.rank, &c->mrec, &c->mrow, &c->tcen,
                      &c->eb0, &c->ebnd};
    for (DevBuf *b : bufs) b->release();
    KdWork *works[] = {&c->kd_work_g};
    for (KdWork *w : works) {
        DevBuf *wb[] = {&w->idx[0], &w->idx[1], &w->val[0], &w->val[1], &w->ext[0], &w->ext[1],
                        &w->hist, &w->cnt, &w->dim, &w->prefix, &w->rank};
        for (DevBuf *b : wb) b->release();
    }
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    if (c->ev_sizes) (void)hipEventDestroy(c->ev_sizes);
    c->side = nullptr;
    c->ev_fork = c->ev_join = c->ev_done = c->ev_sizes = nullptr;
    if (c->stats_host) (void)hipHostFree(c->stats_host);
    c->stats_host = nullptr;
}

int ngd_cull_build(const ngd_mixture *mix, const float *queries, int64_t q,
                   const ngd_cull_params *p, const float *proj, void *stream,
                   ngd_cull **inout)
{
    if (!mix || !p || !proj || !inout)
        return fail(NGD_E_INVAL, "ngd_cull_build: NULL argument");
    if (q < 0 || q >= (int64_t(1) << 31))
        return fail(NGD_E_INVAL, "ngd_cull_build: q=%lld outside [0, 2^31)", (long long)q);
    if (q > 0 && !queries) return fail(NGD_E_INVAL, "ngd_cull_build: queries is NULL");
    if (!aligned4(queries)) return fail(NGD_E_INVAL, "ngd_cull_build: queries not aligned");
    if (p->n_proj < 1 || p->n_proj > NGD_MAX_PROJ)
        return fail(NGD_E_INVAL, "ngd_cull_build: n_proj=%d outside [1, %d]", p->n_proj,
                    NGD_MAX_PROJ);
    if (!(p->tau > 0.0f && p->tau < 1.0f))
        return fail(NGD_E_INVAL, "ngd_cull_build: tau must lie in (0, 1)");
    if (p->tile < 1 || p->tile > 1024)
        return fail(NGD_E_INVAL, "ngd_cull_build: tile=%d outside [1, 1024]", p->tile);
    if (p->key_proj < 0 || p->key_proj > p->n_proj || p->key_bits < 0 ||
        p->key_proj * p->key_bits > 32 || (p->key_proj > 0 && p->key_bits > 16))
        return fail(NGD_E_INVAL, "ngd_cull_build: key_proj=%d key_bits=%d invalid", p->key_proj,
                    p->key_bits);
    if (p->tiling < 0 || p->tiling > 2)
        return fail(NGD_E_INVAL, "ngd_cull_build: tiling=%d (0: k-d, 1: Morton, 2: given order)",
                    p->tiling);
    for (int i = 0; i < p->n_proj * mix->n; ++i)
        if (!std::isfinite(proj[i]))
            return fail(NGD_E_INVAL, "ngd_cull_build: projection vectors must be finite");

    ngd_cull *c = *inout;
    const bool fresh = (c == nullptr);
    if (fresh) {
        c = new (std::nothrow) ngd_cull();
        if (!c) return fail(NGD_E_NOMEM, "ngd_cull_build: host allocation failed");
        if (hipHostMalloc(reinterpret_cast<void **>(&c->stats_host), 3 * sizeof(int64_t),
                          hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            delete c;
            return fail(NGD_E_NOMEM, "ngd_cull_build: pinned host allocation failed");
        }
    }
    auto bail = [&](int code) {
        if (fresh) {
            cull_release(c);
            delete c;
        } else {
            c->mix = nullptr;   // leave the handle unusable rather than half-built
            c->mix_version = -1;
        }
        return code;
    };
    c->mix = mix;
    c->mix_version = mix->version;
    c->queries = queries;
    c->q = q;
    c->n = mix->n;
    c->k = mix->k;
    c->params = *p;
    c->kappa2 = float(-2.0 * std::log(double(p->tau)));
    c->ntiles = (q + p->tile - 1) / p->tile;
    c->tpad = (c->ntiles + 63) / 64 * 64;
    c->nchunks = (mix->k + 63) / 64;
    c->nseg = int(std::min<int64_t>(64, std::max<int64_t>(1, c->nchunks / 16)));
    c->total = 0;
    c->max_per_tile = 0;
    if (!cull_reserve_front(c) ||
        (!c->ev_sizes &&
         hipEventCreateWithFlags(&c->ev_sizes, hipEventDisableTiming) != hipSuccess))
        return bail(fail(NGD_E_NOMEM, "ngd_cull_build: device workspace allocation failed"));
    hipStream_t s = S(stream);
    c->coef_next = false;
    hipError_t e = hipMemcpyAsync(c->proj.p, proj, sizeof(float) * p->n_proj * mix->n,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_cull_build_front(c, mix, queries, s);
    if (e != hipSuccess) return bail(hip_fail(e, "ngd_cull_build (projections, sort, test)"));
    // the only device -> host read: list sizes, gathered into one copy
    e = launch_gather_sizes(c, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->stats_host, c->stats.as<int64_t>() + 1, 3 * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(c->ev_sizes, s);
    // The lists go on at once into the buffers as they are (a rebuild of
    // similar size needs no more), so the device does not wait for the host
    // to read the sizes; lists that do not fit are built again below.
    const int64_t cap_ent =
        int64_t(std::min(c->cand.cap, c->ent_tile.cap) / sizeof(int32_t));
    const int64_t cap_items = int64_t(c->item_tile.cap / sizeof(int32_t));
    if (e == hipSuccess) e = launch_cull_build_lists(c, s, cap_ent, cap_items);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev_sizes);
    if (e != hipSuccess) return bail(hip_fail(e, "ngd_cull_build (list sizes)"));
    c->total = c->stats_host[1];
    c->max_per_tile = (c->ntiles > 0 && c->k > 0) ? c->stats_host[0] : 0;
    c->nitems = c->stats_host[2];
    c->gitems_cap = c->k + (c->total + kItemTiles - 1) / kItemTiles;
    const bool fits = c->total <= cap_ent && c->nitems <= cap_items;
    // before any buffer the lists above write is replaced
    if (!fits && (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(hip_fail(e, "ngd_cull_build (lists)"));
    if (c->total >= (int64_t(1) << 31))
        return bail(fail(NGD_E_NOMEM, "ngd_cull_build: %lld candidates exceed 2^31",
                         (long long)c->total));
    if (!cull_reserve_lists(c))
        return bail(fail(NGD_E_NOMEM, "ngd_cull_build: candidate list allocation failed"));
    c->act_version = -1;
    ++c->build_seq;
    if (c->coef_next) c->coef_seq = c->build_seq;
    c->transposed = false;
    if (!fits) {
        e = launch_cull_build_lists(c, s, c->total, c->nitems);
        if (e != hipSuccess) return bail(hip_fail(e, "ngd_cull_build (lists)"));
    }
    *inout = c;
    return NGD_OK;
}

int ngd_cull_stats(const ngd_cull *c, int64_t *total, int64_t *max_per_tile, int64_t *ntiles)
{
    if (!c) return fail(NGD_E_INVAL, "ngd_cull_stats: cull is NULL");
    if (total) *total = c->total;
    if (max_per_tile) *max_per_tile = c->max_per_tile;
    if (ntiles) *ntiles = c->ntiles;
    return NGD_OK;
}

int ngd_cull_export(const ngd_cull *c, int32_t *perm, int32_t *gperm, int64_t *tile_off,
                    int32_t *cand, int64_t *g_off, int32_t *g_tiles, float *tile_lo,
                    float *tile_hi)
{
    if (!c) return fail(NGD_E_INVAL, "ngd_cull_export: cull is NULL");
    if (!c->mix) return fail(NGD_E_STALE, "ngd_cull_export: cull was not built");
    struct Item {
        void *dst;
        const void *src;
        size_t bytes;
    } items[] = {
        {perm, c->perm.p, sizeof(int32_t) * size_t(c->q)},
        {gperm, c->gperm.p, sizeof(int32_t) * size_t(c->k)},
        {tile_off, c->tile_off.p, sizeof(int64_t) * size_t(c->ntiles + 1)},
        {cand, c->cand.p, sizeof(int32_t) * size_t(c->total)},
        {g_off, c->g_off.p, sizeof(int64_t) * size_t(c->k + 1)},
        {g_tiles, c->g_tiles.p, sizeof(int32_t) * size_t(c->total)},
        {tile_lo, c->tile_lo.p, sizeof(float) * size_t(c->ntiles * c->params.n_proj)},
        {tile_hi, c->tile_hi.p, sizeof(float) * size_t(c->ntiles * c->params.n_proj)},
    };
    hipError_t e = hipSuccess;
    if ((g_off || g_tiles) && !c->transposed) {
        ngd_cull *cm = const_cast<ngd_cull *>(c);
        e = launch_cull_transpose_full(cm, nullptr);
        if (e == hipSuccess) cm->transposed = true;
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    for (const Item &it : items) {
        if (e != hipSuccess) break;
        if (it.dst && it.bytes) e = hipMemcpy(it.dst, it.src, it.bytes, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return hip_fail(e, "ngd_cull_export");
    return NGD_OK;
}

int ngd_cull_destroy(ngd_cull *c)
{
    if (!c) return NGD_OK;
    (void)hipDeviceSynchronize();
    cull_release(c);
    delete c;
    return NGD_OK;
}

static int check_cull(const char *fn, const ngd_mixture *mix, const ngd_cull *c,
                      const float *queries, int64_t q)
{
    if (c->mix != mix || c->mix_version != mix->version)
        return fail(NGD_E_STALE, "%s: cull was built for another mixture or version", fn);
    if (c->queries != queries || c->q != q)
        return fail(NGD_E_STALE, "%s: cull was built for another query buffer or count", fn);
    return NGD_OK;
}

// Coefficient records of the matrix-core forward: grown with the cull.
static int reserve_mfma(const char *fn, ngd_cull *c)
{
    const size_t kk = size_t(c->k > 0 ? c->k : 1);
    const size_t tt = size_t(c->ntiles > 0 ? c->ntiles : 1);
    const size_t ee = size_t(c->total > 0 ? c->total : 1);
    if (!c->mrec.ensure(kk * mfma_rec_bytes(c->n)) || !c->mrow.ensure(kk * sizeof(float)) ||
        !c->tcen.ensure(tt * c->n * sizeof(float)) || !c->eb0.ensure(ee * 4 * 16) ||
        !c->ebnd.ensure(ee * 16)) {
        c->mrec_seq = -1;
        return fail(NGD_E_NOMEM, "%s: coefficient records: allocation failed", fn);
    }
    return NGD_OK;
}

int ngd_eval(const ngd_mixture *mix, const ngd_cull *cull, const float *queries, int64_t q,
             int precision, float *out, void *stream)
{
    if (!mix) return fail(NGD_E_INVAL, "ngd_eval: mixture is NULL");
    if (q < 0 || q >= (int64_t(1) << 31))
        return fail(NGD_E_INVAL, "ngd_eval: q=%lld outside [0, 2^31)", (long long)q);
    if (q > 0 && (!queries || !out)) return fail(NGD_E_INVAL, "ngd_eval: NULL array");
    if (!aligned4(queries) || !aligned4(out))
        return fail(NGD_E_INVAL, "ngd_eval: arrays must be 4-byte aligned");
    if (precision != NGD_FP32 && precision != NGD_BF16_MFMA)
        return fail(NGD_E_INVAL, "ngd_eval: unknown precision %d", precision);
    if (precision == NGD_BF16_MFMA && !cull)
        return fail(NGD_E_INVAL, "ngd_eval: NGD_BF16_MFMA needs a cull");
    if (mix->version == 0) return fail(NGD_E_STALE, "ngd_eval: mixture has no parameters yet");
    if (cull) {
        const int rc = check_cull("ngd_eval", mix, cull, queries, q);
        if (rc) return rc;
    }
    if (q == 0) return NGD_OK;
    hipError_t e;
    if (mix->k == 0 || (cull && cull->nitems == 0)) {
        e = launch_zero_f32(out, 3 * q, S(stream));
    } else if (cull) {
        if (precision == NGD_BF16_MFMA) {
            // the coefficient records are a cache of the cull (grown on use)
            ngd_cull *mc = const_cast<ngd_cull *>(cull);
            const int rc = reserve_mfma("ngd_eval", mc);
            if (rc) return rc;
            e = launch_eval_mfma(mix, mc, out, nullptr, S(stream));
        } else {
            e = launch_eval_culled(mix, cull, out, S(stream));
        }
        if (e == hipSuccess) cull->act_version = mix->version;
    } else {
        e = launch_eval_dense(mix, queries, q, out, S(stream));
    }
    if (e != hipSuccess) return hip_fail(e, "ngd_eval");
    return NGD_OK;
}

int ngd_eval_prepare(const ngd_mixture *mix, const ngd_cull *cull, const float *queries,
                     int64_t q, int precision, void *stream)
{
    if (!mix || !cull) return fail(NGD_E_INVAL, "ngd_eval_prepare: NULL handle");
    if (precision != NGD_FP32 && precision != NGD_BF16_MFMA)
        return fail(NGD_E_INVAL, "ngd_eval_prepare: unknown precision %d", precision);
    if (mix->version == 0) return fail(NGD_E_STALE, "ngd_eval_prepare: mixture has no parameters yet");
    const int rc = check_cull("ngd_eval_prepare", mix, cull, queries, q);
    if (rc) return rc;
    if (precision == NGD_FP32 || q == 0 || mix->k == 0 || cull->nitems == 0) return NGD_OK;
    ngd_cull *mc = const_cast<ngd_cull *>(cull);
    const int rr = reserve_mfma("ngd_eval_prepare", mc);
    if (rr) return rr;
    const hipError_t e = launch_mfma_prepare(mix, mc, S(stream));
    if (e != hipSuccess) return hip_fail(e, "ngd_eval_prepare");
    return NGD_OK;
}

int ngd_eval_stats(const ngd_mixture *mix, const ngd_cull *cull, const float *queries,
                   int64_t q, int precision, int64_t *counts, void *stream)
{
    if (!mix || !cull || !counts) return fail(NGD_E_INVAL, "ngd_eval_stats: NULL argument");
    if (q < 0 || q >= (int64_t(1) << 31))
        return fail(NGD_E_INVAL, "ngd_eval_stats: q=%lld outside [0, 2^31)", (long long)q);
    if (precision != NGD_FP32 && precision != NGD_BF16_MFMA)
        return fail(NGD_E_INVAL, "ngd_eval_stats: unknown precision %d", precision);
    const int rc = check_cull("ngd_eval_stats", mix, cull, queries, q);
    if (rc) return rc;
    for (int i = 0; i < 5; ++i) counts[i] = 0;
    if (q == 0 || mix->k == 0 || cull->nitems == 0) return NGD_OK;
    static std::mutex mu;
    static DevBuf buf[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "ngd_eval_stats");
    if (dev < 0 || dev >= 64) return fail(NGD_E_INVAL, "ngd_eval_stats: device %d", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!buf[dev].ensure(5 * sizeof(unsigned long long)))
        return fail(NGD_E_NOMEM, "ngd_eval_stats: workspace allocation failed");
    if (precision == NGD_BF16_MFMA) {
        const int rm = reserve_mfma("ngd_eval_stats", const_cast<ngd_cull *>(cull));
        if (rm) return rm;
    }
    unsigned long long host[5] = {0, 0, 0, 0, 0};
    e = hipMemcpyAsync(buf[dev].p, host, sizeof(host), hipMemcpyHostToDevice, S(stream));
    if (e == hipSuccess) {
        if (precision == NGD_BF16_MFMA)
            e = launch_eval_mfma(mix, const_cast<ngd_cull *>(cull), nullptr,
                                 buf[dev].as<unsigned long long>(), S(stream));
        else
            e = launch_eval_stats(mix, cull, buf[dev].as<unsigned long long>(), S(stream));
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(host, buf[dev].p, sizeof(host), hipMemcpyDeviceToHost, S(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
    if (e != hipSuccess) return hip_fail(e, "ngd_eval_stats");
    cull->act_version = mix->version;
    for (int i = 0; i < 5; ++i) counts[i] = int64_t(host[i]);
    return NGD_OK;
}

int ngd_eval_backward(const ngd_mixture *mix, const ngd_cull *cull, const float *queries,
                      int64_t q, const float *grad_out, int precision, float *g_mean,
                      float *g_factor, float *g_weight, float *g_colour, void *stream)
{
    if (!mix) return fail(NGD_E_INVAL, "ngd_eval_backward: mixture is NULL");
    if (q < 0 || q >= (int64_t(1) << 31))
        return fail(NGD_E_INVAL, "ngd_eval_backward: q=%lld outside [0, 2^31)", (long long)q);
    if (q > 0 && (!queries || !grad_out))
        return fail(NGD_E_INVAL, "ngd_eval_backward: NULL input array");
    if (mix->k > 0 && (!g_mean || !g_factor || !g_weight || !g_colour))
        return fail(NGD_E_INVAL, "ngd_eval_backward: NULL output array");
    if (!aligned4(queries) || !aligned4(grad_out) || !aligned4(g_mean) || !aligned4(g_factor) ||
        !aligned4(g_weight) || !aligned4(g_colour))
        return fail(NGD_E_INVAL, "ngd_eval_backward: arrays must be 4-byte aligned");
    if (precision != NGD_FP32 && precision != NGD_BF16_MFMA)
        return fail(NGD_E_INVAL, "ngd_eval_backward: unknown precision %d", precision);
    if (precision == NGD_BF16_MFMA && !cull)
        return fail(NGD_E_INVAL, "ngd_eval_backward: NGD_BF16_MFMA needs a cull");
    if (mix->version == 0)
        return fail(NGD_E_STALE, "ngd_eval_backward: mixture has no parameters yet");
    if (cull) {
        const int rc = check_cull("ngd_eval_backward", mix, cull, queries, q);
        if (rc) return rc;
    }
    if (mix->k == 0) return NGD_OK;
    hipError_t e;
    if (cull) {
        // the backward visits the (entry, query group) pairs the forward kept;
        // without a forward on this cull and mixture version, decide them now
        e = hipSuccess;
        if (cull->act_version != mix->version && cull->nitems > 0) {
            if (precision == NGD_BF16_MFMA) {
                const int rm = reserve_mfma("ngd_eval_backward", const_cast<ngd_cull *>(cull));
                if (rm) return rm;
                e = launch_eval_mfma(mix, const_cast<ngd_cull *>(cull), nullptr, nullptr,
                                     S(stream));
            } else {
                e = launch_eval_culled(mix, cull, nullptr, S(stream));
            }
            if (e == hipSuccess) cull->act_version = mix->version;
        }
        if (e == hipSuccess)
            e = launch_backward_culled(mix, const_cast<ngd_cull *>(cull), grad_out, g_mean,
                                       g_factor, g_weight, g_colour, S(stream));
    }
    else
        e = launch_backward_dense(mix, queries, q, grad_out, g_mean, g_factor, g_weight, g_colour,
                                  S(stream));
    if (e != hipSuccess) return hip_fail(e, "ngd_eval_backward");
    return NGD_OK;
}

int ngd_mixture_condition(const ngd_mixture *mix, int p, const float *xc, float *mean_out,
                          float *factor_out, float *weight_out, float *colour_out, void *stream)
{
    const char *who = "ngd_mixture_condition";
    if (!mix) return fail(NGD_E_INVAL, "%s: mixture is NULL", who);
    if (p < 1 || p >= mix->n)
        return fail(NGD_E_INVAL, "%s: p=%d outside [1, n-1=%d]", who, p, mix->n - 1);
    if (!xc) return fail(NGD_E_INVAL, "%s: xc is NULL", who);
    for (int j = 0; j < mix->n - p; ++j)
        if (!std::isfinite(xc[j])) return fail(NGD_E_INVAL, "%s: xc[%d] is not finite", who, j);
    if (mix->k > 0 && (!mean_out || !factor_out || !weight_out || !colour_out))
        return fail(NGD_E_INVAL, "%s: NULL output array", who);
    if (!aligned4(mean_out) || !aligned4(factor_out) || !aligned4(weight_out) ||
        !aligned4(colour_out))
        return fail(NGD_E_INVAL, "%s: arrays must be 4-byte aligned", who);
    if (mix->version == 0) return fail(NGD_E_STALE, "%s: mixture has no parameters yet", who);
    const hipError_t e =
        launch_condition(mix, p, xc, mean_out, factor_out, weight_out, colour_out, S(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return NGD_OK;
}

int ngd_eval_backward_composed(const ngd_mixture *mix, const ngd_cull *cull,
                               const float *queries, int64_t q, const float *grad_out,
                               int precision, float *g_mean, float *g_factor, float *g_weight,
                               float *g_colour, float *g_rel_factor, float *g_rel_mean,
                               void *stream)
{
    const char *who = "ngd_eval_backward_composed";
    if (!mix) return fail(NGD_E_INVAL, "%s: mixture is NULL", who);
    if (mix->kp < 0)
        return fail(NGD_E_INVAL, "%s: the mixture's last update was not composed", who);
    const int64_t kp = mix->kp, kc = mix->k - mix->kp;
    if ((kp > 0 && (!g_mean || !g_factor)) || (kc > 0 && (!g_rel_factor || !g_rel_mean)))
        return fail(NGD_E_INVAL, "%s: NULL output array", who);
    if (!aligned4(g_mean) || !aligned4(g_factor) || !aligned4(g_rel_factor) ||
        !aligned4(g_rel_mean))
        return fail(NGD_E_INVAL, "%s: arrays must be 4-byte aligned", who);
    const int n = mix->n, t = tri(n);
    ngd_mixture *mm = const_cast<ngd_mixture *>(mix);
    const size_t kk = size_t(mix->k > 0 ? mix->k : 1), cc = size_t(kc > 0 ? kc : 1);
    if (!mm->g_abs.ensure(sizeof(float) * kk * (n + t)) ||
        !mm->contrib.ensure(sizeof(float) * cc * (n + t)))
        return fail(NGD_E_NOMEM, "%s: device allocation failed", who);
    float *gm_abs = mm->g_abs.as<float>();
    float *gl_abs = gm_abs + size_t(mix->k) * n;
    // gradients with respect to every Gaussian's absolute parameters (the
    // brightness and colour ones are the result already)
    const int rc = ngd_eval_backward(mix, cull, queries, q, grad_out, precision, gm_abs, gl_abs,
                                     g_weight, g_colour, stream);
    if (rc) return rc;
    if (mix->k == 0) return NGD_OK;
    const hipError_t e = launch_compose_backward(
        n, kp, kc, mix->comp_parent.as<int32_t>(), mix->lfac.as<float>(),
        mix->comp_u.as<float>(), mix->comp_mu.as<float>(), gm_abs, gl_abs, g_mean, g_factor,
        g_rel_factor, g_rel_mean, mm->contrib.as<float>(), S(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return NGD_OK;
}

int ngd_l2_loss(const float *f, const float *target, int64_t q, float *loss, float *grad,
                void *stream)
{
    return l2_loss_impl("ngd_l2_loss", f, target, q, loss, grad, 0.0f, stream);
}

int ngd_l2_loss_noalloc(const float *f, const float *target, int64_t q, float *loss,
                        float *grad, void *stream)
{
    const char *who = "ngd_l2_loss_noalloc";
    if (q < 0 || q > NGD_NOALLOC_MAX_Q)
        return fail(NGD_E_INVAL, "%s: q=%lld outside [0, %lld]", who, (long long)q,
                    (long long)NGD_NOALLOC_MAX_Q);
    if (!loss || (q > 0 && (!f || !target || !grad)))
        return fail(NGD_E_INVAL, "%s: NULL array", who);
    if (!aligned4(f) || !aligned4(target) || !aligned4(grad) || !aligned4(loss))
        return fail(NGD_E_INVAL, "%s: arrays must be 4-byte aligned", who);
    double *parts = nullptr;
    int rc = static_scratch(who, &parts);
    if (rc != NGD_OK) return rc;
    // the same kernels and partition as ngd_l2_loss (kStaticParts partials,
    // each written before the final pass reads it: nothing to clear)
    const hipError_t e = launch_l2_loss(f, target, q, loss, grad, reinterpret_cast<float *>(parts),
                                        kStaticParts, S(stream), 0.0f);
    if (e != hipSuccess) return hip_fail(e, who);
    return NGD_OK;
}

int ngd_rel_l2_loss(const float *f, const float *target, int64_t q, float eps, float *loss,
                    float *grad, void *stream)
{
    if (!(eps > 0.0f) || !std::isfinite(eps))
        return fail(NGD_E_INVAL, "ngd_rel_l2_loss: eps=%g must be finite and > 0", double(eps));
    return l2_loss_impl("ngd_rel_l2_loss", f, target, q, loss, grad, eps, stream);
}

}  // extern "C"
