/*
 * CPU oracle for the N-D Gaussian mixture hot path -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  The product path (the HIP library) never calls it and
 * shares no code, header or constant with it.
 *
 * Everything here is plain float64 written straight from the definitions:
 *
 *   Gaussian (Sec. 3.1, Eq. 1):     G(x - m) = exp(-1/2 (x-m)^T V^-1 (x-m))
 *                                   (unnormalised: no (2 pi)^{-N/2}|V|^{-1/2})
 *   Parameterisation (Eq. 2):       V = L L^T, L lower triangular
 *   Mixture colour (Sec. 4.1, Eq. 8): c(x) = sum_i G_i(x - m_i) alpha_i c_i
 *
 * The quadratic form is evaluated by forward substitution: solve L y = d,
 * then (x-m)^T V^-1 (x-m) = y^T y.  No inverse, no culling, no blocking.
 *
 * Gradients (the paper computes them analytically, Sec. 4.1, and prints no
 * formulas; these follow from the definitions):
 *   with y = L^-1 d, z = L^-T y = V^-1 d, s = g . c, w = alpha G s
 *     dl/dalpha = sum_q G s
 *     dl/dc     = sum_q alpha G g
 *     dl/dm     = sum_q w z                (dG/dm = G z)
 *     dl/dL     = tril(sum_q w z y^T)      (dM = -2 z^T dL y)
 *
 * Inputs are the float32 values the GPU receives, promoted exactly to float64
 * by the caller.  Layouts (all row-major, C-contiguous):
 *   mean   k x n
 *   factor k x n(n+1)/2, packed lower triangle by rows: idx(i,j)=i(i+1)/2+j
 *   weight k
 *   colour k x 3
 *   x      q x n  (queries)
 *   out    q x 3
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_N 32

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the oracle's parallel loops use. */
int ngd_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of the later parallel loops (timing on one core or all);
 * returns the count now in force. */
int ngd_oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

static inline int64_t tri_idx(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

/* Solve L y = d (forward substitution), return y^T y. */
static double mahalanobis_sq(int n, const double *L, const double *d, double *y)
{
    double msq = 0.0;
    for (int r = 0; r < n; ++r) {
        double acc = d[r];
        for (int j = 0; j < r; ++j) acc -= L[tri_idx(r, j)] * y[j];
        y[r] = acc / L[tri_idx(r, r)];
        msq += y[r] * y[r];
    }
    return msq;
}

/* Solve L^T z = y (back substitution). */
static void back_substitute(int n, const double *L, const double *y, double *z)
{
    for (int r = n - 1; r >= 0; --r) {
        double acc = y[r];
        for (int j = r + 1; j < n; ++j) acc -= L[tri_idx(j, r)] * z[j];
        z[r] = acc / L[tri_idx(r, r)];
    }
}

/* One Gaussian's value at one query. */
double ngd_oracle_gaussian(int n, const double *mean, const double *factor,
                           const double *x)
{
    double d[ORACLE_MAX_N], y[ORACLE_MAX_N];
    for (int a = 0; a < n; ++a) d[a] = x[a] - mean[a];
    return exp(-0.5 * mahalanobis_sq(n, factor, d, y));
}

/* Full direct sum (Eq. 8) over all k Gaussians for each of q queries. */
int ngd_oracle_eval(int n, int64_t k, const double *mean, const double *factor,
                    const double *weight, const double *colour, int64_t q,
                    const double *x, double *out)
{
    if (n < 1 || n > ORACLE_MAX_N) return -1;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < q; ++p) {
        double acc[3] = {0.0, 0.0, 0.0};
        double d[ORACLE_MAX_N], y[ORACLE_MAX_N];
        for (int64_t i = 0; i < k; ++i) {
            for (int a = 0; a < n; ++a) d[a] = x[p * n + a] - mean[i * n + a];
            double g = exp(-0.5 * mahalanobis_sq(n, factor + i * tri, d, y));
            for (int ch = 0; ch < 3; ++ch) acc[ch] += weight[i] * colour[i * 3 + ch] * g;
        }
        for (int ch = 0; ch < 3; ++ch) out[p * 3 + ch] = acc[ch];
    }
    return 0;
}

/* The same sum restricted, per query p, to the Gaussians
 * idx[off[p] .. off[p+1]) -- used to compare a culled evaluation against the
 * definition on exactly the pairs it kept. */
int ngd_oracle_eval_lists(int n, const double *mean, const double *factor,
                          const double *weight, const double *colour, int64_t q,
                          const double *x, const int64_t *off, const int32_t *idx,
                          double *out)
{
    if (n < 1 || n > ORACLE_MAX_N) return -1;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < q; ++p) {
        double acc[3] = {0.0, 0.0, 0.0};
        double d[ORACLE_MAX_N], y[ORACLE_MAX_N];
        for (int64_t e = off[p]; e < off[p + 1]; ++e) {
            int64_t i = idx[e];
            for (int a = 0; a < n; ++a) d[a] = x[p * n + a] - mean[i * n + a];
            double g = exp(-0.5 * mahalanobis_sq(n, factor + i * tri, d, y));
            for (int ch = 0; ch < 3; ++ch) acc[ch] += weight[i] * colour[i * 3 + ch] * g;
        }
        for (int ch = 0; ch < 3; ++ch) out[p * 3 + ch] = acc[ch];
    }
    return 0;
}

/* Gradient of l with respect to the parameters of the Gaussians listed in
 * sel[0..nsel) (all k if sel == NULL), given g = dl/df (q x 3), summed over
 * all q queries.  Outputs are indexed by position in sel:
 *   g_mean nsel x n, g_factor nsel x tri, g_weight nsel, g_colour nsel x 3. */
int ngd_oracle_grad(int n, int64_t k, const double *mean, const double *factor,
                    const double *weight, const double *colour, int64_t q,
                    const double *x, const double *g, const int64_t *sel,
                    int64_t nsel, double *g_mean, double *g_factor,
                    double *g_weight, double *g_colour)
{
    if (n < 1 || n > ORACLE_MAX_N) return -1;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    if (!sel) nsel = k;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nsel; ++s) {
        const int64_t i = sel ? sel[s] : s;
        const double *m = mean + i * n, *L = factor + i * tri;
        const double alpha = weight[i], *c = colour + i * 3;
        double gm[ORACLE_MAX_N] = {0}, gl[ORACLE_MAX_N * (ORACLE_MAX_N + 1) / 2] = {0};
        double ga = 0.0, gc[3] = {0.0, 0.0, 0.0};
        double d[ORACLE_MAX_N], y[ORACLE_MAX_N], z[ORACLE_MAX_N];
        for (int64_t p = 0; p < q; ++p) {
            for (int a = 0; a < n; ++a) d[a] = x[p * n + a] - m[a];
            const double G = exp(-0.5 * mahalanobis_sq(n, L, d, y));
            const double *gp = g + p * 3;
            const double sdot = gp[0] * c[0] + gp[1] * c[1] + gp[2] * c[2];
            const double w = alpha * G * sdot;
            ga += G * sdot;
            for (int ch = 0; ch < 3; ++ch) gc[ch] += alpha * G * gp[ch];
            back_substitute(n, L, y, z);
            for (int a = 0; a < n; ++a) {
                gm[a] += w * z[a];
                for (int b = 0; b <= a; ++b) gl[tri_idx(a, b)] += w * z[a] * y[b];
            }
        }
        for (int a = 0; a < n; ++a) g_mean[s * n + a] = gm[a];
        for (int64_t e = 0; e < tri; ++e) g_factor[s * tri + e] = gl[e];
        g_weight[s] = ga;
        for (int ch = 0; ch < 3; ++ch) g_colour[s * 3 + ch] = gc[ch];
    }
    return 0;
}

/* Gradient restricted to (query, Gaussian) pairs: for each listed Gaussian
 * sel[s] the queries qidx[qoff[s] .. qoff[s+1]) only.  Same outputs as
 * ngd_oracle_grad. */
int ngd_oracle_grad_lists(int n, const double *mean, const double *factor,
                          const double *weight, const double *colour,
                          const double *x, const double *g, const int64_t *sel,
                          int64_t nsel, const int64_t *qoff, const int64_t *qidx,
                          double *g_mean, double *g_factor, double *g_weight,
                          double *g_colour)
{
    if (n < 1 || n > ORACLE_MAX_N) return -1;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nsel; ++s) {
        const int64_t i = sel[s];
        const double *m = mean + i * n, *L = factor + i * tri;
        const double alpha = weight[i], *c = colour + i * 3;
        double gm[ORACLE_MAX_N] = {0}, gl[ORACLE_MAX_N * (ORACLE_MAX_N + 1) / 2] = {0};
        double ga = 0.0, gc[3] = {0.0, 0.0, 0.0};
        double d[ORACLE_MAX_N], y[ORACLE_MAX_N], z[ORACLE_MAX_N];
        for (int64_t e = qoff[s]; e < qoff[s + 1]; ++e) {
            const int64_t p = qidx[e];
            for (int a = 0; a < n; ++a) d[a] = x[p * n + a] - m[a];
            const double G = exp(-0.5 * mahalanobis_sq(n, L, d, y));
            const double *gp = g + p * 3;
            const double sdot = gp[0] * c[0] + gp[1] * c[1] + gp[2] * c[2];
            const double w = alpha * G * sdot;
            ga += G * sdot;
            for (int ch = 0; ch < 3; ++ch) gc[ch] += alpha * G * gp[ch];
            back_substitute(n, L, y, z);
            for (int a = 0; a < n; ++a) {
                gm[a] += w * z[a];
                for (int b = 0; b <= a; ++b) gl[tri_idx(a, b)] += w * z[a] * y[b];
            }
        }
        for (int a = 0; a < n; ++a) g_mean[s * n + a] = gm[a];
        for (int64_t e = 0; e < tri; ++e) g_factor[s * tri + e] = gl[e];
        g_weight[s] = ga;
        for (int ch = 0; ch < 3; ++ch) g_colour[s * 3 + ch] = gc[ch];
    }
    return 0;
}

/* Mahalanobis distance squared of every (query, Gaussian) pair listed:
 * msq[e] for the pair (qi[e], gi[e]).  Used by the cull's safety checks. */
int ngd_oracle_msq_pairs(int n, const double *mean, const double *factor,
                         const double *x, int64_t npairs, const int64_t *qi,
                         const int64_t *gi, double *msq)
{
    if (n < 1 || n > ORACLE_MAX_N) return -1;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < npairs; ++e) {
        double d[ORACLE_MAX_N], y[ORACLE_MAX_N];
        for (int a = 0; a < n; ++a) d[a] = x[qi[e] * n + a] - mean[gi[e] * n + a];
        msq[e] = mahalanobis_sq(n, factor + gi[e] * tri, d, y);
    }
    return 0;
}
