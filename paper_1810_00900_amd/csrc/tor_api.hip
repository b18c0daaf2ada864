// Host side of the C ABI declared in include/tor.h: validation, the per-query
// reduction of a click pattern to a conditioned matrix Sigma_C, the launch
// plan of the subset-tree kernels, and the final assembly of p, Tor and the
// error bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dd.hpp"
#include "tor.h"
#include "tor_kernels.h"

#pragma clang fp contract(off)

namespace {

thread_local std::string g_err;

tor_status fail(tor_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(TOR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr long long E(long long r) { return r * (2 * r + 1); }
inline long long pidx(long long a, long long b) { return a * (a + 1) / 2 + b; }

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = bytes + bytes / 8;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Bound constants: the relative error of the alternating sum is at most
// c * n * u_term * R (R = cancellation ratio), u_term = 2^-53 for binary64
// terms and 2^-104 for double-double terms (Joldes-Muller-Popescu bounds of
// 3u^2..5u^2 per operation), c = 16 a safety factor for the ~4 dependent
// operations per tree level.
constexpr double kBoundC = 16.0;
constexpr double kUF64 = 1.1102230246251565e-16;   // 2^-53
constexpr double kUDD = 4.930380657631324e-32;     // 2^-104

}  // namespace

struct tor_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    DevBuf pool, descA, descB, partA, partB;
    Partial *host_res = nullptr;
    bool timing = false;
    int task_modes = 9;
    int wave_grid = 65536;
    size_t mem_budget = (size_t)64 << 30;
    tor_stats stats{};
    hipEvent_t ev[6] = {};
};

struct tor_state {
    tor_ctx *ctx = nullptr;
    int m = 0;
    std::vector<double> cov;
};

// ------------------------------------------------------------------ host math

namespace {

tor_status validate_cov(const double *cov, int m) {
    if (!cov) return fail(TOR_EINVAL, "cov is NULL");
    if (m <= 0) return fail(TOR_EINVAL, "m must be positive (got %d)", m);
    if (m > 100000) return fail(TOR_ETOOBIG, "m = %d too large", m);
    const size_t d = 2 * (size_t)m;
    double amax = 0.0;
    for (size_t i = 0; i < d * d; i++) {
        double v = cov[i];
        if (!std::isfinite(v)) return fail(TOR_EINVAL, "cov has a non-finite entry at %zu", i);
        amax = std::max(amax, std::fabs(v));
    }
    const double tol = 1e-12 * amax;
    for (size_t i = 0; i < d; i++)
        for (size_t j = 0; j < i; j++)
            if (std::fabs(cov[i * d + j] - cov[j * d + i]) > tol)
                return fail(TOR_EINVAL, "cov is not symmetric at (%zu, %zu)", i, j);
    return TOR_OK;
}

// Validation of the part of cov a pattern reads: the rows and columns of the
// observed modes (clicked or not) must be finite and symmetric to 1e-12
// relative to the largest entry of that block.
tor_status validate_cov_block(const double *cov, int m, const int8_t *pattern) {
    if (!cov) return fail(TOR_EINVAL, "cov is NULL");
    if (!pattern) return fail(TOR_EINVAL, "pattern is NULL");
    if (m <= 0) return fail(TOR_EINVAL, "m must be positive (got %d)", m);
    if (m > 100000) return fail(TOR_ETOOBIG, "m = %d too large", m);
    const size_t d = 2 * (size_t)m;
    std::vector<int> q;
    for (int i = 0; i < m; i++) {
        if (pattern[i] < -1 || pattern[i] > 1)
            return fail(TOR_EINVAL, "pattern[%d] = %d is not in {-1, 0, 1}", i, (int)pattern[i]);
        if (pattern[i] >= 0) {
            q.push_back(2 * i);
            q.push_back(2 * i + 1);
        }
    }
    double amax = 0.0;
    for (int a : q)
        for (int b : q) {
            double v = cov[(size_t)a * d + b];
            if (!std::isfinite(v)) return fail(TOR_EINVAL, "cov has a non-finite entry at (%d, %d)", a, b);
            amax = std::max(amax, std::fabs(v));
        }
    const double tol = 1e-12 * amax;
    for (size_t x = 0; x < q.size(); x++)
        for (size_t y = 0; y < x; y++)
            if (std::fabs(cov[(size_t)q[x] * d + q[y]] - cov[(size_t)q[y] * d + q[x]]) > tol)
                return fail(TOR_EINVAL, "cov is not symmetric at (%d, %d)", q[x], q[y]);
    return TOR_OK;
}

// sigma_Q entry (double-double) for global quadrature indices
inline dd sigq(const double *cov, int m, int ga, int gb) {
    int r = std::max(ga, gb), c = std::min(ga, gb);
    double v = cov[(size_t)r * (size_t)(2 * m) + (size_t)c];
    if (ga == gb) {
        dd o;
        two_sum(v, 0.5, o.hi, o.lo);
        return o;
    }
    return dd_from(v);
}

// In-place double-double Cholesky of the d x d symmetric matrix A (full
// row-major storage, lower triangle used).  On return the lower triangle
// holds L, rinv[j] = 1 / L_jj.  Returns false on a non-positive pivot.
bool dd_cholesky(std::vector<dd> &A, int d, std::vector<dd> &rinv, double *log_det) {
    rinv.assign(d, dd_from(0.0));
    double ld = 0.0;
    for (int j = 0; j < d; j++) {
        dd s = A[(size_t)j * d + j];
        for (int t = 0; t < j; t++) s = dd_sub(s, dd_mul(A[(size_t)j * d + t], A[(size_t)j * d + t]));
        if (!(s.hi > 0.0)) return false;
        dd r = dd_rsqrt(s);
        rinv[j] = r;
        A[(size_t)j * d + j] = dd_mul(s, r);
        ld += std::log(s.hi) + std::log1p(s.lo / s.hi);
        for (int i = j + 1; i < d; i++) {
            dd v = A[(size_t)i * d + j];
            for (int t = 0; t < j; t++) v = dd_sub(v, dd_mul(A[(size_t)i * d + t], A[(size_t)j * d + t]));
            A[(size_t)i * d + j] = dd_mul(v, r);
        }
    }
    if (log_det) *log_det = ld;
    return true;
}

// Reduce a pattern to Sigma_C (2n x 2n full, double-double) and P_vac(N).
// Marginal patterns (N empty): Sigma_C = sigma_Q[C].  Otherwise the vacuum
// conditioning of Eq. MatrixUpdate over all of N at once:
// sigma_Q[N] = L L^T, W = L^-1 sigma_Q[N, C], Sigma_C = sigma_Q[C] - W^T W,
// P_vac(N) = prod 1/L_ii.
tor_status reduce_pattern(const double *cov, int m, const int8_t *pattern, std::vector<dd> &sig, int &n,
                          dd &pvac, double &log_pvac) {
    if (!pattern) return fail(TOR_EINVAL, "pattern is NULL");
    std::vector<int> C, N;
    for (int i = 0; i < m; i++) {
        int v = pattern[i];
        if (v == 1) C.push_back(i);
        else if (v == 0) N.push_back(i);
        else if (v != -1) return fail(TOR_EINVAL, "pattern[%d] = %d is not in {-1, 0, 1}", i, v);
    }
    n = (int)C.size();
    if (n > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "%d clicks > %d", n, TOR_MAX_CLICKS);
    const int dc = 2 * n, dn = 2 * (int)N.size();
    sig.assign((size_t)dc * dc, dd_from(0.0));
    for (int a = 0; a < dc; a++)
        for (int b = 0; b <= a; b++) {
            dd v = sigq(cov, m, 2 * C[a / 2] + (a & 1), 2 * C[b / 2] + (b & 1));
            sig[(size_t)a * dc + b] = v;
            sig[(size_t)b * dc + a] = v;
        }
    pvac = dd_from(1.0);
    log_pvac = 0.0;
    if (dn == 0) return TOR_OK;
    std::vector<dd> L((size_t)dn * dn), rinv;
    for (int a = 0; a < dn; a++)
        for (int b = 0; b <= a; b++) {
            dd v = sigq(cov, m, 2 * N[a / 2] + (a & 1), 2 * N[b / 2] + (b & 1));
            L[(size_t)a * dn + b] = v;
            L[(size_t)b * dn + a] = v;
        }
    double ld = 0.0;
    if (!dd_cholesky(L, dn, rinv, &ld))
        return fail(TOR_ENOTPD, "sigma_Q restricted to the no-click modes is not positive definite");
    log_pvac = -0.5 * ld;
    for (int i = 0; i < dn; i++) pvac = dd_mul(pvac, rinv[i]);
    if (dc == 0) return TOR_OK;
    std::vector<dd> W((size_t)dn * dc);
    for (int c = 0; c < dc; c++) {
        int gc = 2 * C[c / 2] + (c & 1);
        for (int i = 0; i < dn; i++) {
            dd v = sigq(cov, m, 2 * N[i / 2] + (i & 1), gc);
            for (int t = 0; t < i; t++) v = dd_sub(v, dd_mul(L[(size_t)i * dn + t], W[(size_t)t * dc + c]));
            W[(size_t)i * dc + c] = dd_mul(v, rinv[i]);
        }
    }
    for (int a = 0; a < dc; a++)
        for (int b = 0; b <= a; b++) {
            dd acc = dd_from(0.0);
            for (int t = 0; t < dn; t++) acc = dd_add(acc, dd_mul(W[(size_t)t * dc + a], W[(size_t)t * dc + b]));
            dd v = dd_sub(sig[(size_t)a * dc + b], acc);
            sig[(size_t)a * dc + b] = v;
            sig[(size_t)b * dc + a] = v;
        }
    return TOR_OK;
}

// ------------------------------------------------------------------ GPU plan

double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

// Subset sum T, A of the packed (row-major lower) double-double matrix of n
// modes, on the GPU.  Tree plan: the top n - J levels are expanded in HBM (one
// launch per level), the remaining J modes of each of the 2^(n-J) nodes by the
// wave tier.
tor_status gpu_subset_sum(tor_ctx *ctx, const std::vector<dd> &packed, int n, bool use_dd, dd &T, double &A) {
    if (n == 0) {
        T = dd_from(1.0);
        A = 1.0;
        return TOR_OK;
    }
    const int J = std::min(n, ctx->task_modes);
    const int G = n - J;
    const long long ntasks = 1LL << G;
    const size_t es = use_dd ? sizeof(dd) : sizeof(double);
    // pool layout: root, then the include children of every HBM level
    std::vector<unsigned long long> child_base(G + 1);
    unsigned long long total = (unsigned long long)E(n);
    for (int d = 0; d < G; d++) {
        child_base[d] = total;
        total += (1ULL << d) * (unsigned long long)E(n - d - 1);
    }
    const size_t pool_bytes = total * es;
    const size_t desc_bytes = (size_t)ntasks * sizeof(NodeDesc);
    const size_t part_bytes = (size_t)ntasks * sizeof(Partial);
    if (pool_bytes + 2 * desc_bytes + 2 * part_bytes > ctx->mem_budget)
        return fail(TOR_ENOMEM, "n = %d needs %.2f GB of device memory (budget %.2f GB)", n,
                    (pool_bytes + 2.0 * desc_bytes + 2.0 * part_bytes) / 1e9, ctx->mem_budget / 1e9);
    if (ctx->pool.ensure(pool_bytes) != hipSuccess || ctx->descA.ensure(desc_bytes) != hipSuccess ||
        ctx->descB.ensure(desc_bytes) != hipSuccess || ctx->partA.ensure(part_bytes) != hipSuccess ||
        ctx->partB.ensure(part_bytes / 256 + 4 * sizeof(Partial)) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of %.2f GB failed", pool_bytes / 1e9);
    hipStream_t st = ctx->stream;
    // upload the root
    const size_t ne = (size_t)E(n);
    std::vector<unsigned char> stage(ne * es);
    for (int a = 0; a < 2 * n; a++)
        for (int b = 0; b <= a; b++) {
            dd v = packed[(size_t)pidx(a, b)];
            if (use_dd) {
                ((dd *)stage.data())[pidx(a, b)] = v;
            } else {
                ((double *)stage.data())[pidx(a, b)] = v.hi + v.lo;
            }
        }
    HIP_TRY(hipMemcpyAsync(ctx->pool.p, stage.data(), ne * es, hipMemcpyHostToDevice, st));
    NodeDesc root{0ULL, 1.0, 0.0, 1.0};
    HIP_TRY(hipMemcpyAsync(ctx->descA.p, &root, sizeof root, hipMemcpyHostToDevice, st));
    NodeDesc *cur = (NodeDesc *)ctx->descA.p, *nxt = (NodeDesc *)ctx->descB.p;
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[0], st));
    for (int d = 0; d < G; d++) {
        HIP_TRY(tor_launch_expand(use_dd, cur, 1LL << d, n - d, ctx->pool.p, child_base[d], nxt, 1 << 20, st));
        std::swap(cur, nxt);
    }
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[1], st));
    HIP_TRY(tor_launch_wave(use_dd, J, cur, ntasks, ctx->pool.p, (Partial *)ctx->partA.p, ctx->wave_grid, st));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[2], st));
    Partial *pin = (Partial *)ctx->partA.p, *pout = (Partial *)ctx->partB.p;
    long long cnt = ntasks;
    int nred = 0;
    while (cnt > 1) {
        const long long chunk = 1024;
        HIP_TRY(tor_launch_reduce(pin, cnt, chunk, pout, st));
        cnt = (cnt + chunk - 1) / chunk;
        std::swap(pin, pout);
        nred++;
    }
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[3], st));
    HIP_TRY(hipMemcpyAsync(ctx->host_res, pin, sizeof(Partial), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    T = dd_make(ctx->host_res->t_hi, ctx->host_res->t_lo);
    A = ctx->host_res->a;
    if (ctx->timing) {
        ctx->stats.expand_ms += elapsed(ctx->ev[0], ctx->ev[1]);
        ctx->stats.wave_ms += elapsed(ctx->ev[1], ctx->ev[2]);
        ctx->stats.reduce_ms += elapsed(ctx->ev[2], ctx->ev[3]);
    }
    ctx->stats.expand_launches += G;
    ctx->stats.wave_launches += 1;
    ctx->stats.reduce_launches += nred;
    ctx->stats.subsets += std::ldexp(1.0, n);
    if (!std::isfinite(T.hi) || !std::isfinite(A))
        return fail(TOR_ENOTPD, "a Schur pivot was not positive (non-physical or near-singular covariance)");
    return TOR_OK;
}

void pack_lower(const std::vector<dd> &full, int n, std::vector<dd> &packed) {
    const int d = 2 * n;
    packed.assign((size_t)E(n), dd_from(0.0));
    for (int a = 0; a < d; a++)
        for (int b = 0; b <= a; b++) packed[(size_t)pidx(a, b)] = full[(size_t)a * d + b];
}

// Full evaluation from Sigma_C: PD check and log det on the host, the subset
// sum on the GPU with the requested precision policy, and the final fields.
tor_status evaluate(tor_ctx *ctx, const std::vector<dd> &sig, int n, dd pvac, double log_pvac, tor_prec prec,
                    double tol, tor_result *out) {
    if (!out) return fail(TOR_EINVAL, "out is NULL");
    if (prec != TOR_PREC_AUTO && prec != TOR_PREC_F64 && prec != TOR_PREC_DD)
        return fail(TOR_EINVAL, "bad precision %d", (int)prec);
    if (!(tol > 0.0)) tol = 1e-10;
    std::vector<dd> chol = sig, rinv;
    double log_det = 0.0;
    if (n > 0 && !dd_cholesky(chol, 2 * n, rinv, &log_det))
        return fail(TOR_ENOTPD, "Sigma_C is not positive definite");
    std::vector<dd> packed;
    pack_lower(sig, n, packed);
    dd T;
    double A;
    int used = prec == TOR_PREC_DD ? TOR_PREC_DD : TOR_PREC_F64;
    tor_status s = gpu_subset_sum(ctx, packed, n, used == TOR_PREC_DD, T, A);
    if (s < 0) return s;
    auto bound_of = [&](int pu, dd t, double a) {
        double R = a / std::fabs(t.hi);
        return kBoundC * std::max(n, 1) * (pu == TOR_PREC_DD ? kUDD : kUF64) * R;
    };
    double bound = bound_of(used, T, A);
    if (prec == TOR_PREC_AUTO && !(bound <= tol) && n > 0) {
        used = TOR_PREC_DD;
        s = gpu_subset_sum(ctx, packed, n, true, T, A);
        if (s < 0) return s;
        bound = bound_of(used, T, A);
    }
    dd p = dd_mul(pvac, T);
    std::memset(out, 0, sizeof *out);
    out->p = p.hi + p.lo;
    out->p_lo = p.lo - (out->p - p.hi);
    out->log_p = out->p > 0 ? log_pvac + std::log(T.hi) + std::log1p(T.lo / T.hi) : -INFINITY;
    out->T = T.hi;
    out->T_lo = T.lo;
    out->tor = std::exp(0.5 * log_det) * (T.hi + T.lo);
    out->abs_sum = A;
    out->cancel_ratio = A / std::fabs(T.hi);
    out->rel_err_bound = bound;
    out->log_pvac_n = log_pvac;
    out->n_clicks = n;
    out->prec_used = used;
    out->status = bound <= tol ? TOR_OK : TOR_WARN_PRECISION;
    return out->status;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *tor_last_error(void) { return g_err.c_str(); }

tor_status tor_ctx_create(int device, tor_ctx **out) {
    if (!out) return fail(TOR_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(TOR_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    tor_ctx *c = new (std::nothrow) tor_ctx();
    if (!c) return fail(TOR_ENOMEM, "host allocation failed");
    c->device = device;
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(TOR_EDEVICE, "hipStreamCreate failed");
    }
    c->stream = c->own_stream;
    if (hipHostMalloc((void **)&c->host_res, sizeof(Partial) * 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(c->own_stream);
        delete c;
        return fail(TOR_ENOMEM, "pinned allocation failed");
    }
    for (auto &e : c->ev) (void)hipEventCreate(&e);
    *out = c;
    return TOR_OK;
}

void tor_ctx_destroy(tor_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->pool.release();
    c->descA.release();
    c->descB.release();
    c->partA.release();
    c->partB.release();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->host_res) (void)hipHostFree(c->host_res);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

tor_status tor_ctx_set_stream(tor_ctx *c, void *stream) {
    if (!c) return fail(TOR_EINVAL, "ctx is NULL");
    c->stream = stream ? (hipStream_t)stream : c->own_stream;
    return TOR_OK;
}

tor_status tor_ctx_set_option(tor_ctx *c, tor_option opt, int64_t v) {
    if (!c) return fail(TOR_EINVAL, "ctx is NULL");
    switch (opt) {
    case TOR_OPT_TIMING: c->timing = v != 0; return TOR_OK;
    case TOR_OPT_TASK_MODES:
        if (v < 1 || v > 9) return fail(TOR_EINVAL, "task modes must be in 1..9");
        c->task_modes = (int)v;
        return TOR_OK;
    case TOR_OPT_WAVE_GRID:
        if (v < 1 || v > (1LL << 30)) return fail(TOR_EINVAL, "bad wave grid cap");
        c->wave_grid = (int)v;
        return TOR_OK;
    case TOR_OPT_MEM_BUDGET:
        if (v < (1 << 20)) return fail(TOR_EINVAL, "memory budget too small");
        c->mem_budget = (size_t)v;
        return TOR_OK;
    }
    return fail(TOR_EINVAL, "unknown option %d", (int)opt);
}

tor_status tor_ctx_get_stats(const tor_ctx *c, tor_stats *out) {
    if (!c || !out) return fail(TOR_EINVAL, "NULL argument");
    *out = c->stats;
    return TOR_OK;
}

tor_status tor_ctx_reset_stats(tor_ctx *c) {
    if (!c) return fail(TOR_EINVAL, "ctx is NULL");
    c->stats = tor_stats{};
    return TOR_OK;
}

tor_status tor_probability(tor_ctx *ctx, const double *cov, int32_t m, const int8_t *pattern, tor_prec prec,
                           double tol, tor_result *out) {
    if (!ctx) return fail(TOR_EINVAL, "ctx is NULL");
    tor_status s = validate_cov_block(cov, m, pattern);
    if (s) return s;
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<dd> sig;
    int n = 0;
    dd pvac;
    double log_pvac;
    s = reduce_pattern(cov, m, pattern, sig, n, pvac, log_pvac);
    if (s) return s;
    return evaluate(ctx, sig, n, pvac, log_pvac, prec, tol, out);
}

tor_status tor_subset_sum(tor_ctx *ctx, const double *sigma_hi, const double *sigma_lo, int32_t n, tor_prec prec,
                          double tol, tor_result *out) {
    if (!ctx || !sigma_hi) return fail(TOR_EINVAL, "NULL argument");
    if (n < 0) return fail(TOR_EINVAL, "n must be >= 0");
    if (n > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "n = %d > %d", n, TOR_MAX_CLICKS);
    HIP_TRY(hipSetDevice(ctx->device));
    const int d = 2 * n;
    std::vector<dd> sig((size_t)d * d);
    double amax = 0.0;
    for (int i = 0; i < d * d; i++) {
        double h = sigma_hi[i], l = sigma_lo ? sigma_lo[i] : 0.0;
        if (!std::isfinite(h) || !std::isfinite(l)) return fail(TOR_EINVAL, "non-finite entry %d", i);
        two_sum(h, l, sig[i].hi, sig[i].lo);
        amax = std::max(amax, std::fabs(h));
    }
    for (int i = 0; i < d; i++)
        for (int j = 0; j < i; j++) {
            // use the lower triangle; check symmetry of the leading words
            if (std::fabs(sigma_hi[i * d + j] - sigma_hi[j * d + i]) > 1e-12 * amax)
                return fail(TOR_EINVAL, "Sigma is not symmetric at (%d, %d)", i, j);
            sig[(size_t)j * d + i] = sig[(size_t)i * d + j];
        }
    return evaluate(ctx, sig, n, dd_from(1.0), 0.0, prec, tol, out);
}

tor_status tor_state_create(tor_ctx *ctx, const double *cov, int32_t m, tor_state **out) {
    if (!ctx || !out) return fail(TOR_EINVAL, "NULL argument");
    *out = nullptr;
    tor_status s = validate_cov(cov, m);
    if (s) return s;
    tor_state *st = new (std::nothrow) tor_state();
    if (!st) return fail(TOR_ENOMEM, "host allocation failed");
    st->ctx = ctx;
    st->m = m;
    try {
        st->cov.assign(cov, cov + 4 * (size_t)m * m);
    } catch (...) {
        delete st;
        return fail(TOR_ENOMEM, "host allocation failed");
    }
    *out = st;
    return TOR_OK;
}

void tor_state_destroy(tor_state *st) { delete st; }

tor_status tor_batch(tor_ctx *ctx, const tor_state *st, int32_t nq, const int8_t *patterns, tor_prec prec,
                     double tol, tor_result *out) {
    if (!ctx || !st || !out || (nq > 0 && !patterns)) return fail(TOR_EINVAL, "NULL argument");
    if (st->ctx != ctx) return fail(TOR_EINVAL, "state belongs to another context");
    if (nq < 0) return fail(TOR_EINVAL, "nq < 0");
    HIP_TRY(hipSetDevice(ctx->device));
    tor_status first = TOR_OK;
    for (int q = 0; q < nq; q++) {
        std::vector<dd> sig;
        int n = 0;
        dd pvac;
        double log_pvac;
        tor_status s = reduce_pattern(st->cov.data(), st->m, patterns + (size_t)q * st->m, sig, n, pvac, log_pvac);
        if (s == TOR_OK) s = evaluate(ctx, sig, n, pvac, log_pvac, prec, tol, &out[q]);
        if (s < 0) {
            std::memset(&out[q], 0, sizeof out[q]);
            out[q].status = s;
            if (first >= 0) first = s;
        } else if (s == TOR_WARN_PRECISION && first == TOR_OK) {
            first = s;
        }
    }
    return first;
}

}  // extern "C"
