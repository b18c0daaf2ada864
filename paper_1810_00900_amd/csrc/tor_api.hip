// Host side of the C ABI declared in include/tor.h: validation, the per-query
// reduction of a click pattern to a conditioned matrix Sigma_C, the launch
// plan of the subset-tree kernels, and the final assembly of p, Tor and the
// error bound.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dd.hpp"
#include "qd.hpp"
#include "tor.h"
#include "tor_gather.h"
#include "tor_invert.h"
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
// entries of an r-mode packed matrix with D leading mean rows (D = 0 or 1)
constexpr long long EN(long long r, int D) { return (2 * r + D) * (2 * r + D + 1) / 2; }
constexpr int MR(int D) { return D != 0 ? 1 : 0; }  // mean rows of a tree kind (0, 1 or -1)
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
constexpr double kUQD = 2.4308653429145085e-63;    // 2^-208 (quad-double terms)

}  // namespace

// Workspace of tor_batch_async_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  In host code its name is only a
// stand-in: the device address of each GPU's copy comes from
// hipGetSymbolAddress (scratch_setup, at context creation) and is the only
// address host code passes on.
static __device__ __align__(256) unsigned char scratch[TOR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
std::string g_scratch_err[kMaxScratchDevices];

// Resolve this device's copy of scratch (the caller has made `device`
// current); once per device.  A failure is kept and reported by the
// allocation-free entry point, not by context creation.
void scratch_setup(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return;
    }
    g_scratch_ptr[device] = ptr;
}

void *scratch_of(int device, std::string *err) {
    if (device < 0 || device >= kMaxScratchDevices) {
        *err = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}

}  // namespace

// tor_probability gathers (C, N) on the device from one copy of the covariance
// when the pattern observes at least half of the modes and has at least this
// many no-click modes (host packing of the (C, N) matrix costs more than the copy).
constexpr int kDeviceGatherNoClick = 64;

// Panel workgroups per blocked-conditioning launch before a workgroup takes
// several column groups (eight per CU).
constexpr long long kPanelWorkgroups = 2048;

struct tor_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    DevBuf pool, descA, descB, partA, partB, jobs, cond;
    DevBuf apool, abuf;  // tor_batch_async: tree pool, plan and job tables
    size_t async_pool = (size_t)4 << 30;
    int chain_clicks = 15;  // click cap of chains without postselection
    int cond_block = TOR_COND_BLOCK;  // no-click modes per conditioning launch pair (1: one launch per mode)
    bool fused = true;  // small zero-mean trees in one launch (tor_fused.hip)
    DevBuf cov_tmp;     // tor_probability: device copy of the caller's covariance for device-side gathers
    DevBuf screen;      // its screen's words and the observed rows
    unsigned long long *screen_host = nullptr;  // pinned copy of the screen's words
    DevBuf fctr;        // completion counters of the single-launch path (zero between launches)
    unsigned char *pin_stage = nullptr;  // pinned upload buffer of the single-launch path
    size_t pin_cap = 0;
    DevBuf kbuf, koff, hbuf, hoff, c_out, c_status, c_tp, c_tu, c_sub;
    DevBuf klobuf, hlobuf, c_tr, c_tb;  // double-double chain tables; per-step ratio and bound
    int chain_prec = TOR_PREC_F64;      // term precision of gbs_sample / gbs_trace chains
    Partial *host_res = nullptr;
    size_t host_res_cap = 0;
    std::vector<unsigned char> host_jobs, host_stage;
    bool timing = false;
    // wave-tier task size per precision [f64, dd] unless tuned: measured best
    // on MI355X for the large trees (n >= 24)
    int task_modes[2] = {11, 10};
    // autotuned task size per (precision, n); 0 = use task_modes
    int tuned[2][TOR_MAX_CLICKS + 1] = {};
    // persistent-server schedule per n (double-double terms): depth-first
    // levels per unit plus one; 0 = the default rule
    int ps_t1[TOR_MAX_CLICKS + 1] = {};
    int wave_grid = 65536;
    size_t mem_budget = (size_t)64 << 30;
    tor_stats stats{};
    hipEvent_t ev[6] = {};
};

struct tor_state {
    tor_ctx *ctx = nullptr;
    int device = 0;  // the context's device, kept for the release of dcov
    int m = 0;
    std::vector<double> cov;
    std::vector<double> mean;  // displaced states only (2m entries), else empty
    DevBuf dmean;               // device copy of the mean for tor_batch_async (made on first use)
    DevBuf dcov;  // device copy for tor_batch_async (made on first use)
    // tor_state_invert: sigma_Q^-1 in packed lower storage (double-double or
    // quad-double words), det(sigma_Q)^-1/2 and log det sigma_Q
    int inv_prec = 0;  // 0: not inverted; TOR_PREC_DD or TOR_PREC_QD
    std::vector<dd> inv;
    std::vector<qd> inv_q;
    dd det_rsqrt = {1.0, 0.0};
    double log_det_sigq = 0.0;
    // displaced states: h = sigma_Q^-1 mu (2m words), mu^T sigma_Q^-1 mu and
    // det(sigma_Q)^-1/2 exp(-mu^T sigma_Q^-1 mu / 2)
    std::vector<dd> inv_h;
    std::vector<qd> inv_h_q;  // h in quad-double words (quad-double inverse)
    dd mu_k_mu = {0.0, 0.0};
    dd det_rsqrt_mean = {1.0, 0.0};
    DevBuf dinv;   // device copy of the inverse in double-double words for tor_batch_async (first use)
    DevBuf dinvh;  // device copy of h (displaced states), likewise
    DevBuf dK;  // the sampler's tables for the persistent server (first use): K_j offsets, then K_j
    size_t k_off_bytes = 0;
    std::mutex dev_mu;  // guards the creation of the device copies (dcov, dmean)
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
    // symmetry, in 32 x 32 tiles (the transposed reads of a tile stay in cache)
    const double tol = 1e-12 * amax;
    const size_t nq = q.size();
    for (size_t x0 = 0; x0 < nq; x0 += 32)
        for (size_t y0 = 0; y0 <= x0; y0 += 32)
            for (size_t x = x0; x < std::min(nq, x0 + 32); x++)
                for (size_t y = y0; y < std::min(x, y0 + 32); y++)
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

// A pattern reduced to what the subset tree needs.  Marginal patterns (no
// no-click modes): Sigma_C = sigma_Q[C] and P_vac = 1, formed here.  Otherwise
// the vacuum conditioning of Eq. MatrixUpdate over N runs on the GPU
// (condition_on_gpu): `packed` holds sigma_Q over (C, N), clicked modes first,
// in packed lower storage, and each step conditions on the last remaining
// mode; P_vac(N) is the product of the steps' pivot factors q.
struct Reduced {
    std::vector<dd> sig;  // Sigma_C, 2n x 2n full (zero-mean states)
    int n = 0;
    int D = 0;            // 1: displaced state; `packed` has the mean row first and
                          // holds the conditioned matrix once cond is cleared
    dd pvac = {1.0, 0.0};
    double log_pvac = 0.0;
    bool cond = false;          // conditioning on N still to do
    int k = 0;                  // |N|
    std::vector<dd> packed;     // sigma_Q over (C, N), EN(n + k, D) entries
    // gathered on the device instead (queries of a state): the rows of (C, N)
    // as global quadrature indices; packed stays empty until conditioned
    const tor_state *st = nullptr;
    std::vector<int> g;
    // full pattern on an inverted state: sig holds G = sigma_Q^-1 over C (not
    // Sigma_C = G^-1), and the tree's sum of G times tscale = (-1)^n det(G)^1/2
    // is the sum of Sigma_C
    bool jacobi = false;
    dd tscale = {1.0, 0.0};
    dd pdirect = {1.0, 0.0};  // (-1)^n det(sigma_Q)^-1/2: p = pdirect T(G)
    // sum over the elimination steps that formed the tree's matrix of their
    // unit roundoff: k u for k no-click conditioning steps, m u for the m
    // sweeps of a state's inverse (0 for a marginal pattern, whose sigma_Q[C]
    // is exact); enters the error bound beside the tree's own n u
    double cond_u = 0.0;
};

// Displaced state (mean mu, hbar = 1, interleaved like cov): the packed matrix
// over (C, N) gets a leading row [0, mu^T] (rows of mode k: 1 + 2k, 2 + 2k), so
// that each vacuum-conditioning step moves the mean with the covariance
// (r_A <- r_A - sigma_AB sigma_Q[B]^-1 r_B, Sec. II) and each pivot factor q
// gains exp(-w^T w / 2), w = L^-1 r_B, L the Cholesky factor of the pivot
// block (the vacuum overlap of a displaced Gaussian).  Conditioning runs on the
// GPU when N is not empty.
tor_status reduce_pattern_disp(const double *cov, const double *mean, int m, const int8_t *pattern,
                               Reduced &out, bool defer = false) {
    if (!pattern) return fail(TOR_EINVAL, "pattern is NULL");
    if (!mean) return fail(TOR_EINVAL, "mean is NULL");
    std::vector<int> C, N;
    for (int i = 0; i < m; i++) {
        int v = pattern[i];
        if (v == 1) C.push_back(i);
        else if (v == 0) N.push_back(i);
        else if (v != -1) return fail(TOR_EINVAL, "pattern[%d] = %d is not in {-1, 0, 1}", i, v);
    }
    const int n = (int)C.size(), k = (int)N.size();
    if (n > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "%d clicks > %d", n, TOR_MAX_CLICKS);
    if (n + k > TOR_COND_MAX_MODES)
        return fail(TOR_ETOOBIG, "%d observed modes > %d", n + k, TOR_COND_MAX_MODES);
    std::vector<int> g;  // quadrature index of each covariance row of the (C, N) matrix
    for (int c : C) {
        g.push_back(2 * c);
        g.push_back(2 * c + 1);
    }
    for (int c : N) {
        g.push_back(2 * c);
        g.push_back(2 * c + 1);
    }
    for (int q : g)
        if (!std::isfinite(mean[q])) return fail(TOR_EINVAL, "mean[%d] is not finite", q);
    out = Reduced();
    out.n = n;
    out.k = k;
    out.D = 1;
    if (defer && k > 0) {  // gathered on the device by condition_on_gpu
        out.g = std::move(g);
        out.cond = true;
        return TOR_OK;
    }
    const int d = (int)g.size();
    out.packed.resize((size_t)EN(n + k, 1));
    out.packed[0] = dd_from(0.0);
    for (int a = 0; a < d; a++) {
        out.packed[(size_t)pidx(a + 1, 0)] = dd_from(mean[g[a]]);
        for (int b = 0; b <= a; b++) out.packed[(size_t)pidx(a + 1, b + 1)] = sigq(cov, m, g[a], g[b]);
    }
    out.cond = k > 0;
    return TOR_OK;
}

tor_status reduce_pattern(const double *cov, int m, const int8_t *pattern, Reduced &out, bool defer = false) {
    if (!pattern) return fail(TOR_EINVAL, "pattern is NULL");
    std::vector<int> C, N;
    for (int i = 0; i < m; i++) {
        int v = pattern[i];
        if (v == 1) C.push_back(i);
        else if (v == 0) N.push_back(i);
        else if (v != -1) return fail(TOR_EINVAL, "pattern[%d] = %d is not in {-1, 0, 1}", i, v);
    }
    const int n = (int)C.size(), k = (int)N.size();
    if (n > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "%d clicks > %d", n, TOR_MAX_CLICKS);
    out = Reduced();
    out.n = n;
    out.k = k;
    if (k == 0) {
        const int dc = 2 * n;
        out.sig.assign((size_t)dc * dc, dd_from(0.0));
        for (int a = 0; a < dc; a++)
            for (int b = 0; b <= a; b++) {
                dd v = sigq(cov, m, 2 * C[a / 2] + (a & 1), 2 * C[b / 2] + (b & 1));
                out.sig[(size_t)a * dc + b] = v;
                out.sig[(size_t)b * dc + a] = v;
            }
        return TOR_OK;
    }
    if (n + k > TOR_COND_MAX_MODES)
        return fail(TOR_ETOOBIG, "%d observed modes > %d for a pattern with no-click modes", n + k,
                    TOR_COND_MAX_MODES);
    std::vector<int> g;  // quadrature index of each row of the (C, N) matrix
    for (int c : C) {
        g.push_back(2 * c);
        g.push_back(2 * c + 1);
    }
    for (int c : N) {
        g.push_back(2 * c);
        g.push_back(2 * c + 1);
    }
    out.cond = true;
    if (defer) {  // gathered on the device by condition_on_gpu
        out.g = std::move(g);
        return TOR_OK;
    }
    const int d = (int)g.size();
    out.packed.resize((size_t)E(n + k));
    for (int a = 0; a < d; a++)
        for (int b = 0; b <= a; b++) out.packed[(size_t)pidx(a, b)] = sigq(cov, m, g[a], g[b]);
    return TOR_OK;
}

// Words of the matrix a query's conditioning starts from.
size_t cond_words(const Reduced *r) { return r->st ? (size_t)EN(r->n + r->k, r->D) : r->packed.size(); }

// The host packing of a deferred query (its state lives on another device).
void host_pack(Reduced *r) {
    const tor_state *st = r->st;
    const int o = r->D, d = (int)r->g.size();
    r->packed.assign((size_t)EN(r->n + r->k, o), dd_from(0.0));
    for (int a = 0; a < d; a++) {
        if (o) r->packed[(size_t)pidx(a + 1, 0)] = dd_from(st->mean[r->g[a]]);
        for (int b = 0; b <= a; b++)
            r->packed[(size_t)pidx(a + o, b + o)] = sigq(st->cov.data(), st->m, r->g[a], r->g[b]);
    }
    r->st = nullptr;
    std::vector<int>().swap(r->g);
}

// Generation of device data made for states (incremented by every new device
// copy): a persistent kernel's workgroups acquire device memory again when a
// request carries a newer generation than they last acquired.
std::atomic<unsigned int> g_data_gen{1};

// Device copies of a state's covariance (and mean) for the device-side
// gathers, made once; the caller has the state's device current.
tor_status state_on_device(const tor_state *st) {
    tor_state *ms = const_cast<tor_state *>(st);  // the device copies are a cache of the state
    std::lock_guard<std::mutex> lk(ms->dev_mu);
    const size_t cov_bytes = 4 * (size_t)st->m * (size_t)st->m * sizeof(double);
    if (!ms->dcov.p) {
        if (ms->dcov.ensure(cov_bytes) != hipSuccess) return fail(TOR_ENOMEM, "device copy of the state failed");
        HIP_TRY(hipMemcpy(ms->dcov.p, st->cov.data(), cov_bytes, hipMemcpyHostToDevice));
        g_data_gen++;
    }
    if (!st->mean.empty() && !ms->dmean.p) {
        const size_t mb = st->mean.size() * sizeof(double);
        if (ms->dmean.ensure(mb) != hipSuccess) return fail(TOR_ENOMEM, "device copy of the mean failed");
        HIP_TRY(hipMemcpy(ms->dmean.p, st->mean.data(), mb, hipMemcpyHostToDevice));
        g_data_gen++;
    }
    return TOR_OK;
}

// ------------------------------------------------------------------ GPU plan

double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

// One subset sum to evaluate on the GPU: the packed (row-major lower)
// double-double matrix of n modes.
struct SumIn {
    const std::vector<dd> *packed = nullptr;
    int n = 0;
    int D = 0;  // 1: displaced, the mean row first (EN(n, 1) entries); -1: the same
                // layout in the information form (sigma_Q^-1 mu first, exp(+|w|^2 / 2))
};
struct SumOut {
    dd T = {1.0, 0.0};
    double A = 1.0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device bytes one subset sum of n modes needs (pool + descriptors + partials).
// Task size (modes per wave-tier task) for a tree of n modes: the autotuned
// choice for (precision, n) if any, else the context's setting.
int task_modes_for(const tor_ctx *ctx, bool use_dd, int n) {
    int t = (n >= 0 && n <= TOR_MAX_CLICKS) ? ctx->tuned[use_dd ? 1 : 0][n] : 0;
    return std::min(n, t > 0 ? t : ctx->task_modes[use_dd ? 1 : 0]);
}

size_t sum_bytes(int n, int J, size_t es, int D = 0) {
    if (n == 0) return 0;
    D = MR(D);  // mean rows
    J = std::min(n, J);
    const int G = n - J;
    unsigned long long total = (unsigned long long)EN(n, D);
    for (int d = 0; d < G; d++) total += (1ULL << d) * (unsigned long long)EN(n - d - 1, D);
    const size_t nt = (size_t)1 << G;
    return total * es + 2 * nt * sizeof(NodeDesc) + nt * sizeof(Partial) + (nt / 512 + 8) * sizeof(Partial) +
           1024;
}

// Single-launch path (tor_fused.hip): every tree of the group is zero-mean
// with at most TOR_FUSED_MAX_N modes and the group has at most
// TOR_FUSED_MAX_TASKS wave-tier tasks.

bool fused_fits(const tor_ctx *ctx, const std::vector<SumIn> &in, const std::vector<int> &idx, bool use_dd) {
    if (!ctx->fused || idx.empty()) return false;
    long long tasks = 0;
    for (int q : idx) {
        if (in[q].D != 0 || in[q].n < 1 || in[q].n > TOR_FUSED_MAX_N) return false;
        tasks += 1LL << (in[q].n - task_modes_for(ctx, use_dd, in[q].n));
    }
    return tasks <= TOR_FUSED_MAX_TASKS;
}

// Depth-first levels of a unit: about 1024 units (one one-wave workgroup
// each, a task deep) fill the device; the levels beyond are walked depth
// first inside the units.
int fused_levels(int G) { return std::max(0, std::min(TOR_FUSED_TMAX, G - 10)); }

tor_status gpu_group_fused(tor_ctx *ctx, const std::vector<SumIn> &in, const std::vector<int> &idx, bool use_dd,
                           std::vector<SumOut> &out) {
    const size_t es = use_dd ? sizeof(dd) : sizeof(double);
    struct Plan {
        int q, n, J, g, t;
        long long tasks, nblk;
        size_t root_off, part_off, ctr_off;
    };
    std::vector<Plan> P;
    size_t roots = 0, parts = 0, ctrs = 0;
    for (int q : idx) {
        Plan p;
        p.q = q;
        p.n = in[q].n;
        p.J = task_modes_for(ctx, use_dd, p.n);
        const int G = p.n - p.J;
        p.t = fused_levels(G);
        p.g = G - p.t;
        p.tasks = 1LL << G;
        p.nblk = (p.tasks + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
        p.root_off = roots;
        roots += (size_t)EN(p.n, 0);
        p.part_off = parts;
        parts += (size_t)(p.tasks + (p.nblk > 1 ? p.nblk : 0));
        p.ctr_off = ctrs;
        ctrs += (size_t)(1 + p.nblk);
        P.push_back(p);
    }
    // one launch per task size, larger tasks first
    std::vector<size_t> order(P.size());
    for (size_t i = 0; i < P.size(); i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return P[a].J > P[b].J; });
    struct Launch {
        int J;
        size_t first;
        int count;
        long long units;
        long long stride;
    };
    std::vector<Launch> L;
    long long ws_words = 0;
    for (size_t k = 0; k < order.size(); k++) {
        const Plan &p = P[order[k]];
        if (L.empty() || L.back().J != p.J) L.push_back({p.J, k, 0, 0, 0});
        Launch &l = L.back();
        l.count++;
        l.units += 1LL << p.g;
        l.stride = std::max(l.stride, (long long)(1 + p.t) * EN(p.J + p.t, 0));
    }
    for (Launch &l : L) {
        const long long grid = std::min<long long>(l.units, ctx->wave_grid);
        ws_words = std::max(ws_words, grid * l.stride);
    }
    const size_t off_roots = align_up(P.size() * sizeof(FusedJob), 256);
    const size_t up_bytes = off_roots + roots * es;
    const size_t part_bytes = parts * sizeof(Partial);
    if (up_bytes + part_bytes + (size_t)ws_words * es > ctx->mem_budget)
        return fail(TOR_ENOMEM, "subset sums need %.2f GB of device memory (budget %.2f GB)",
                    (up_bytes + part_bytes + (double)ws_words * es) / 1e9, ctx->mem_budget / 1e9);
    const size_t ctr_cap = ctx->fctr.cap;
    if (ctx->jobs.ensure(up_bytes) != hipSuccess || ctx->partA.ensure(part_bytes) != hipSuccess ||
        ctx->pool.ensure((size_t)ws_words * es) != hipSuccess || ctx->fctr.ensure(ctrs * sizeof(unsigned)) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of %.2f MB failed", (up_bytes + part_bytes) / 1e6);
    hipStream_t st = ctx->stream;
    if (ctx->fctr.cap != ctr_cap)  // a new counter buffer starts at zero (the kernel leaves it so)
        HIP_TRY(hipMemsetAsync(ctx->fctr.p, 0, ctx->fctr.cap, st));
    if (ctx->pin_cap < up_bytes) {
        if (ctx->pin_stage) (void)hipHostFree(ctx->pin_stage);
        ctx->pin_stage = nullptr;
        ctx->pin_cap = 0;
        if (hipHostMalloc((void **)&ctx->pin_stage, up_bytes + up_bytes / 8, hipHostMallocDefault) != hipSuccess)
            return fail(TOR_ENOMEM, "pinned allocation failed");
        ctx->pin_cap = up_bytes + up_bytes / 8;
    }
    if (ctx->host_res_cap < P.size()) {
        if (ctx->host_res) (void)hipHostFree(ctx->host_res);
        ctx->host_res = nullptr;
        ctx->host_res_cap = 0;
        if (hipHostMalloc((void **)&ctx->host_res, sizeof(Partial) * P.size(), hipHostMallocDefault) != hipSuccess)
            return fail(TOR_ENOMEM, "pinned allocation failed");
        ctx->host_res_cap = P.size();
    }
    unsigned char *dj = (unsigned char *)ctx->jobs.p;
    long long begin = 0;
    int prevJ = -1;
    for (size_t k = 0; k < order.size(); k++) {
        const size_t i = order[k];
        const Plan &p = P[i];
        if (p.J != prevJ) begin = 0;  // unit indices are flat within a launch
        prevJ = p.J;
        FusedJob job;
        job.root = dj + off_roots + p.root_off * es;
        job.part = (Partial *)ctx->partA.p + p.part_off;
        job.ctr = (unsigned *)ctx->fctr.p + p.ctr_off;
        job.res = ctx->host_res + i;
        job.begin = begin;
        job.n = p.n;
        job.g = p.g;
        job.t = p.t;
        std::memcpy(ctx->pin_stage + k * sizeof(FusedJob), &job, sizeof job);
        begin += 1LL << p.g;
        const std::vector<dd> &pk = *in[p.q].packed;
        unsigned char *dst = ctx->pin_stage + off_roots + p.root_off * es;
        if (use_dd) std::memcpy(dst, pk.data(), (size_t)EN(p.n, 0) * sizeof(dd));
        else
            for (long long e = 0; e < EN(p.n, 0); e++) ((double *)dst)[e] = pk[(size_t)e].hi + pk[(size_t)e].lo;
    }
    HIP_TRY(hipMemcpyAsync(dj, ctx->pin_stage, up_bytes, hipMemcpyHostToDevice, st));
    if (ctx->timing) {
        HIP_TRY(hipEventRecord(ctx->ev[0], st));
        HIP_TRY(hipEventRecord(ctx->ev[1], st));
    }
    for (const Launch &l : L) {
        const int grid = (int)std::min<long long>(l.units, ctx->wave_grid);
        HIP_TRY(tor_launch_fused(use_dd, l.J, (const FusedJob *)dj + l.first, l.count, l.units, ctx->pool.p,
                                 l.stride, grid, st));
    }
    if (ctx->timing) {
        HIP_TRY(hipEventRecord(ctx->ev[2], st));
        HIP_TRY(hipEventRecord(ctx->ev[3], st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (ctx->timing) {
        ctx->stats.wave_ms += elapsed(ctx->ev[1], ctx->ev[2]);
    }
    ctx->stats.wave_launches += (int64_t)L.size();
    ctx->stats.fused_launches += (int64_t)L.size();
    for (size_t i = 0; i < P.size(); i++) {
        SumOut &o = out[P[i].q];
        o.T = dd_make(ctx->host_res[i].t_hi, ctx->host_res[i].t_lo);
        o.A = ctx->host_res[i].a;
        ctx->stats.subsets += std::ldexp(1.0, P[i].n);
    }
    return TOR_OK;
}

// Evaluate a group of subset sums in shared launches.  The top n - J levels of
// every tree are expanded in HBM (one launch per depth, all trees that reach it),
// then one wave-tier launch per distinct J, then the per-tree reduction stages,
// then one gather of the results.  The work and the reduction order of each
// tree do not depend on the other trees in the group.  Every tree of a group
// has the same mean-row offset D.
tor_status gpu_group(tor_ctx *ctx, const std::vector<SumIn> &in, const std::vector<int> &idx, bool use_dd,
                     std::vector<SumOut> &out) {
    if (fused_fits(ctx, in, idx, use_dd)) return gpu_group_fused(ctx, in, idx, use_dd, out);
    const size_t es = use_dd ? sizeof(dd) : sizeof(double);
    const int D = idx.empty() ? 0 : in[idx[0]].D, mrows = MR(D);  // tree kind, mean rows
    struct Plan {
        int q, n, J, G;
        long long nt;
        unsigned long long root_off;
        std::vector<unsigned long long> child_base;
        long long desc_off;
    };
    std::vector<Plan> P;
    unsigned long long roots = 0;
    long long desc_total = 0;
    int Gmax = 0;
    for (int q : idx) {
        Plan p;
        p.q = q;
        p.n = in[q].n;
        p.J = task_modes_for(ctx, use_dd, p.n);
        p.G = p.n - p.J;
        p.nt = 1LL << p.G;
        p.root_off = roots;
        roots += (unsigned long long)EN(p.n, mrows);
        p.desc_off = desc_total;
        desc_total += p.nt;
        Gmax = std::max(Gmax, p.G);
        P.push_back(std::move(p));
    }
    if (P.empty()) return TOR_OK;
    unsigned long long pool_total = roots;
    for (auto &p : P) {
        p.child_base.resize(p.G);
        for (int d = 0; d < p.G; d++) {
            p.child_base[d] = pool_total;
            pool_total += (1ULL << d) * (unsigned long long)EN(p.n - d - 1, mrows);
        }
    }
    // reduction stages: stage outputs laid out one after another in partB
    struct RStage {
        std::vector<ReduceJob> jobs;
        long long blocks = 0;
    };
    std::vector<RStage> stages;
    std::vector<const Partial *> final_src(P.size(), nullptr);
    std::vector<long long> cnt(P.size());
    std::vector<long long> src_off(P.size());  // element offset of the current stage input
    std::vector<int> src_buf(P.size(), 0);       // 0 = partA, 1 = partB
    long long partB_used = 0;
    for (size_t i = 0; i < P.size(); i++) {
        cnt[i] = P[i].nt;
        src_off[i] = P[i].desc_off;
    }
    // sizes first (pointers filled after allocation)
    struct RPlan {
        size_t i;
        long long in_off, out_off, count;
        int in_buf;
    };
    std::vector<std::vector<RPlan>> rplans;
    for (;;) {
        std::vector<RPlan> st;
        for (size_t i = 0; i < P.size(); i++) {
            if (cnt[i] <= 1) continue;
            long long nb = (cnt[i] + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
            st.push_back({i, src_off[i], partB_used, cnt[i], src_buf[i]});
            src_off[i] = partB_used;
            src_buf[i] = 1;
            partB_used += nb;
            cnt[i] = nb;
        }
        if (st.empty()) break;
        rplans.push_back(std::move(st));
    }
    const size_t pool_bytes = pool_total * es;
    const size_t desc_bytes = (size_t)desc_total * sizeof(NodeDesc);
    const size_t partA_bytes = (size_t)desc_total * sizeof(Partial);
    const size_t partB_bytes = (size_t)(partB_used + 1) * sizeof(Partial);
    // job buffer layout
    size_t nexp = 0;
    for (int d = 0; d < Gmax; d++)
        for (auto &p : P)
            if (p.G > d) nexp++;
    size_t nred = 0;
    for (auto &st : rplans) nred += st.size();
    const size_t off_roots = 0;
    const size_t off_exp = align_up(off_roots + P.size() * sizeof(NodeDesc), 64);
    const size_t off_wave = align_up(off_exp + nexp * sizeof(ExpandJob), 64);
    const size_t off_red = align_up(off_wave + P.size() * sizeof(WaveJob), 64);
    const size_t off_gsrc = align_up(off_red + nred * sizeof(ReduceJob), 64);
    const size_t off_res = align_up(off_gsrc + P.size() * sizeof(Partial *), 64);
    const size_t job_bytes = off_res + P.size() * sizeof(Partial);
    if (pool_bytes + 2 * desc_bytes + partA_bytes + partB_bytes + job_bytes > ctx->mem_budget)
        return fail(TOR_ENOMEM, "subset sums need %.2f GB of device memory (budget %.2f GB)",
                    (pool_bytes + 2.0 * desc_bytes + partA_bytes + partB_bytes) / 1e9, ctx->mem_budget / 1e9);
    if (ctx->pool.ensure(pool_bytes) != hipSuccess || ctx->descA.ensure(desc_bytes) != hipSuccess ||
        ctx->descB.ensure(desc_bytes) != hipSuccess || ctx->partA.ensure(partA_bytes) != hipSuccess ||
        ctx->partB.ensure(partB_bytes) != hipSuccess || ctx->jobs.ensure(job_bytes) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of %.2f GB failed", pool_bytes / 1e9);
    if (ctx->host_jobs.size() < job_bytes) ctx->host_jobs.resize(job_bytes);
    unsigned char *hj = ctx->host_jobs.data();
    unsigned char *dj = (unsigned char *)ctx->jobs.p;
    NodeDesc *descA = (NodeDesc *)ctx->descA.p, *descB = (NodeDesc *)ctx->descB.p;
    Partial *partA = (Partial *)ctx->partA.p, *partB = (Partial *)ctx->partB.p;
    auto level_ptr = [&](const Plan &p, size_t pi, int d) -> NodeDesc * {
        if (d == 0) return (NodeDesc *)(dj + off_roots) + pi;
        return ((d & 1) ? descB : descA) + p.desc_off;
    };
    // root descriptors
    for (size_t i = 0; i < P.size(); i++) {
        NodeDesc r{P[i].root_off, 1.0, 0.0, 1.0};
        std::memcpy(hj + off_roots + i * sizeof(NodeDesc), &r, sizeof r);
    }
    // expansion jobs, grouped by depth
    std::vector<std::pair<size_t, int>> exp_launch;  // (first job index, count) per depth
    size_t ej = 0;
    for (int d = 0; d < Gmax; d++) {
        size_t first = ej;
        for (size_t i = 0; i < P.size(); i++) {
            const Plan &p = P[i];
            if (p.G <= d) continue;
            ExpandJob job{level_ptr(p, i, d), level_ptr(p, i, d + 1), p.child_base[d], p.n - d, mrows};
            std::memcpy(hj + off_exp + ej * sizeof(ExpandJob), &job, sizeof job);
            ej++;
        }
        exp_launch.push_back({first, (int)(ej - first)});
    }
    // wave jobs grouped by J (descending J, then query order)
    std::vector<size_t> order(P.size());
    for (size_t i = 0; i < P.size(); i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return P[a].J > P[b].J; });
    struct WGroup {
        int J;
        size_t first;
        int count;
        long long total;
    };
    std::vector<WGroup> wgroups;
    for (size_t k = 0; k < order.size(); k++) {
        const size_t i = order[k];
        const Plan &p = P[i];
        if (wgroups.empty() || wgroups.back().J != p.J) wgroups.push_back({p.J, k, 0, 0});
        WGroup &g = wgroups.back();
        WaveJob job{level_ptr(p, i, p.G), partA + p.desc_off, g.total};
        std::memcpy(hj + off_wave + k * sizeof(WaveJob), &job, sizeof job);
        g.count++;
        g.total += p.nt;
    }
    // reduction jobs
    std::vector<std::pair<size_t, std::pair<int, long long>>> red_launch;
    size_t rj = 0;
    for (auto &st : rplans) {
        size_t first = rj;
        long long blocks = 0;
        for (auto &r : st) {
            ReduceJob job{(r.in_buf ? partB : partA) + r.in_off, partB + r.out_off, r.count, blocks};
            std::memcpy(hj + off_red + rj * sizeof(ReduceJob), &job, sizeof job);
            blocks += (r.count + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
            rj++;
        }
        red_launch.push_back({first, {(int)(rj - first), blocks}});
    }
    // gather sources: the last stage output of each tree
    for (size_t i = 0; i < P.size(); i++) {
        const Partial *src = src_buf[i] ? partB + src_off[i] : partA + src_off[i];
        std::memcpy(hj + off_gsrc + i * sizeof(Partial *), &src, sizeof src);
    }
    // upload the roots and the job tables
    hipStream_t st = ctx->stream;
    std::vector<unsigned char> &stage = ctx->host_stage;
    if (stage.size() < roots * es) stage.resize(roots * es);
    for (auto &p : P) {
        const std::vector<dd> &pk = *in[p.q].packed;
        for (long long e = 0; e < EN(p.n, mrows); e++) {
            if (use_dd) ((dd *)stage.data())[p.root_off + e] = pk[(size_t)e];
            else ((double *)stage.data())[p.root_off + e] = pk[(size_t)e].hi + pk[(size_t)e].lo;
        }
    }
    HIP_TRY(hipMemcpyAsync(ctx->pool.p, stage.data(), roots * es, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dj, hj, off_res, hipMemcpyHostToDevice, st));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[0], st));
    for (int d = 0; d < Gmax; d++) {
        auto [first, count] = exp_launch[d];
        HIP_TRY(tor_launch_expand(use_dd, (const ExpandJob *)(dj + off_exp) + first, count, d, ctx->pool.p, 1 << 20,
                                  st, nullptr, D));
    }
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[1], st));
    for (auto &g : wgroups)
        HIP_TRY(tor_launch_wave(use_dd, g.J, (const WaveJob *)(dj + off_wave) + g.first, g.count, g.total,
                                ctx->pool.p, ctx->wave_grid, st, nullptr, D));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[2], st));
    for (auto &rl : red_launch)
        HIP_TRY(tor_launch_reduce((const ReduceJob *)(dj + off_red) + rl.first, rl.second.first, rl.second.second,
                                  st));
    HIP_TRY(tor_launch_gather((const Partial *const *)(dj + off_gsrc), (int)P.size(), (Partial *)(dj + off_res),
                              st));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[3], st));
    if (ctx->host_res_cap < P.size()) {
        if (ctx->host_res) (void)hipHostFree(ctx->host_res);
        ctx->host_res = nullptr;
        ctx->host_res_cap = 0;
        if (hipHostMalloc((void **)&ctx->host_res, sizeof(Partial) * P.size(), hipHostMallocDefault) != hipSuccess)
            return fail(TOR_ENOMEM, "pinned allocation failed");
        ctx->host_res_cap = P.size();
    }
    HIP_TRY(hipMemcpyAsync(ctx->host_res, dj + off_res, sizeof(Partial) * P.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ctx->timing) {
        ctx->stats.expand_ms += elapsed(ctx->ev[0], ctx->ev[1]);
        ctx->stats.wave_ms += elapsed(ctx->ev[1], ctx->ev[2]);
        ctx->stats.reduce_ms += elapsed(ctx->ev[2], ctx->ev[3]);
    }
    ctx->stats.expand_launches += Gmax;
    ctx->stats.wave_launches += (int64_t)wgroups.size();
    ctx->stats.reduce_launches += (int64_t)red_launch.size() + 1;
    for (size_t i = 0; i < P.size(); i++) {
        SumOut &o = out[P[i].q];
        o.T = dd_make(ctx->host_res[i].t_hi, ctx->host_res[i].t_lo);
        o.A = ctx->host_res[i].a;
        ctx->stats.subsets += std::ldexp(1.0, P[i].n);
    }
    return TOR_OK;
}

// Evaluate subset sums in groups that fit the memory budget.
tor_status gpu_sums(tor_ctx *ctx, const std::vector<SumIn> &in, const std::vector<int> &which, bool use_dd,
                    std::vector<SumOut> &out) {
    const size_t es = use_dd ? sizeof(dd) : sizeof(double);
    bool mixed = false;
    for (int q : which) mixed |= in[q].D != in[which[0]].D;
    if (mixed) {  // zero-mean, displaced and information-form trees go to separate groups
        std::vector<int> w[3];
        for (int q : which) w[in[q].D + 1].push_back(q);
        for (int k = 0; k < 3; k++) {
            tor_status s = gpu_sums(ctx, in, w[k], use_dd, out);
            if (s) return s;
        }
        return TOR_OK;
    }
    std::vector<int> group;
    size_t bytes = 0;
    for (int q : which) {
        if (in[q].n == 0) {
            out[q] = SumOut{};
            continue;
        }
        size_t b = sum_bytes(in[q].n, task_modes_for(ctx, use_dd, in[q].n), es, in[q].D);
        if (!group.empty() && (bytes + b > ctx->mem_budget / 2 || group.size() >= 65536)) {
            tor_status s = gpu_group(ctx, in, group, use_dd, out);
            if (s) return s;
            group.clear();
            bytes = 0;
        }
        group.push_back(q);
        bytes += b;
    }
    return gpu_group(ctx, in, group, use_dd, out);
}

// Run the no-click conditioning of every reduced pattern with r.cond set, all
// of them in shared launches: step t conditions every query with more than t
// no-click modes on its last remaining mode (condition_kernel), so a batch
// takes max |N| launches.  Afterwards r.sig, r.pvac and r.log_pvac hold the
// conditioned matrix and the vacuum probability of N; r.cond is cleared.
tor_status condition_on_gpu(tor_ctx *ctx, const std::vector<Reduced *> &all) {
    std::vector<Reduced *> rs;
    for (Reduced *r : all)
        if (r->cond) rs.push_back(r);
    // queries of a state are gathered on the device from its device copy
    for (Reduced *r : rs) {
        if (!r->st) continue;
        if (r->st->device != ctx->device) {
            host_pack(r);
            continue;
        }
        tor_status s = state_on_device(r->st);
        if (s) return s;
    }
    size_t first = 0;
    while (first < rs.size()) {
        // a group that fits half the memory budget (at least one query)
        size_t last = first, bytes = 0;
        while (last < rs.size()) {
            const Reduced *rl = rs[last];
            size_t b = cond_words(rl) * sizeof(dd) + 64;
            if (ctx->cond_block > 1)  // the block's scaled pivot columns
                b += 2 * (size_t)ctx->cond_block * (size_t)(2 * (rl->n + rl->k) + rl->D) * sizeof(dd);
            if (last > first && bytes + b > ctx->mem_budget / 2) break;
            bytes += b;
            last++;
        }
        const size_t nq = last - first;
        std::vector<size_t> off(nq);
        size_t tot = 0, gtot = 0;
        int kmax = 0;
        std::vector<GatherJob> gjobs;
        long long gentries = 0;
        for (size_t i = 0; i < nq; i++) {
            const Reduced *r = rs[first + i];
            off[i] = tot;
            tot += cond_words(r);
            kmax = std::max(kmax, r->k);
            if (r->st) {
                GatherJob gj{};
                gj.begin = gentries;
                gj.m = r->st->m;
                gj.R = (int)r->g.size();
                gentries += (long long)cond_words(r);
                gjobs.push_back(gj);
                gtot += r->g.size();
            }
        }
        // jobs of every step (or block of steps), in step order
        const int CB = ctx->cond_block;
        std::vector<CondJob> jobs;
        std::vector<CondBlockJob> bjobs;
        struct Step {
            size_t first;
            int count;
            long long blocks, blocks2;  // the launch's workgroups (blocked: panel, bulk)
            int rmax;
        };
        std::vector<Step> steps;
        // blocked: each query's scaled pivot columns of a block, 2 CB rows of
        // ld = its row count, after the matrices
        std::vector<size_t> voff(nq);
        size_t vtot = 0;
        if (CB > 1)
            for (size_t i = 0; i < nq; i++) {
                voff[i] = tot + vtot;
                vtot += 2 * (size_t)CB * (size_t)(2 * (rs[first + i]->n + rs[first + i]->k) + rs[first + i]->D);
            }
        // device layout: the matrices (and columns), then [accumulators | step
        // jobs | gather jobs | gather rows], the latter staged from the host in
        // one copy
        const size_t acc_off = align_up((tot + vtot) * sizeof(dd), 256);
        const size_t job_off = align_up(acc_off + nq * 3 * sizeof(double), 256);
        if (CB <= 1) {
            for (int t = 0; t < kmax; t++) {
                Step st{jobs.size(), 0, 0, 0, 1};
                for (size_t i = 0; i < nq; i++) {
                    const Reduced *r = rs[first + i];
                    if (r->k <= t) continue;
                    CondJob j{};
                    j.r = r->n + r->k - t;
                    j.d = r->D;
                    j.begin = st.blocks;
                    jobs.push_back(j);
                    st.blocks += std::max<long long>(1, (EN(j.r - 1, j.d) + TOR_COND_CHUNK - 1) / TOR_COND_CHUNK);
                    st.count++;
                    st.rmax = std::max(st.rmax, j.r);
                }
                steps.push_back(st);
            }
        } else {
            for (int t0 = 0; t0 < kmax; t0 += CB) {
                Step st{bjobs.size(), 0, 0, 0, 1};
                // every panel workgroup takes the block's steps before its
                // columns: a launch of many queries gives each workgroup
                // several column groups, so that about kPanelWorkgroups run
                long long one = 0;
                for (size_t i = 0; i < nq; i++) {
                    const Reduced *r = rs[first + i];
                    if (r->k > t0) one += cond_panel_blocks(r->n + r->k - t0, std::min(CB, r->k - t0), r->D, 1);
                }
                const int passes = (int)std::max(1LL, (one + kPanelWorkgroups - 1) / kPanelWorkgroups);
                for (size_t i = 0; i < nq; i++) {
                    const Reduced *r = rs[first + i];
                    if (r->k <= t0) continue;
                    CondBlockJob j{};
                    j.r = r->n + r->k - t0;
                    j.b = std::min(CB, r->k - t0);
                    j.d = r->D;
                    j.ld = 2 * (r->n + r->k) + r->D;
                    j.passes = passes;
                    j.begin_panel = st.blocks;
                    j.begin_bulk = st.blocks2;
                    bjobs.push_back(j);
                    st.blocks += cond_panel_blocks(j.r, j.b, j.d, passes);
                    st.blocks2 += cond_bulk_blocks(j.r, j.b, j.d);
                    st.count++;
                }
                steps.push_back(st);
            }
        }
        const size_t job_bytes = CB <= 1 ? jobs.size() * sizeof(CondJob) : bjobs.size() * sizeof(CondBlockJob);
        const size_t gjob_off = align_up(job_off + job_bytes, 256);
        const size_t gidx_off = align_up(gjob_off + gjobs.size() * sizeof(GatherJob), 256);
        const size_t total_bytes = gidx_off + gtot * sizeof(int);
        if (total_bytes > ctx->mem_budget)
            return fail(TOR_ENOMEM, "conditioning needs %.2f GB of device memory", total_bytes / 1e9);
        if (ctx->cond.ensure(total_bytes) != hipSuccess)
            return fail(TOR_ENOMEM, "device allocation of %.2f GB failed", total_bytes / 1e9);
        unsigned char *dbase = (unsigned char *)ctx->cond.p;
        dd *dmat = (dd *)dbase;
        double *dacc = (double *)(dbase + acc_off);
        // job pointers (device addresses)
        size_t ji = 0;
        if (CB <= 1) {
            for (int t = 0; t < kmax; t++)
                for (size_t i = 0; i < nq; i++) {
                    const Reduced *r = rs[first + i];
                    if (r->k <= t) continue;
                    jobs[ji].mat = dmat + off[i];
                    jobs[ji].acc = dacc + 3 * i;
                    jobs[ji].qout = nullptr;
                    ji++;
                }
        } else {
            for (int t0 = 0; t0 < kmax; t0 += CB)
                for (size_t i = 0; i < nq; i++) {
                    const Reduced *r = rs[first + i];
                    if (r->k <= t0) continue;
                    bjobs[ji].mat = dmat + off[i];
                    bjobs[ji].V = dmat + voff[i];
                    bjobs[ji].acc = dacc + 3 * i;
                    ji++;
                }
        }
        // the staged tail: accumulators, step jobs, gather jobs and rows
        std::vector<unsigned char> &stage = ctx->host_stage;
        const size_t tail = total_bytes - acc_off;
        if (stage.size() < tail) stage.resize(tail);
        auto at = [&](size_t dev_off) { return stage.data() + (dev_off - acc_off); };  // staged byte
        for (size_t i = 0; i < nq; i++) {
            const double a0[3] = {1.0, 0.0, 0.0};
            std::memcpy(at(acc_off) + i * 3 * sizeof(double), a0, sizeof a0);
        }
        if (CB <= 1) std::memcpy(at(job_off), jobs.data(), job_bytes);
        else std::memcpy(at(job_off), bjobs.data(), job_bytes);
        {
            size_t gi = 0, gw = 0;
            int *gidx = (int *)at(gidx_off);
            for (size_t i = 0; i < nq; i++) {
                const Reduced *r = rs[first + i];
                if (!r->st) continue;
                GatherJob &gj = gjobs[gi++];
                gj.cov = (const double *)r->st->dcov.p;
                gj.mean = r->D ? (const double *)r->st->dmean.p : nullptr;
                gj.g = (const int *)(dbase + gidx_off) + gw;
                gj.out = dmat + off[i];
                std::memcpy(gidx + gw, r->g.data(), r->g.size() * sizeof(int));
                gw += r->g.size();
            }
            std::memcpy(at(gjob_off), gjobs.data(), gjobs.size() * sizeof(GatherJob));
        }
        hipStream_t st = ctx->stream;
        for (size_t i = 0; i < nq; i++)  // host-packed matrices
            if (!rs[first + i]->st)
                HIP_TRY(hipMemcpyAsync(dmat + off[i], rs[first + i]->packed.data(),
                                       rs[first + i]->packed.size() * sizeof(dd), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dbase + acc_off, stage.data(), tail, hipMemcpyHostToDevice, st));
        HIP_TRY(tor_launch_cond_gather((const GatherJob *)(dbase + gjob_off), (int)gjobs.size(), gentries, st));
        if (CB <= 1) {
            const CondJob *djobs = (const CondJob *)(dbase + job_off);
            for (const Step &sp : steps)
                HIP_TRY(tor_launch_condition(djobs + sp.first, sp.count, sp.blocks, sp.rmax, st));
        } else {
            const CondBlockJob *djobs = (const CondBlockJob *)(dbase + job_off);
            for (const Step &sp : steps) {
                HIP_TRY(tor_launch_cond_panel(djobs + sp.first, sp.count, sp.blocks, st));
                HIP_TRY(tor_launch_cond_bulk(djobs + sp.first, sp.count, sp.blocks2, st));
            }
        }
        // results: the leading block of each matrix and the accumulators
        std::vector<std::vector<dd>> lead(nq);
        for (size_t i = 0; i < nq; i++) {
            const Reduced *r = rs[first + i];
            lead[i].resize((size_t)EN(r->n, r->D));
            if (!lead[i].empty())
                HIP_TRY(hipMemcpyAsync(lead[i].data(), dmat + off[i], lead[i].size() * sizeof(dd),
                                       hipMemcpyDeviceToHost, st));
        }
        std::vector<double> accs(3 * nq);
        HIP_TRY(hipMemcpyAsync(accs.data(), dacc, accs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        ctx->stats.condition_launches += (int64_t)steps.size() * (CB <= 1 ? 1 : 2);
        for (size_t i = 0; i < nq; i++) {
            Reduced *r = rs[first + i];
            const dd *pk = lead[i].data();
            const double *acc = accs.data() + 3 * i;
            r->pvac = dd_make(acc[0], acc[1]);
            r->log_pvac = acc[2];
            r->cond_u = r->k * kUDD;  // k double-double conditioning steps
            r->cond = false;
            r->st = nullptr;
            std::vector<int>().swap(r->g);
            if (r->D) {  // keep the packed form: the leading block with its mean row
                r->packed.swap(lead[i]);
                continue;
            }
            const int dc = 2 * r->n;
            r->sig.assign((size_t)dc * dc, dd_from(0.0));
            for (int a = 0; a < dc; a++)
                for (int b = 0; b <= a; b++) {
                    r->sig[(size_t)a * dc + b] = pk[pidx(a, b)];
                    r->sig[(size_t)b * dc + a] = pk[pidx(a, b)];
                }
            std::vector<dd>().swap(r->packed);
        }
        first = last;
    }
    return TOR_OK;
}

void pack_lower(const std::vector<dd> &full, int n, std::vector<dd> &packed) {
    const int d = 2 * n;
    packed.assign((size_t)E(n), dd_from(0.0));
    for (int a = 0; a < d; a++)
        for (int b = 0; b <= a; b++) packed[(size_t)pidx(a, b)] = full[(size_t)a * d + b];
}

// A query reduced to its conditioned matrix, ready for the GPU.
struct Prepared {
    std::vector<dd> packed;
    int n = 0;
    int D = 0;            // 1: displaced (packed has the mean row first)
    double quad = 0.0;    // displaced: mu_C^T Sigma_C^-1 mu_C of the conditioned mean
    dd pvac = {1.0, 0.0};
    double log_pvac = 0.0;
    double log_det = 0.0;
    bool scaled = false;  // the tree sums G = Sigma_C^-1: multiply its (T, A) by tscale
    dd tscale = {1.0, 0.0};
    dd pdirect = {1.0, 0.0};  // scaled: p = pdirect T(G)
    double cond_u = 0.0;      // as Reduced::cond_u
    tor_status status = TOR_OK;
    std::string err;
};

// PD check and log det of Sigma_C on the host; packs Sigma_C.
// PD check and log det of Sigma_C by a binary64 Cholesky (log det only feeds
// the reported Torontonian; the subset tree itself stops with a non-positive
// pivot on the GPU as well).
bool f64_cholesky_logdet(const std::vector<dd> &A, int d, double *log_det, std::vector<double> *Lout = nullptr) {
    std::vector<double> L((size_t)d * d);
    double ld = 0.0;
    for (int j = 0; j < d; j++) {
        double s = A[(size_t)j * d + j].hi + A[(size_t)j * d + j].lo;
        for (int t = 0; t < j; t++) s -= L[(size_t)j * d + t] * L[(size_t)j * d + t];
        if (!(s > 0.0)) return false;
        const double l = std::sqrt(s);
        L[(size_t)j * d + j] = l;
        ld += std::log(s);
        for (int i = j + 1; i < d; i++) {
            double v = A[(size_t)i * d + j].hi + A[(size_t)i * d + j].lo;
            for (int t = 0; t < j; t++) v -= L[(size_t)i * d + t] * L[(size_t)j * d + t];
            L[(size_t)i * d + j] = v / l;
        }
    }
    *log_det = ld;
    if (Lout) Lout->swap(L);
    return true;
}

tor_status prepare(const std::vector<dd> &sig, int n, dd pvac, double log_pvac, Prepared &p) {
    p.n = n;
    p.pvac = pvac;
    p.log_pvac = log_pvac;
    if (n > 0 && !f64_cholesky_logdet(sig, 2 * n, &p.log_det))
        return fail(TOR_ENOTPD, "Sigma_C is not positive definite");
    pack_lower(sig, n, p.packed);
    return TOR_OK;
}

// A-priori relative error bound of a subset sum, first order in the unit
// roundoffs: every term det(Sigma_C[Y])^-1/2 is a product of at most n pivot
// factors, each the result of a few rounded operations on Schur complements,
// so its relative error is a small multiple of n u (u of the term precision);
// the elimination steps that formed Sigma_C from sigma_Q (k no-click
// conditioning steps of Eq. MatrixUpdate, or the m sweeps of a state's
// inverse) are each backward stable, the exact step of a matrix perturbed by a
// few u_c relative to sigma_Q >= I/2, and those perturbations add up over the
// steps, moving every term by a small multiple of k u_c more (cond_u = k u_c).
// Errors of the terms add up to R = sum|t| / |T| times the relative error of
// the largest terms; the constant 16 covers the per-step constants.
// Displaced states: every term also carries exp(-x/2), x <= quad (the largest
// exponent of any term: the quadratic form of a principal block's inverse is
// at most that of the whole matrix); the rounding of x enters the term's
// relative error in proportion to x, hence the factor (1 + quad).
double bound_of(int used, int n, dd T, double A, double quad = 0.0, double cond_u = 0.0) {
    double R = A / std::fabs(T.hi);
    const double u = used == TOR_PREC_QD ? kUQD : used == TOR_PREC_DD ? kUDD : kUF64;
    return kBoundC * (std::max(n, 1) * u + cond_u) * R * (1.0 + quad);
}

// mu^T Sigma^-1 mu of an n-mode packed matrix with its mean row first
// (binary64 Cholesky of the covariance block; 0 for D = 0 or n = 0, +inf if
// the block is not positive definite).
double quad_of(const std::vector<dd> &packed, int n, int D) {
    if (!D || n == 0) return 0.0;
    const int d = 2 * n;
    std::vector<double> L((size_t)d * d, 0.0), z(d);
    double quad = 0.0;
    for (int j = 0; j < d; j++) {
        const dd djj = packed[(size_t)pidx(j + 1, j + 1)];
        double sjj = djj.hi + djj.lo;
        for (int t = 0; t < j; t++) sjj -= L[(size_t)j * d + t] * L[(size_t)j * d + t];
        if (!(sjj > 0.0)) return INFINITY;
        const double l = std::sqrt(sjj);
        L[(size_t)j * d + j] = l;
        for (int i = j + 1; i < d; i++) {
            const dd dij = packed[(size_t)pidx(i + 1, j + 1)];
            double v = dij.hi + dij.lo;
            for (int t = 0; t < j; t++) v -= L[(size_t)i * d + t] * L[(size_t)j * d + t];
            L[(size_t)i * d + j] = v / l;
        }
        const dd mu = packed[(size_t)pidx(j + 1, 0)];
        double v = mu.hi + mu.lo;
        for (int t = 0; t < j; t++) v -= L[(size_t)j * d + t] * z[t];
        z[j] = v / l;
        quad += z[j] * z[j];
    }
    return quad;
}

// Displaced state: `packed` is the conditioned matrix with its mean row
// (EN(n, 1) entries).  PD check, log det Sigma_C and mu_C^T Sigma_C^-1 mu_C by
// a binary64 Cholesky of the covariance block.
tor_status prepare_disp(std::vector<dd> &&packed, int n, dd pvac, double log_pvac, Prepared &p) {
    p.n = n;
    p.D = 1;
    p.pvac = pvac;
    p.log_pvac = log_pvac;
    const int d = 2 * n;
    if (n > 0) {
        std::vector<dd> sig((size_t)d * d);
        for (int a = 0; a < d; a++)
            for (int b = 0; b <= a; b++) {
                sig[(size_t)a * d + b] = packed[(size_t)pidx(a + 1, b + 1)];
                sig[(size_t)b * d + a] = packed[(size_t)pidx(a + 1, b + 1)];
            }
        std::vector<double> L;
        if (!f64_cholesky_logdet(sig, d, &p.log_det, &L)) return fail(TOR_ENOTPD, "Sigma_C is not positive definite");
        std::vector<double> z(d);
        double quad = 0.0;
        for (int a = 0; a < d; a++) {
            const dd mu = packed[(size_t)pidx(a + 1, 0)];
            double v = mu.hi + mu.lo;
            for (int t = 0; t < a; t++) v -= L[(size_t)a * d + t] * z[t];
            z[a] = v / L[(size_t)a * d + a];
            quad += z[a] * z[a];
        }
        p.quad = quad;
    }
    p.packed = std::move(packed);
    return TOR_OK;
}

// Every mode observed (1 or 0) and at least one no-click mode.
bool is_full_pattern(const int8_t *pattern, int m) {
    bool zero = false;
    for (int i = 0; i < m; i++) {
        if (pattern[i] == 0) zero = true;
        else if (pattern[i] != 1) return false;
    }
    return zero;
}

// A full pattern on an inverted state (Jacobi's complementary-minor identity,
// det sigma_Q[S] = det sigma_Q det K[S^c] with K = sigma_Q^-1): Sigma_C =
// G^-1 with G = K[C], so every term of the subset sum of Sigma_C is
// det(G)^1/2 times a term of the subset sum of G with the complementary set,
// T(Sigma_C) = (-1)^n det(G)^1/2 T(G), and P_vac(N) = (det sigma_Q det G)^-1/2.
// G is gathered in double-double (the quad-double inverse rounded when the
// state holds that one); det(G)^(+-1/2) from its double-double Cholesky.
tor_status reduce_pattern_jacobi_disp(const tor_state *st, const int8_t *pattern, Reduced &out);

// Elimination error carried by G = K[C] gathered from a state's inverse: the
// m sweeps that formed K (unit roundoff of the inverse's words), plus one
// rounding of a quad-double inverse to the double-double words of the tree.
double inverse_cond_u(const tor_state *st) {
    return st->inv_prec == TOR_PREC_QD ? st->m * kUQD + kUDD : st->m * kUDD;
}

tor_status reduce_pattern_jacobi(const tor_state *st, const int8_t *pattern, Reduced &out) {
    if (!st->mean.empty()) return reduce_pattern_jacobi_disp(st, pattern, out);
    std::vector<int> C;
    for (int i = 0; i < st->m; i++)
        if (pattern[i] == 1) C.push_back(i);
    const int n = (int)C.size();
    if (n > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "%d clicks > %d", n, TOR_MAX_CLICKS);
    out = Reduced();
    out.n = n;
    out.k = st->m - n;
    out.jacobi = true;
    const int dc = 2 * n;
    out.sig.assign((size_t)dc * dc, dd_from(0.0));
    for (int a = 0; a < dc; a++)
        for (int b = 0; b <= a; b++) {  // C ascending: global row >= global column
            const size_t e = (size_t)pidx(2 * C[a / 2] + (a & 1), 2 * C[b / 2] + (b & 1));
            const dd v = st->inv_prec == TOR_PREC_QD ? qd_to_dd(st->inv_q[e]) : st->inv[e];
            out.sig[(size_t)a * dc + b] = v;
            out.sig[(size_t)b * dc + a] = v;
        }
    dd root = dd_from(1.0), rroot = dd_from(1.0);  // det(G)^1/2, det(G)^-1/2
    double log_det_g = 0.0;
    if (n > 0) {
        std::vector<dd> L = out.sig, rinv;
        if (!dd_cholesky(L, dc, rinv, &log_det_g)) return fail(TOR_ENOTPD, "sigma_Q^-1 over C is not positive definite");
        for (int j = 0; j < dc; j++) {
            root = dd_mul(root, L[(size_t)j * dc + j]);
            rroot = dd_mul(rroot, rinv[j]);
        }
    }
    out.pvac = dd_mul(st->det_rsqrt, rroot);
    out.log_pvac = -0.5 * (st->log_det_sigq + log_det_g);
    out.cond_u = inverse_cond_u(st);
    out.tscale = (n & 1) ? dd_neg(root) : root;
    out.pdirect = (n & 1) ? dd_neg(st->det_rsqrt) : st->det_rsqrt;
    return TOR_OK;
}

// A full pattern of an inverted displaced state.  With h = K mu, the vacuum
// probability of S = Y + N (complement Z = C \ Y) is
//   det(sigma_Q)^-1/2 exp(-mu^T K mu / 2) det(G[Z])^-1/2 exp(+h_Z^T G[Z]^-1 h_Z / 2)
// (mu_S^T sigma_Q[S]^-1 mu_S = mu^T K mu - h_Z^T K[Z]^-1 h_Z), so p is
// (-1)^n det(sigma_Q)^-1/2 exp(-mu^T K mu / 2) times the information-form
// subset sum of [0, h_C; h_C, G] (tree kind -1).  The reported sum of Sigma_C
// with its conditioned mean is that sum times (-1)^n det(G)^1/2
// exp(-h_C^T G^-1 h_C / 2), and P_vac(N) = det(sigma_Q)^-1/2 det(G)^-1/2
// exp(-mu^T K mu / 2) exp(+h_C^T G^-1 h_C / 2); h_C^T G^-1 h_C from the
// double-double Cholesky of G.
tor_status reduce_pattern_jacobi_disp(const tor_state *st, const int8_t *pattern, Reduced &out) {
    std::vector<int> C;
    for (int i = 0; i < st->m; i++)
        if (pattern[i] == 1) C.push_back(i);
    const int n = (int)C.size();
    if (n > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "%d clicks > %d", n, TOR_MAX_CLICKS);
    out = Reduced();
    out.n = n;
    out.k = st->m - n;
    out.D = 1;
    out.jacobi = true;
    const int dc = 2 * n;
    std::vector<int> g(dc);
    for (int a = 0; a < dc; a++) g[a] = 2 * C[a / 2] + (a & 1);
    out.packed.assign((size_t)EN(n, 1), dd_from(0.0));
    std::vector<dd> G((size_t)dc * dc);
    for (int a = 0; a < dc; a++) {
        out.packed[(size_t)pidx(a + 1, 0)] = st->inv_h[g[a]];
        for (int b = 0; b <= a; b++) {
            const size_t e = (size_t)pidx(g[a], g[b]);
            const dd v = st->inv_prec == TOR_PREC_QD ? qd_to_dd(st->inv_q[e]) : st->inv[e];
            out.packed[(size_t)pidx(a + 1, b + 1)] = v;
            G[(size_t)a * dc + b] = v;
            G[(size_t)b * dc + a] = v;
        }
    }
    dd root = dd_from(1.0), rroot = dd_from(1.0), q = dd_from(0.0);  // det(G)^(+-1/2), h_C^T G^-1 h_C
    double log_det_g = 0.0;
    if (n > 0) {
        std::vector<dd> rinv;
        if (!dd_cholesky(G, dc, rinv, &log_det_g))
            return fail(TOR_ENOTPD, "sigma_Q^-1 over C is not positive definite");
        std::vector<dd> z(dc);
        for (int a = 0; a < dc; a++) {
            root = dd_mul(root, G[(size_t)a * dc + a]);
            rroot = dd_mul(rroot, rinv[a]);
            dd v = st->inv_h[g[a]];
            for (int t = 0; t < a; t++) v = dd_sub(v, dd_mul(G[(size_t)a * dc + t], z[t]));
            z[a] = dd_mul(v, rinv[a]);
            q = dd_add(q, dd_mul(z[a], z[a]));
        }
    }
    const dd half_q = dd_make(0.5 * q.hi, 0.5 * q.lo);
    out.cond_u = inverse_cond_u(st);
    out.pvac = dd_mul(dd_mul(st->det_rsqrt_mean, rroot), dd_exp(half_q));
    out.log_pvac = -0.5 * (st->log_det_sigq + log_det_g) - 0.5 * (st->mu_k_mu.hi + st->mu_k_mu.lo) +
                   (half_q.hi + half_q.lo);
    const dd ts = dd_mul(root, dd_exp(dd_neg(half_q)));
    out.tscale = (n & 1) ? dd_neg(ts) : ts;
    out.pdirect = (n & 1) ? dd_neg(st->det_rsqrt_mean) : st->det_rsqrt_mean;
    return TOR_OK;
}

// A pattern of a state (zero-mean or displaced) reduced for the subset tree.
// Full patterns on an inverted zero-mean state take the complementary-minor
// route (no conditioning); the quad-double inverse also serves binary64 and
// double-double terms.
tor_status reduce_for_state(const tor_state *st, const int8_t *pattern, Reduced &out) {
    if (!pattern) return fail(TOR_EINVAL, "pattern is NULL");
    if (st->inv_prec && is_full_pattern(pattern, st->m)) return reduce_pattern_jacobi(st, pattern, out);
    tor_status s;
    if (!st->mean.empty()) s = reduce_pattern_disp(st->cov.data(), st->mean.data(), st->m, pattern, out, true);
    else s = reduce_pattern(st->cov.data(), st->m, pattern, out, true);
    if (s == TOR_OK && out.cond) out.st = st;  // gathered on the device from the state's copy
    return s;
}

// A reduced pattern, conditioned if it had no-click modes, made ready for the GPU.
tor_status prepare_reduced(Reduced &r, Prepared &p) {
    p.cond_u = r.cond_u;
    if (r.D) {
        tor_status s = prepare_disp(std::move(r.packed), r.n, r.pvac, r.log_pvac, p);
        if (s == TOR_OK && r.jacobi) {  // [0, h_C; h_C, G]: the information-form tree
            p.D = -1;                   // quad = h_C^T G^-1 h_C bounds its exponents
            p.log_det = -p.log_det;
            p.scaled = true;
            p.tscale = r.tscale;
            p.pdirect = r.pdirect;
        }
        return s;
    }
    tor_status s = prepare(r.sig, r.n, r.pvac, r.log_pvac, p);
    if (s == TOR_OK && r.jacobi) {  // prepare saw G: log det Sigma_C = -log det G
        p.log_det = -p.log_det;
        p.scaled = true;
        p.tscale = r.tscale;
        p.pdirect = r.pdirect;
    }
    return s;
}

void finalize(const Prepared &p, const SumOut &s, int used, double tol, tor_result *out) {
    const dd T = p.scaled ? dd_mul(p.tscale, s.T) : s.T;
    const double A = p.scaled ? std::fabs(p.tscale.hi) * s.A : s.A;
    // p = P_vac(N) T(Sigma_C); for the sum of G it is formed directly as
    // (-1)^n det(sigma_Q)^-1/2 T(G)
    dd pr = p.scaled ? dd_mul(p.pdirect, s.T) : dd_mul(p.pvac, T);
    std::memset(out, 0, sizeof *out);
    out->p = pr.hi + pr.lo;
    out->p_lo = pr.lo - (out->p - pr.hi);
    out->log_p = out->p > 0 ? p.log_pvac + std::log(T.hi) + std::log1p(T.lo / T.hi) : -INFINITY;
    out->T = T.hi;
    out->T_lo = T.lo;
    out->tor = std::exp(0.5 * p.log_det) * (T.hi + T.lo);
    out->abs_sum = A;
    out->cancel_ratio = A / std::fabs(T.hi);
    out->rel_err_bound = bound_of(used, p.n, T, A, p.quad, p.cond_u);
    out->log_pvac_n = p.log_pvac;
    out->n_clicks = p.n;
    out->prec_used = used;
    out->status = out->rel_err_bound <= tol ? TOR_OK : TOR_WARN_PRECISION;
}

// ------------------------------------------------------------------ quad-double tier

// Subset sum of one packed n-mode matrix in quad-double: the top n - J levels
// expanded in HBM (slots [coefficient][matrix]), J = min(n, 8)-mode wave
// tasks, fixed-order reduction stages, one result.
tor_status gpu_sum_qd(tor_ctx *ctx, const std::vector<qd> &packed, int n, SumOut &out, int D = 0) {
    if (n == 0) {
        out = SumOut{};
        return TOR_OK;
    }
    // displaced trees: seven-mode tasks (the eight-mode working set with the
    // mean row needs 56 KB of LDS, two workgroups per CU)
    const int J = std::min(n, D ? TOR_QD_TASK_MAX - 1 : TOR_QD_TASK_MAX), G = n - J;
    const int mrows = MR(D);  // D = -1 (information form) has the displaced layout
    const long long nt = 1LL << G;
    const size_t es = sizeof(qd);
    // pool: root slot, then per level 2^d child slots of EN(n - d - 1, MR(D)) + 1 words
    std::vector<unsigned long long> child_base(G);
    unsigned long long words = 1 + (unsigned long long)EN(n, mrows);
    for (int d = 0; d < G; d++) {
        child_base[d] = words;
        words += (1ULL << d) * (unsigned long long)(EN(n - d - 1, mrows) + 1);
    }
    // reduction stages over partials (stage outputs one after another in partB)
    std::vector<ReduceJobQ> red;
    std::vector<long long> red_blocks;
    long long cnt = nt, partB_used = 0;
    bool in_b = false;
    long long in_off = 0;
    struct RS {
        bool in_b;
        long long in_off, out_off, count;
    };
    std::vector<RS> rs;
    while (cnt > 1) {
        const long long nb = (cnt + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
        rs.push_back({in_b, in_off, partB_used, cnt});
        in_b = true;
        in_off = partB_used;
        partB_used += nb;
        cnt = nb;
    }
    const size_t pool_bytes = words * es;
    const size_t desc_bytes = (size_t)nt * sizeof(NodeDesc);
    const size_t partA_bytes = (size_t)nt * sizeof(PartialQ);
    const size_t partB_bytes = (size_t)(partB_used + 1) * sizeof(PartialQ);
    const size_t off_root = 0;
    const size_t off_exp = align_up(sizeof(NodeDesc), 64);
    const size_t off_wave = align_up(off_exp + G * sizeof(ExpandJob), 64);
    const size_t off_red = align_up(off_wave + sizeof(WaveJob), 64);
    const size_t job_bytes = off_red + rs.size() * sizeof(ReduceJobQ);
    if (pool_bytes + 2 * desc_bytes + partA_bytes + partB_bytes + job_bytes > ctx->mem_budget)
        return fail(TOR_ENOMEM, "a quad-double subset sum of %d modes needs %.2f GB of device memory (budget %.2f GB)",
                    n, (pool_bytes + 2.0 * desc_bytes + partA_bytes + partB_bytes) / 1e9, ctx->mem_budget / 1e9);
    if (ctx->pool.ensure(pool_bytes) != hipSuccess || ctx->descA.ensure(desc_bytes) != hipSuccess ||
        ctx->descB.ensure(desc_bytes) != hipSuccess || ctx->partA.ensure(partA_bytes) != hipSuccess ||
        ctx->partB.ensure(partB_bytes) != hipSuccess || ctx->jobs.ensure(job_bytes) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of %.2f GB failed", pool_bytes / 1e9);
    unsigned char *dj = (unsigned char *)ctx->jobs.p;
    NodeDesc *descA = (NodeDesc *)ctx->descA.p, *descB = (NodeDesc *)ctx->descB.p;
    PartialQ *partA = (PartialQ *)ctx->partA.p, *partB = (PartialQ *)ctx->partB.p;
    auto level_ptr = [&](int d) -> NodeDesc * {
        if (d == 0) return (NodeDesc *)(dj + off_root);
        return (d & 1) ? descB : descA;
    };
    std::vector<unsigned char> hj(job_bytes);
    const NodeDesc root{1, 1.0, 0.0, 1.0};  // the matrix starts after the coefficient word
    std::memcpy(hj.data() + off_root, &root, sizeof root);
    for (int d = 0; d < G; d++) {
        ExpandJob job{level_ptr(d), level_ptr(d + 1), child_base[d], n - d, mrows};
        std::memcpy(hj.data() + off_exp + d * sizeof(ExpandJob), &job, sizeof job);
    }
    const WaveJob wj{level_ptr(G), (Partial *)partA, 0};
    std::memcpy(hj.data() + off_wave, &wj, sizeof wj);
    for (size_t k = 0; k < rs.size(); k++) {
        ReduceJobQ job{(rs[k].in_b ? partB : partA) + rs[k].in_off, partB + rs[k].out_off, rs[k].count, 0};
        std::memcpy(hj.data() + off_red + k * sizeof(ReduceJobQ), &job, sizeof job);
    }
    // root slot: coefficient 1, then the matrix
    std::vector<qd> root_words(1 + (size_t)EN(n, mrows));
    root_words[0] = qd_from(1.0);
    for (long long e = 0; e < EN(n, mrows); e++) root_words[1 + (size_t)e] = packed[(size_t)e];
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemcpyAsync(ctx->pool.p, root_words.data(), root_words.size() * es, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dj, hj.data(), job_bytes, hipMemcpyHostToDevice, st));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[0], st));
    for (int d = 0; d < G; d++)
        HIP_TRY(tor_launch_expand_qd((const ExpandJob *)(dj + off_exp) + d, 1, d, ctx->pool.p, 1 << 20, st, D));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[1], st));
    HIP_TRY(tor_launch_wave_qd(J, (const WaveJob *)(dj + off_wave), 1, nt, ctx->pool.p, ctx->wave_grid, st, D));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[2], st));
    for (size_t k = 0; k < rs.size(); k++)
        HIP_TRY(tor_launch_reduce_qd((const ReduceJobQ *)(dj + off_red) + k, 1,
                                     (rs[k].count + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK, st));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev[3], st));
    PartialQ res;
    const PartialQ *src = rs.empty() ? partA : partB + (partB_used - 1);
    HIP_TRY(hipMemcpyAsync(&res, src, sizeof res, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ctx->timing) {
        ctx->stats.expand_ms += elapsed(ctx->ev[0], ctx->ev[1]);
        ctx->stats.wave_ms += elapsed(ctx->ev[1], ctx->ev[2]);
        ctx->stats.reduce_ms += elapsed(ctx->ev[2], ctx->ev[3]);
    }
    ctx->stats.expand_launches += G;
    ctx->stats.wave_launches += 1;
    ctx->stats.reduce_launches += (int64_t)rs.size();
    ctx->stats.subsets += std::ldexp(1.0, n);
    out.T = qd_to_dd(qd_make(res.t0, res.t1, res.t2, res.t3));
    out.A = res.a;
    return TOR_OK;
}

// Vacuum conditioning of one reduced pattern (r.cond set) in quad-double, one
// two-kernel step per no-click mode; returns the conditioned leading block.
tor_status condition_qd(tor_ctx *ctx, const Reduced &r, std::vector<qd> &sigc, dd &pvac, double &log_pvac) {
    const int n = r.n, k = r.k, D = r.D;
    const size_t words = r.packed.size();
    const size_t cols_off = align_up(words * sizeof(qd), 256);
    const size_t cols_words = 2 * (2 * (size_t)(n + k) - 2 + D) + 2;
    const size_t acc_off = align_up(cols_off + cols_words * sizeof(qd), 256);
    const size_t job_off = align_up(acc_off + 3 * sizeof(double), 256);
    const size_t total_bytes = job_off + (size_t)k * sizeof(CondJobQ);
    if (total_bytes > ctx->mem_budget)
        return fail(TOR_ENOMEM, "conditioning needs %.2f GB of device memory", total_bytes / 1e9);
    if (ctx->cond.ensure(total_bytes) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of %.2f GB failed", total_bytes / 1e9);
    unsigned char *db = (unsigned char *)ctx->cond.p;
    std::vector<unsigned char> stage(total_bytes);
    qd *hm = (qd *)stage.data();
    for (size_t e = 0; e < words; e++) hm[e] = qd_from_dd(r.packed[e]);
    const double a0[3] = {1.0, 0.0, 0.0};
    std::memcpy(stage.data() + acc_off, a0, sizeof a0);
    std::vector<long long> blocks(k);
    for (int t = 0; t < k; t++) {
        CondJobQ j{};
        j.mat = db;
        j.acc = (double *)(db + acc_off);
        j.cols = db + cols_off;
        j.qout = nullptr;
        j.r = n + k - t;
        j.d = D;
        j.begin = 0;
        blocks[t] = std::max<long long>(1, (EN(j.r - 1, D) + TOR_COND_CHUNK - 1) / TOR_COND_CHUNK);
        std::memcpy(stage.data() + job_off + t * sizeof(CondJobQ), &j, sizeof j);
    }
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemcpyAsync(db, stage.data(), total_bytes, hipMemcpyHostToDevice, st));
    for (int t = 0; t < k; t++)
        HIP_TRY(tor_launch_condition_qd((const CondJobQ *)(db + job_off) + t, 1, blocks[t], st));
    sigc.assign((size_t)EN(n, D), qd_from(0.0));
    double acc[3];
    HIP_TRY(hipMemcpyAsync(sigc.data(), db, sigc.size() * sizeof(qd), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(acc, db + acc_off, sizeof acc, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    ctx->stats.condition_launches += 2 * (int64_t)k;
    pvac = dd_make(acc[0], acc[1]);
    log_pvac = acc[2];
    return TOR_OK;
}

// Probability of one pattern with quad-double terms (conditioning included).
// With st (a state inverted in quad-double) a full pattern takes the
// complementary-minor route with G gathered from the quad-double inverse.
tor_status probability_qd(tor_ctx *ctx, const double *cov, int m, const int8_t *pattern, double tol,
                          tor_result *out, const tor_state *st = nullptr) {
    Reduced red;
    const bool jacobi = st && st->inv_prec == TOR_PREC_QD && pattern && is_full_pattern(pattern, m);
    tor_status s = jacobi ? reduce_pattern_jacobi(st, pattern, red) : reduce_pattern(cov, m, pattern, red);
    if (s) return s;
    std::vector<qd> sigc;
    Prepared p;
    p.n = red.n;
    if (jacobi) {
        std::vector<int> C;
        for (int i = 0; i < m; i++)
            if (pattern[i] == 1) C.push_back(i);
        const int dc = 2 * red.n;
        sigc.assign((size_t)E(red.n), qd_from(0.0));
        for (int a = 0; a < dc; a++)
            for (int b = 0; b <= a; b++)
                sigc[(size_t)pidx(a, b)] = st->inv_q[(size_t)pidx(2 * C[a / 2] + (a & 1), 2 * C[b / 2] + (b & 1))];
        p.pvac = red.pvac;
        p.log_pvac = red.log_pvac;
        p.scaled = true;
        p.tscale = red.tscale;
        p.pdirect = red.pdirect;
        p.cond_u = m * kUQD;  // the quad-double inverse's sweeps, no rounding
    } else if (red.cond) {
        s = condition_qd(ctx, red, sigc, p.pvac, p.log_pvac);
        if (s) return s;
        p.cond_u = red.k * kUQD;
    } else {
        const int dc = 2 * red.n;
        sigc.assign((size_t)E(red.n), qd_from(0.0));
        for (int a = 0; a < dc; a++)
            for (int b = 0; b <= a; b++) sigc[(size_t)pidx(a, b)] = qd_from_dd(red.sig[(size_t)a * dc + b]);
    }
    if (red.n > 0) {  // PD check and log det from the binary64 rounding
        const int dc = 2 * red.n;
        std::vector<dd> full((size_t)dc * dc);
        for (int a = 0; a < dc; a++)
            for (int b = 0; b <= a; b++) {
                const dd v = qd_to_dd(sigc[(size_t)pidx(a, b)]);
                full[(size_t)a * dc + b] = v;
                full[(size_t)b * dc + a] = v;
            }
        if (!f64_cholesky_logdet(full, dc, &p.log_det)) return fail(TOR_ENOTPD, "Sigma_C is not positive definite");
        if (jacobi) p.log_det = -p.log_det;  // the matrix was G = Sigma_C^-1
    }
    SumOut so;
    s = gpu_sum_qd(ctx, sigc, red.n, so);
    if (s) return s;
    if (!std::isfinite(so.T.hi) || !std::isfinite(so.A)) {
        std::memset(out, 0, sizeof *out);
        out->status = TOR_ENOTPD;
        return fail(TOR_ENOTPD, "a Schur pivot was not positive (non-physical or near-singular covariance)");
    }
    if (!(tol > 0.0)) tol = 1e-10;
    finalize(p, so, TOR_PREC_QD, tol, out);
    return out->status;
}

// Probability of one pattern of a displaced state with quad-double terms:
// the packed matrix with its mean row, conditioned in qd when the pattern has
// no-click modes, then the qd tree with the pivots' overlap factors.
tor_status probability_qd_disp(tor_ctx *ctx, const double *cov, const double *mean, int m, const int8_t *pattern,
                               double tol, tor_result *out, const tor_state *st = nullptr) {
    if (st && st->inv_prec == TOR_PREC_QD && pattern && is_full_pattern(pattern, m)) {
        // inverted state: the information-form tree over [0, h_C; h_C, G] in qd
        Reduced red;
        tor_status s = reduce_pattern_jacobi_disp(st, pattern, red);  // the dd factors
        if (s) return s;
        std::vector<int> C;
        for (int i = 0; i < m; i++)
            if (pattern[i] == 1) C.push_back(i);
        const int dc = 2 * red.n;
        std::vector<qd> sigc((size_t)EN(red.n, 1), qd_from(0.0));
        for (int a = 0; a < dc; a++) {
            const int ga = 2 * C[a / 2] + (a & 1);
            sigc[(size_t)pidx(a + 1, 0)] = st->inv_h_q[ga];
            for (int b = 0; b <= a; b++)
                sigc[(size_t)pidx(a + 1, b + 1)] = st->inv_q[(size_t)pidx(ga, 2 * C[b / 2] + (b & 1))];
        }
        Prepared p;
        s = prepare_reduced(red, p);  // log det Sigma_C, quad = h_C^T G^-1 h_C, tree kind -1
        if (s) return s;
        p.cond_u = m * kUQD;  // the quad-double inverse's sweeps, no rounding
        SumOut so;
        s = gpu_sum_qd(ctx, sigc, red.n, so, -1);
        if (s) return s;
        if (!std::isfinite(so.T.hi) || !std::isfinite(so.A)) {
            std::memset(out, 0, sizeof *out);
            out->status = TOR_ENOTPD;
            return fail(TOR_ENOTPD, "a Schur pivot was not positive (non-physical or near-singular covariance)");
        }
        if (!(tol > 0.0)) tol = 1e-10;
        finalize(p, so, TOR_PREC_QD, tol, out);
        return out->status;
    }
    Reduced red;
    tor_status s = reduce_pattern_disp(cov, mean, m, pattern, red);
    if (s) return s;
    std::vector<qd> sigc;
    dd pvac = dd_from(1.0);
    double log_pvac = 0.0;
    if (red.cond) {
        s = condition_qd(ctx, red, sigc, pvac, log_pvac);
        if (s) return s;
    } else {
        sigc.resize(red.packed.size());
        for (size_t e = 0; e < sigc.size(); e++) sigc[e] = qd_from_dd(red.packed[e]);
    }
    // PD check, log det Sigma_C and the bound's mu_C^T Sigma_C^-1 mu_C from the
    // double-double rounding
    std::vector<dd> rounded(sigc.size());
    for (size_t e = 0; e < sigc.size(); e++) rounded[e] = qd_to_dd(sigc[e]);
    Prepared p;
    s = prepare_disp(std::move(rounded), red.n, pvac, log_pvac, p);
    if (s) return s;
    p.cond_u = red.cond ? red.k * kUQD : 0.0;
    SumOut so;
    s = gpu_sum_qd(ctx, sigc, red.n, so, 1);
    if (s) return s;
    if (!std::isfinite(so.T.hi) || !std::isfinite(so.A)) {
        std::memset(out, 0, sizeof *out);
        out->status = TOR_ENOTPD;
        return fail(TOR_ENOTPD, "a Schur pivot was not positive (non-physical or near-singular covariance)");
    }
    if (!(tol > 0.0)) tol = 1e-10;
    finalize(p, so, TOR_PREC_QD, tol, out);
    return out->status;
}

// Evaluate prepared queries with the precision policy; results in out[i].
// Queries whose preparation failed keep their error status.
tor_status evaluate_many(tor_ctx *ctx, std::vector<Prepared> &qs, tor_prec prec, double tol, tor_result *out) {
    if (prec != TOR_PREC_AUTO && prec != TOR_PREC_F64 && prec != TOR_PREC_DD) {
        for (size_t i = 0; i < qs.size(); i++) {  // every result carries the error
            std::memset(&out[i], 0, sizeof out[i]);
            out[i].status = TOR_EINVAL;
        }
        return fail(TOR_EINVAL, "precision %d is not supported here (TOR_PREC_QD: tor_probability and "
                                "tor_subset_sum only)", (int)prec);
    }
    if (!(tol > 0.0)) tol = 1e-10;
    std::vector<SumIn> in(qs.size());
    std::vector<int> ok;
    for (size_t i = 0; i < qs.size(); i++) {
        in[i].packed = &qs[i].packed;
        in[i].n = qs[i].n;
        in[i].D = qs[i].D;
        if (qs[i].status == TOR_OK) ok.push_back((int)i);
    }
    std::vector<SumOut> res(qs.size());
    std::vector<int> used(qs.size(), prec == TOR_PREC_DD ? TOR_PREC_DD : TOR_PREC_F64);
    auto fail_all = [&](tor_status e) {
        for (size_t i = 0; i < qs.size(); i++) {
            std::memset(&out[i], 0, sizeof out[i]);
            out[i].status = e;
        }
        return e;
    };
    tor_status s = gpu_sums(ctx, in, ok, prec == TOR_PREC_DD, res);
    if (s < 0) return fail_all(s);
    if (prec == TOR_PREC_AUTO) {
        std::vector<int> redo;
        for (int i : ok)
            if (qs[i].n > 0 &&
                !(bound_of(TOR_PREC_F64, qs[i].n, res[i].T, res[i].A, qs[i].quad, qs[i].cond_u) <= tol))
                redo.push_back(i);
        if (!redo.empty()) {
            s = gpu_sums(ctx, in, redo, true, res);
            if (s < 0) return fail_all(s);
            for (int i : redo) used[i] = TOR_PREC_DD;
        }
    }
    tor_status first = TOR_OK;
    for (size_t i = 0; i < qs.size(); i++) {
        if (qs[i].status != TOR_OK) {
            std::memset(&out[i], 0, sizeof out[i]);
            out[i].status = qs[i].status;
            if (first >= 0) first = qs[i].status;
            continue;
        }
        if (!std::isfinite(res[i].T.hi) || !std::isfinite(res[i].A)) {
            std::memset(&out[i], 0, sizeof out[i]);
            out[i].status = TOR_ENOTPD;
            if (first >= 0) {
                first = fail(TOR_ENOTPD, "a Schur pivot was not positive (non-physical or near-singular covariance)");
            }
            continue;
        }
        finalize(qs[i], res[i], used[i], tol, &out[i]);
        if (out[i].status == TOR_WARN_PRECISION && first == TOR_OK) first = TOR_WARN_PRECISION;
    }
    return first;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

tor_status tor_load_tuning(tor_ctx *ctx, const char *cache_path);

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
    if (hipHostMalloc((void **)&c->host_res, sizeof(Partial) * 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(c->own_stream);
        delete c;
        return fail(TOR_ENOMEM, "pinned allocation failed");
    }
    c->host_res_cap = 64;
    for (auto &e : c->ev) (void)hipEventCreate(&e);
    scratch_setup(device);
    // tuning table: TOR_TUNE_CACHE if set, else the table shipped beside the
    // library (tor_tuning.json); a missing or unreadable table is not an error
    const char *tc = std::getenv("TOR_TUNE_CACHE");
    if (tc && *tc) {
        if (tor_load_tuning(c, tc) != TOR_OK) g_err.clear();
    } else if (!tc) {
        Dl_info info;
        if (dladdr((void *)&tor_ctx_create, &info) && info.dli_fname) {
            std::string path(info.dli_fname);
            const size_t slash = path.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tor_tuning.json";
            if (FILE *f = std::fopen(path.c_str(), "r")) {
                std::fclose(f);
                if (tor_load_tuning(c, path.c_str()) != TOR_OK) g_err.clear();
            }
        }
    }
    *out = c;
    return TOR_OK;
}

void tor_ctx_destroy(tor_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    // stream-ordered batches may still run on the callers' streams
    if (c->abuf.p || c->apool.p) (void)hipDeviceSynchronize();
    c->pool.release();
    c->descA.release();
    c->descB.release();
    c->partA.release();
    c->partB.release();
    c->jobs.release();
    c->cond.release();
    c->apool.release();
    c->abuf.release();
    for (DevBuf *b : {&c->kbuf, &c->koff, &c->hbuf, &c->hoff, &c->c_out, &c->c_status, &c->c_tp, &c->c_tu,
                      &c->c_sub, &c->klobuf, &c->hlobuf, &c->c_tr, &c->c_tb})
        b->release();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    c->fctr.release();
    c->cov_tmp.release();
    c->screen.release();
    if (c->screen_host) (void)hipHostFree(c->screen_host);
    if (c->host_res) (void)hipHostFree(c->host_res);
    if (c->pin_stage) (void)hipHostFree(c->pin_stage);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    (void)hipGetLastError();  // leave no error for the next checked call
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
        if (v < 1 || v > TOR_TASK_MAX) return fail(TOR_EINVAL, "task modes must be in 1..%d", TOR_TASK_MAX);
        c->task_modes[0] = c->task_modes[1] = (int)v;
        std::memset(c->tuned, 0, sizeof c->tuned);  // an explicit size overrides the tuning table
        return TOR_OK;
    case TOR_OPT_WAVE_GRID:
        if (v < 1 || v > (1LL << 30)) return fail(TOR_EINVAL, "bad wave grid cap");
        c->wave_grid = (int)v;
        return TOR_OK;
    case TOR_OPT_MEM_BUDGET:
        if (v < (1 << 20)) return fail(TOR_EINVAL, "memory budget too small");
        c->mem_budget = (size_t)v;
        return TOR_OK;
    case TOR_OPT_ASYNC_POOL:
        if (v < (1 << 20)) return fail(TOR_EINVAL, "async pool too small");
        c->async_pool = (size_t)v;
        return TOR_OK;
    case TOR_OPT_CHAIN_CLICKS:
        if (v < 1 || v > TOR_CHAIN_CLICKS) return fail(TOR_EINVAL, "chain click cap must be in 1..%d", TOR_CHAIN_CLICKS);
        c->chain_clicks = (int)v;
        return TOR_OK;
    case TOR_OPT_COND_BLOCK:
        if (v < 1 || v > TOR_COND_BLOCK) return fail(TOR_EINVAL, "conditioning block must be in 1..%d", TOR_COND_BLOCK);
        c->cond_block = (int)v;
        return TOR_OK;
    case TOR_OPT_CHAIN_PREC:
        if (v != TOR_PREC_F64 && v != TOR_PREC_DD)
            return fail(TOR_EINVAL, "chain term precision must be TOR_PREC_F64 or TOR_PREC_DD");
        c->chain_prec = (int)v;
        return TOR_OK;
    case TOR_OPT_FUSED:
        if (v != 0 && v != 1) return fail(TOR_EINVAL, "the single-launch switch must be 0 or 1");
        c->fused = v != 0;
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
    // A pattern that observes most modes, many of them without a click: the
    // covariance goes to the device in one copy and the (C, N) matrix is
    // gathered there, as for the queries of a state (the same words as the
    // host packing), instead of being packed entry by entry on the host; the
    // finiteness and symmetry checks of the observed block then run on the
    // device too (the host's scan, with its message, only when they fail).
    bool on_device = false;
    if (cov && pattern && m > 0 && m <= 100000 && prec != TOR_PREC_QD) {
        int observed = 0, noclick = 0;
        bool valid = true;
        for (int i = 0; i < m && valid; i++) {
            valid = pattern[i] >= -1 && pattern[i] <= 1;
            observed += pattern[i] != -1;
            noclick += pattern[i] == 0;
        }
        on_device = valid && noclick >= kDeviceGatherNoClick && 2 * observed >= m;
    }
    tor_status s;
    if (!on_device) {
        s = validate_cov_block(cov, m, pattern);
        if (s) return s;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    if (!out) return fail(TOR_EINVAL, "out is NULL");
    if (prec == TOR_PREC_QD) return probability_qd(ctx, cov, m, pattern, tol, out);
    Reduced red;
    tor_state tmp;
    s = reduce_pattern(cov, m, pattern, red, on_device);
    if (s) {
        if (on_device) {  // a bad covariance is reported first, as on the host path
            tor_status v = validate_cov_block(cov, m, pattern);
            if (v) return v;
        }
        return s;
    }
    const bool screened = on_device && red.cond;
    if (screened) {
        const size_t cov_bytes = 4 * (size_t)m * (size_t)m * sizeof(double);
        const size_t g_bytes = red.g.size() * sizeof(int);
        if (ctx->cov_tmp.ensure(cov_bytes) != hipSuccess || ctx->screen.ensure(g_bytes + 64) != hipSuccess)
            return fail(TOR_ENOMEM, "device copy of the covariance failed");
        if (!ctx->screen_host &&
            hipHostMalloc((void **)&ctx->screen_host, 4 * sizeof(unsigned long long), hipHostMallocDefault) !=
                hipSuccess) {
            ctx->screen_host = nullptr;
            return fail(TOR_ENOMEM, "pinned allocation failed");
        }
        hipStream_t st = ctx->stream;
        unsigned long long *words = (unsigned long long *)ctx->screen.p;
        int *dg = (int *)((unsigned char *)ctx->screen.p + 64);
        HIP_TRY(hipMemcpyAsync(ctx->cov_tmp.p, cov, cov_bytes, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dg, red.g.data(), g_bytes, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemsetAsync(words, 0, 4 * sizeof(unsigned long long), st));
        HIP_TRY(tor_launch_cov_screen((const double *)ctx->cov_tmp.p, m, dg, (int)red.g.size(), words, st));
        HIP_TRY(hipMemcpyAsync(ctx->screen_host, words, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        tmp.ctx = ctx;
        tmp.device = ctx->device;
        tmp.m = m;
        tmp.dcov.p = ctx->cov_tmp.p;  // borrowed: tmp never releases it
        tmp.dcov.cap = ctx->cov_tmp.cap;
        red.st = &tmp;
    }
    s = condition_on_gpu(ctx, {&red});
    tmp.dcov.p = nullptr;
    if (screened) {
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        double amax, asym;
        std::memcpy(&amax, &ctx->screen_host[0], sizeof amax);
        std::memcpy(&asym, &ctx->screen_host[2], sizeof asym);
        if (ctx->screen_host[1] || asym > 1e-12 * amax) {
            tor_status v = validate_cov_block(cov, m, pattern);  // the host's scan names the entry
            if (v) return v;
        }
    }
    if (s) return s;
    std::vector<Prepared> qs(1);
    s = prepare(red.sig, red.n, red.pvac, red.log_pvac, qs[0]);
    if (s) return s;
    qs[0].cond_u = red.cond_u;
    return evaluate_many(ctx, qs, prec, tol, out);
}

tor_status tor_probability_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                     const int8_t *pattern, tor_prec prec, double tol, tor_result *out) {
    if (!ctx) return fail(TOR_EINVAL, "ctx is NULL");
    tor_status s = validate_cov_block(cov, m, pattern);
    if (s) return s;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!out) return fail(TOR_EINVAL, "out is NULL");
    if (prec == TOR_PREC_QD) return probability_qd_disp(ctx, cov, mean, m, pattern, tol, out);
    Reduced red;
    s = reduce_pattern_disp(cov, mean, m, pattern, red);
    if (s) return s;
    s = condition_on_gpu(ctx, {&red});
    if (s) return s;
    std::vector<Prepared> qs(1);
    s = prepare_disp(std::move(red.packed), red.n, red.pvac, red.log_pvac, qs[0]);
    if (s) return s;
    qs[0].cond_u = red.cond_u;
    return evaluate_many(ctx, qs, prec, tol, out);
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
    if (!out) return fail(TOR_EINVAL, "out is NULL");
    std::vector<Prepared> qs(1);
    tor_status s = prepare(sig, n, dd_from(1.0), 0.0, qs[0]);
    if (s) return s;
    if (prec == TOR_PREC_QD) {
        std::vector<qd> pk((size_t)E(n));
        for (int a = 0; a < 2 * n; a++)
            for (int b = 0; b <= a; b++) pk[(size_t)pidx(a, b)] = qd_from_dd(sig[(size_t)a * 2 * n + b]);
        SumOut so;
        s = gpu_sum_qd(ctx, pk, n, so);
        if (s) return s;
        if (!(tol > 0.0)) tol = 1e-10;
        finalize(qs[0], so, TOR_PREC_QD, tol, out);
        return out->status;
    }
    return evaluate_many(ctx, qs, prec, tol, out);
}

tor_status tor_state_create(tor_ctx *ctx, const double *cov, int32_t m, tor_state **out) {
    if (!ctx || !out) return fail(TOR_EINVAL, "NULL argument");
    *out = nullptr;
    tor_status s = validate_cov(cov, m);
    if (s) return s;
    tor_state *st = new (std::nothrow) tor_state();
    if (!st) return fail(TOR_ENOMEM, "host allocation failed");
    st->ctx = ctx;
    st->device = ctx->device;
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

tor_status tor_state_create_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                      tor_state **out) {
    if (!ctx || !out || !mean) return fail(TOR_EINVAL, "NULL argument");
    *out = nullptr;
    for (int i = 0; i < 2 * m; i++)
        if (!std::isfinite(mean[i])) return fail(TOR_EINVAL, "mean[%d] is not finite", i);
    tor_state *st = nullptr;
    tor_status s = tor_state_create(ctx, cov, m, &st);
    if (s) return s;
    try {
        st->mean.assign(mean, mean + 2 * (size_t)m);
    } catch (...) {
        tor_state_destroy(st);
        return fail(TOR_ENOMEM, "host allocation failed");
    }
    *out = st;
    return TOR_OK;
}

void tor_state_destroy(tor_state *st) {
    if (!st) return;
    if (st->dcov.p || st->dmean.p || st->dinv.p || st->dinvh.p || st->dK.p) {
        (void)hipSetDevice(st->device);
        st->dcov.release();
        st->dmean.release();
        st->dinv.release();
        st->dinvh.release();
        st->dK.release();
        (void)hipGetLastError();  // leave no error for the next checked call
    }
    delete st;
}

tor_status tor_state_invert(tor_state *st, tor_prec prec) {
    if (!st) return fail(TOR_EINVAL, "state is NULL");
    if (prec != TOR_PREC_AUTO && prec != TOR_PREC_F64 && prec != TOR_PREC_DD && prec != TOR_PREC_QD)
        return fail(TOR_EINVAL, "precision %d is not a tor_prec", (int)prec);
    const int m = st->m;
    if (m > TOR_INVERT_MAX_MODES) return fail(TOR_ETOOBIG, "m = %d > %d modes for the inverse", m, TOR_INVERT_MAX_MODES);
    const bool q = prec == TOR_PREC_QD;
    tor_ctx *ctx = st->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    const int d = 2 * m;
    const size_t ent = (size_t)E(m), es = q ? sizeof(qd) : sizeof(dd);
    const size_t cols_off = align_up(ent * es, 256);
    const size_t piv_off = align_up(cols_off + 2 * (size_t)d * es, 256);
    const size_t acc_off = align_up(piv_off + 3 * es, 256);
    const size_t total = acc_off + 3 * sizeof(double);
    const size_t cov_bytes = 4 * (size_t)m * (size_t)m * sizeof(double);  // the state's device copy of sigma
    if (total + cov_bytes > ctx->mem_budget)
        return fail(TOR_ENOMEM, "the inverse needs %.2f GB of device memory", (total + cov_bytes) / 1e9);
    struct Scoped {  // the device buffer lives for this call only
        DevBuf b;
        ~Scoped() { b.release(); }
    } buf;
    if (buf.b.ensure(total) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of %.2f GB failed", total / 1e9);
    unsigned char *db = (unsigned char *)buf.b.p;
    // sigma_Q packed on the device from the state's device copy of sigma
    // (made once per state and kept for the gathers), then the sweeps, the
    // negation of -sigma_Q^-1 and one copy into the state's host words
    tor_status ds = state_on_device(st);
    if (ds) return ds;
    hipStream_t hs = ctx->stream;
    double *dacc = (double *)(db + acc_off);
    HIP_TRY(tor_launch_pack_sigq(q, (const double *)st->dcov.p, m, db, dacc, hs));
    for (int k = 0; k < m; k++) HIP_TRY(tor_launch_sweep(q, db, m, k, db + cols_off, db + piv_off, dacc, hs));
    HIP_TRY(tor_launch_negate(q, db, m, hs));
    std::vector<dd> inv;
    std::vector<qd> inv_q;
    if (q) inv_q.resize(ent);
    else inv.resize(ent);
    HIP_TRY(hipMemcpyAsync(q ? (void *)inv_q.data() : (void *)inv.data(), db, ent * es, hipMemcpyDeviceToHost, hs));
    double acc[3];
    HIP_TRY(hipMemcpyAsync(acc, dacc, sizeof acc, hipMemcpyDeviceToHost, hs));
    HIP_TRY(hipStreamSynchronize(hs));
    if (!(acc[0] > 0.0) || !std::isfinite(acc[0]) || !std::isfinite(acc[2]))
        return fail(TOR_ENOTPD, "a pivot of sigma_Q was not positive");
    st->inv_prec = 0;
    st->dinv.release();  // device copies of an earlier inverse are stale
    st->dinvh.release();
    st->inv.swap(inv);
    st->inv_q.swap(inv_q);
    st->det_rsqrt = dd_make(acc[0], acc[1]);
    st->log_det_sigq = -2.0 * acc[2];
    std::vector<dd>().swap(st->inv_h);
    std::vector<qd>().swap(st->inv_h_q);
    st->mu_k_mu = dd_from(0.0);
    st->det_rsqrt_mean = st->det_rsqrt;
    if (!st->mean.empty() && q) {  // h = K mu and mu^T K mu in quad-double
        st->inv_h_q.assign(d, qd_from(0.0));
        st->inv_h.assign(d, dd_from(0.0));
        qd mkm = qd_from(0.0);
        for (int a = 0; a < d; a++) {
            qd s = qd_from(0.0);
            for (int b = 0; b < d; b++)
                s = qd_add(s, qd_mul_d(st->inv_q[(size_t)(a >= b ? pidx(a, b) : pidx(b, a))], st->mean[b]));
            st->inv_h_q[a] = s;
            st->inv_h[a] = qd_to_dd(s);
            mkm = qd_add(mkm, qd_mul_d(s, st->mean[a]));
        }
        st->mu_k_mu = qd_to_dd(mkm);
    } else if (!st->mean.empty()) {  // h = K mu and mu^T K mu in double-double
        st->inv_h.assign(d, dd_from(0.0));
        for (int a = 0; a < d; a++) {
            dd s = dd_from(0.0);
            for (int b = 0; b < d; b++) {
                const size_t e = (size_t)(a >= b ? pidx(a, b) : pidx(b, a));
                s = dd_add(s, dd_mul_d(st->inv[e], st->mean[b]));
            }
            st->inv_h[a] = s;
            st->mu_k_mu = dd_add(st->mu_k_mu, dd_mul_d(s, st->mean[a]));
        }
    }
    if (!st->mean.empty()) {
        const dd hm = dd_make(-0.5 * st->mu_k_mu.hi, -0.5 * st->mu_k_mu.lo);
        st->det_rsqrt_mean = dd_mul(st->det_rsqrt, dd_exp(hm));
    }
    st->inv_prec = q ? TOR_PREC_QD : TOR_PREC_DD;
    return TOR_OK;
}

tor_status tor_batch(tor_ctx *ctx, const tor_state *st, int32_t nq, const int8_t *patterns, tor_prec prec,
                     double tol, tor_result *out) {
    if (!ctx || !st || !out || (nq > 0 && !patterns)) return fail(TOR_EINVAL, "NULL argument");
    if (st->ctx != ctx) return fail(TOR_EINVAL, "state belongs to another context");
    if (nq < 0) return fail(TOR_EINVAL, "nq < 0");
    HIP_TRY(hipSetDevice(ctx->device));
    if (prec == TOR_PREC_QD) {  // quad-double conditioning and trees, one query at a time
        tor_status first = TOR_OK;
        for (int q = 0; q < nq; q++) {
            std::memset(&out[q], 0, sizeof out[q]);
            const int8_t *pat = patterns + (size_t)q * st->m;
            tor_status s = st->mean.empty()
                               ? probability_qd(ctx, st->cov.data(), st->m, pat, tol, &out[q], st)
                               : probability_qd_disp(ctx, st->cov.data(), st->mean.data(), st->m, pat, tol, &out[q],
                                                     st);
            if (s < 0) {
                std::memset(&out[q], 0, sizeof out[q]);
                out[q].status = s;
                if (s == TOR_EDEVICE) return s;
            }
            if (s < 0 && first >= 0) first = s;
            else if (s == TOR_WARN_PRECISION && first == TOR_OK) first = s;
        }
        return first;
    }
    std::vector<Prepared> qs((size_t)nq);
    std::vector<Reduced> red((size_t)nq);
    std::vector<Reduced *> rp;
    for (int q = 0; q < nq; q++) {
        tor_status s = reduce_for_state(st, patterns + (size_t)q * st->m, red[q]);
        if (s != TOR_OK) qs[q].status = s;
        else rp.push_back(&red[q]);
    }
    tor_status cs = condition_on_gpu(ctx, rp);
    if (cs < 0) {
        for (int q = 0; q < nq; q++) {
            std::memset(&out[q], 0, sizeof out[q]);
            out[q].status = cs;
        }
        return cs;
    }
    for (int q = 0; q < nq; q++) {
        if (qs[q].status != TOR_OK) continue;
        tor_status s = prepare_reduced(red[q], qs[q]);
        if (s != TOR_OK) {
            qs[q].status = s;
            qs[q].n = 0;
        }
    }
    return evaluate_many(ctx, qs, prec, tol, out);
}

tor_status tor_batch_displaced(tor_ctx *ctx, const tor_state *st, const double *mean, int32_t nq,
                               const int8_t *patterns, tor_prec prec, double tol, tor_result *out) {
    if (!ctx || !st || !out || !mean || (nq > 0 && !patterns)) return fail(TOR_EINVAL, "NULL argument");
    if (st->ctx != ctx) return fail(TOR_EINVAL, "state belongs to another context");
    if (nq < 0) return fail(TOR_EINVAL, "nq < 0");
    HIP_TRY(hipSetDevice(ctx->device));
    if (prec == TOR_PREC_QD) {  // quad-double conditioning and trees, one query at a time
        tor_status first = TOR_OK;
        for (int q = 0; q < nq; q++) {
            std::memset(&out[q], 0, sizeof out[q]);
            tor_status s =
                probability_qd_disp(ctx, st->cov.data(), mean, st->m, patterns + (size_t)q * st->m, tol, &out[q]);
            if (s < 0) {
                std::memset(&out[q], 0, sizeof out[q]);
                out[q].status = s;
                if (s == TOR_EDEVICE) return s;
            }
            if (s < 0 && first >= 0) first = s;
            else if (s == TOR_WARN_PRECISION && first == TOR_OK) first = s;
        }
        return first;
    }
    std::vector<Prepared> qs((size_t)nq);
    std::vector<Reduced> red((size_t)nq);
    std::vector<Reduced *> rp;
    for (int q = 0; q < nq; q++) {
        tor_status s = reduce_pattern_disp(st->cov.data(), mean, st->m, patterns + (size_t)q * st->m, red[q]);
        if (s != TOR_OK) qs[q].status = s;
        else rp.push_back(&red[q]);
    }
    tor_status cs = condition_on_gpu(ctx, rp);
    if (cs < 0) {
        for (int q = 0; q < nq; q++) {
            std::memset(&out[q], 0, sizeof out[q]);
            out[q].status = cs;
        }
        return cs;
    }
    for (int q = 0; q < nq; q++) {
        if (qs[q].status != TOR_OK) continue;
        qs[q].cond_u = red[q].cond_u;
        tor_status s = prepare_disp(std::move(red[q].packed), red[q].n, red[q].pvac, red[q].log_pvac, qs[q]);
        if (s != TOR_OK) {
            qs[q].status = s;
            qs[q].n = 0;
        }
    }
    return evaluate_many(ctx, qs, prec, tol, out);
}

}  // extern "C"

namespace {

// Enqueue a stream-ordered batch.  With st the queries are patterns of that
// state (its device copies are made on first use); with st == nullptr they
// are marginal patterns of the zero-mean covariance d_cov (caller-owned
// device memory, 2m x 2m row-major).  With ws == nullptr the workspace is the
// context's own (grown on demand); otherwise it is ws[0 .. ws_bytes), and
// nothing is allocated: the tree pool takes what the plan tables leave.
tor_status batch_async_impl(tor_ctx *ctx, const tor_state *st, const double *d_cov, int32_t m, int32_t nq,
                            const int8_t *d_patterns, tor_prec prec, double tol, tor_result *d_out, void *stream,
                            unsigned char *ws, size_t ws_bytes) {
    if (!(tol > 0.0)) tol = 1e-10;
    const bool use_dd = prec != TOR_PREC_F64;
    const int used = use_dd ? TOR_PREC_DD : TOR_PREC_F64;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t hs = stream ? (hipStream_t)stream : ctx->stream;
    tor_state *ms = const_cast<tor_state *>(st);  // the device copies are a cache of the state
    const size_t cov_bytes = 4 * (size_t)m * (size_t)m * sizeof(double);
    if (st) {
        tor_status ds = state_on_device(st);
        if (ds) return ds;
        d_cov = (const double *)ms->dcov.p;
    }
    const int D = (st && !st->mean.empty()) ? 1 : 0;
    // task sizes and the launches any pattern of this state can need
    AsyncPlan P{};
    P.nq = nq;
    P.m = m;
    P.is_dd = use_dd;
    P.D = D;
    P.mean = D ? (const double *)ms->dmean.p : nullptr;
    // full patterns of an inverted state: the inverse (and h = K mu) on the
    // device; a displaced state's full patterns are a second tree kind (the
    // information form) beside its displaced trees
    P.nkinds = 1;
    if (st && st->inv_prec) {
        const size_t ent = (size_t)E(m);
        std::lock_guard<std::mutex> lk(ms->dev_mu);
        if (!ms->dinv.p) {
            std::vector<dd> h(ent);
            for (size_t e = 0; e < ent; e++) h[e] = st->inv_prec == TOR_PREC_QD ? qd_to_dd(st->inv_q[e]) : st->inv[e];
            if (ms->dinv.ensure(ent * sizeof(dd)) != hipSuccess)
                return fail(TOR_ENOMEM, "device copy of the inverse failed");
            HIP_TRY(hipMemcpy(ms->dinv.p, h.data(), ent * sizeof(dd), hipMemcpyHostToDevice));
            g_data_gen++;
        }
        if (D && !ms->dinvh.p) {
            if (ms->dinvh.ensure(st->inv_h.size() * sizeof(dd)) != hipSuccess)
                return fail(TOR_ENOMEM, "device copy of h failed");
            HIP_TRY(hipMemcpy(ms->dinvh.p, st->inv_h.data(), st->inv_h.size() * sizeof(dd), hipMemcpyHostToDevice));
            g_data_gen++;
        }
        P.inv = ms->dinv.p;
        P.inv_h = D ? ms->dinvh.p : nullptr;
        P.det_rsqrt_hi = st->det_rsqrt_mean.hi;  // = det_rsqrt for a zero-mean state
        P.det_rsqrt_lo = st->det_rsqrt_mean.lo;
        P.log_det_sigq = st->log_det_sigq;
        P.mu_k_mu = st->mu_k_mu.hi + st->mu_k_mu.lo;
        P.inv_cond_u = inverse_cond_u(st);
        P.nkinds = D ? 2 : 1;
    }
    const int nmax = std::min(TOR_MAX_CLICKS, m);
    int gcap = 0, jmax = 1;
    long long max_tasks[TOR_TASK_MAX + 1] = {};  // per J: tasks of the largest tree
    long long nt_max = 1;
    bool jused[TOR_TASK_MAX + 1] = {};
    for (int n = 0; n <= TOR_MAX_CLICKS; n++) {
        P.J_of_n[n] = n >= 1 ? task_modes_for(ctx, use_dd, n) : 1;
        if (n < 1 || n > nmax) continue;
        const int J = std::min(n, P.J_of_n[n]), G = n - J;
        gcap = std::max(gcap, G);
        jmax = std::max(jmax, J);
        jused[J] = true;
        max_tasks[J] = std::max(max_tasks[J], 1LL << G);
        nt_max = std::max(nt_max, 1LL << G);
    }
    P.gcap = gcap;
    P.jmax = jmax;
    const size_t es = use_dd ? sizeof(dd) : sizeof(double);
    const int stride = gcap + TOR_TASK_MAX + 1;  // launch dimensions per tree kind
    // workspace layout for a tree pool of pool_cap scalars: the plan tables,
    // then (given workspace) the pool
    size_t o_q = 0, o_roots = 0, o_dA = 0, o_dB = 0, o_pA = 0, o_pB = 0, o_ej = 0, o_wj = 0, o_rj = 0, o_dims = 0;
    auto layout = [&](long long pool_cap) {
        P.pool_cap = pool_cap;
        P.desc_cap = P.pool_cap / 16 + nq;
        P.pb_cap = P.desc_cap / TOR_REDUCE_CHUNK + (long long)TOR_ASYNC_STAGES * nq + 8;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off = align_up(off + bytes, 256);
            return o;
        };
        o_q = take((size_t)nq * sizeof(AsyncQuery));
        o_roots = take((size_t)nq * sizeof(NodeDesc));
        o_dA = take((size_t)P.desc_cap * sizeof(NodeDesc));
        o_dB = take((size_t)P.desc_cap * sizeof(NodeDesc));
        o_pA = take((size_t)P.desc_cap * sizeof(Partial));
        o_pB = take((size_t)P.pb_cap * sizeof(Partial));
        o_ej = take((size_t)P.nkinds * std::max(gcap, 1) * nq * sizeof(ExpandJob));
        o_wj = take((size_t)P.nkinds * (TOR_TASK_MAX + 1) * nq * sizeof(WaveJob));
        o_rj = take((size_t)TOR_ASYNC_STAGES * nq * sizeof(ReduceJob));
        o_dims = take(((size_t)P.nkinds * stride + TOR_ASYNC_STAGES) * sizeof(LaunchDims));
        return off;  // bytes of the tables
    };
    unsigned char *b = nullptr;
    if (ws) {
        // the tables grow by about (6 + nq-dependent) bytes per pool scalar
        // (descriptors at pool_cap / 16): size the pool to fill the rest
        const size_t fixed = layout(0);
        if (fixed + 4096 > ws_bytes)
            return fail(TOR_ETOOBIG, "nq = %d: the plan tables alone exceed the %zu-byte workspace", nq, ws_bytes);
        long long cap = (long long)((ws_bytes - fixed - 4096) / (es + 7));
        while (cap > 0 && align_up(layout(cap), 256) + (size_t)cap * es > ws_bytes) cap -= cap / 64 + 1;
        if (cap <= 0) return fail(TOR_ETOOBIG, "nq = %d leaves no tree pool in the workspace", nq);
        const size_t tab = align_up(layout(cap), 256);
        b = ws;
        P.pool = ws + tab;
    } else {
        const size_t abytes = layout((long long)(ctx->async_pool / es)), pbytes = (size_t)P.pool_cap * es;
        if (abytes + pbytes + cov_bytes > ctx->mem_budget)
            return fail(TOR_ENOMEM, "async workspace of %.2f GB exceeds the memory budget", (abytes + pbytes) / 1e9);
        if (ctx->abuf.ensure(abytes) != hipSuccess || ctx->apool.ensure(pbytes) != hipSuccess)
            return fail(TOR_ENOMEM, "device allocation of the async workspace (%.2f GB) failed", (abytes + pbytes) / 1e9);
        b = (unsigned char *)ctx->abuf.p;
        P.pool = ctx->apool.p;
    }
    P.q = (AsyncQuery *)(b + o_q);
    P.roots = (NodeDesc *)(b + o_roots);
    P.descA = (NodeDesc *)(b + o_dA);
    P.descB = (NodeDesc *)(b + o_dB);
    P.partA = (Partial *)(b + o_pA);
    P.partB = (Partial *)(b + o_pB);
    P.exp_jobs = (ExpandJob *)(b + o_ej);
    P.wave_jobs = (WaveJob *)(b + o_wj);
    P.red_jobs = (ReduceJob *)(b + o_rj);
    P.dims = (LaunchDims *)(b + o_dims);
    // scan, plan, roots; then the tree launches with device-side dimensions
    HIP_TRY(tor_launch_async_prologue(d_patterns, d_cov, P, hs));
    for (int k = 0; k < P.nkinds; k++) {  // kind 1: the information-form trees (tree kind -1)
        const int Dk = k ? -1 : D;
        for (int d = 0; d < gcap; d++) {
            const long long bound = std::min<long long>(1LL << 20, ((long long)nq << d) / 4 + 1);
            HIP_TRY(tor_launch_expand(use_dd, P.exp_jobs + ((size_t)k * gcap + d) * nq, 0, d, P.pool, (int)bound,
                                      hs, P.dims + k * stride + d, Dk));
        }
        for (int J = jmax; J >= 1; J--) {
            if (!jused[J]) continue;
            const long long bound = std::min<long long>(ctx->wave_grid, (long long)nq * max_tasks[J]);
            HIP_TRY(tor_launch_wave(use_dd, J, P.wave_jobs + ((size_t)k * (TOR_TASK_MAX + 1) + J) * nq, 0, 0, P.pool,
                                    (int)bound, hs, P.dims + k * stride + gcap + J, Dk));
        }
    }
    long long c = nt_max;
    for (int s = 0; s < TOR_ASYNC_STAGES && c > 1; s++) {
        c = (c + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
        const long long bound = std::min<long long>(1LL << 20, (long long)nq * c);
        HIP_TRY(tor_launch_reduce(P.red_jobs + (size_t)s * nq, 0, bound, hs, P.dims + P.nkinds * stride + s));
    }
    HIP_TRY(tor_launch_async_finalize(P, tol, used, d_out, hs));
    ctx->stats.expand_launches += (int64_t)gcap * P.nkinds;
    return TOR_OK;
}

}  // namespace

extern "C" {

tor_status tor_batch_async(tor_ctx *ctx, const tor_state *st, int32_t nq, const int8_t *d_patterns, tor_prec prec,
                           double tol, tor_result *d_out, void *stream) {
    if (!ctx || !st) return fail(TOR_EINVAL, "NULL argument");
    if (st->ctx != ctx) return fail(TOR_EINVAL, "state belongs to another context");
    if (nq < 0) return fail(TOR_EINVAL, "nq < 0");
    if (prec != TOR_PREC_AUTO && prec != TOR_PREC_F64 && prec != TOR_PREC_DD)
        return fail(TOR_EINVAL, "bad precision %d", (int)prec);
    if (nq == 0) return TOR_OK;
    if (!d_patterns || !d_out) return fail(TOR_EINVAL, "NULL device pointer");
    if (nq > (1 << 24)) return fail(TOR_ETOOBIG, "nq = %d > 2^24", nq);
    return batch_async_impl(ctx, st, nullptr, st->m, nq, d_patterns, prec, tol, d_out, stream, nullptr, 0);
}

tor_status tor_batch_async_noalloc(tor_ctx *ctx, const double *d_cov, int32_t m, int32_t nq,
                                   const int8_t *d_patterns, tor_prec prec, double tol, tor_result *d_out,
                                   void *stream) {
    if (!ctx) return fail(TOR_EINVAL, "ctx is NULL");
    if (m <= 0) return fail(TOR_EINVAL, "m must be positive (got %d)", m);
    if (m > TOR_COND_MAX_MODES * 100) return fail(TOR_ETOOBIG, "m = %d too large", m);
    if (nq < 0) return fail(TOR_EINVAL, "nq < 0");
    if (prec != TOR_PREC_AUTO && prec != TOR_PREC_F64 && prec != TOR_PREC_DD)
        return fail(TOR_EINVAL, "bad precision %d", (int)prec);
    if (nq == 0) return TOR_OK;
    if (!d_cov || !d_patterns || !d_out) return fail(TOR_EINVAL, "NULL device pointer");
    if (nq > TOR_NOALLOC_MAX_QUERIES)
        return fail(TOR_ETOOBIG, "nq = %d > %d queries per call", nq, TOR_NOALLOC_MAX_QUERIES);
    std::string err;
    void *ws = scratch_of(ctx->device, &err);
    if (!ws) return fail(TOR_EDEVICE, "no scratch address for device %d: %s", ctx->device, err.c_str());
    return batch_async_impl(ctx, nullptr, d_cov, m, nq, d_patterns, prec, tol, d_out, stream,
                            (unsigned char *)ws, TOR_NOALLOC_SCRATCH_BYTES);
}

// ------------------------------------------------------------------ sampler

}  // extern "C"

namespace {

// K_j = (sigma_Q[modes 0..j])^-1 for every j, from one double-double Cholesky
// sigma_Q = L L^T: with M = L^-1 (lower triangular) the leading block of M is
// the inverse factor of the leading block, so K_j[a][b] = sum_{t <= 2j+1}
// M[t][a] M[t][b], accumulated row pair by row pair.  Rounded to binary64.
tor_status build_k_tables(const double *cov, int m, std::vector<double> &K, std::vector<unsigned long long> &koff,
                          const double *mean = nullptr, std::vector<double> *H = nullptr,
                          std::vector<unsigned long long> *hoff = nullptr, std::vector<double> *Klo = nullptr,
                          std::vector<double> *Hlo = nullptr) {
    const int d = 2 * m;
    std::vector<dd> L((size_t)d * d), rinv;
    for (int a = 0; a < d; a++)
        for (int b = 0; b <= a; b++) {
            dd v = sigq(cov, m, a, b);
            L[(size_t)a * d + b] = v;
            L[(size_t)b * d + a] = v;
        }
    if (!dd_cholesky(L, d, rinv, nullptr)) return fail(TOR_ENOTPD, "sigma_Q is not positive definite");
    std::vector<dd> Mi((size_t)d * d, dd_from(0.0));
    for (int c = 0; c < d; c++) {
        Mi[(size_t)c * d + c] = rinv[c];
        for (int i = c + 1; i < d; i++) {
            dd acc = dd_from(0.0);
            for (int t = c; t < i; t++) acc = dd_add(acc, dd_mul(L[(size_t)i * d + t], Mi[(size_t)t * d + c]));
            Mi[(size_t)i * d + c] = dd_neg(dd_mul(acc, rinv[i]));
        }
    }
    koff.assign(m + 1, 0);
    for (int j = 0; j < m; j++) koff[j + 1] = koff[j] + (unsigned long long)(2 * j + 2) * (2 * j + 2);
    K.assign(koff[m], 0.0);
    // displaced states: h_j = K_j mu[0..2j+1] = sum_{t < 2j+2} M[t]^T (M[t] . mu),
    // accumulated row pair by row pair like K_j (z_t = M[t] . mu)
    std::vector<dd> z, hacc;
    if (mean) {
        z.assign(d, dd_from(0.0));
        for (int t = 0; t < d; t++)
            for (int b = 0; b <= t; b++) z[t] = dd_add(z[t], dd_mul(Mi[(size_t)t * d + b], dd_from(mean[b])));
        hacc.assign(d, dd_from(0.0));
        hoff->assign(m + 1, 0);
        for (int j = 0; j < m; j++) (*hoff)[j + 1] = (*hoff)[j] + (unsigned long long)(2 * j + 2);
        H->assign((*hoff)[m], 0.0);
        if (Hlo) Hlo->assign((*hoff)[m], 0.0);
    }
    if (Klo) Klo->assign(koff[m], 0.0);
    std::vector<dd> acc((size_t)d * d, dd_from(0.0));
    for (int j = 0; j < m; j++) {
        const int D = 2 * j + 2;
        for (int t = 2 * j; t < D; t++) {
            for (int a = 0; a <= t; a++)
                for (int b = 0; b <= a; b++)
                    acc[(size_t)a * d + b] =
                        dd_add(acc[(size_t)a * d + b], dd_mul(Mi[(size_t)t * d + a], Mi[(size_t)t * d + b]));
            if (mean)
                for (int a = 0; a <= t; a++) hacc[a] = dd_add(hacc[a], dd_mul(Mi[(size_t)t * d + a], z[t]));
        }
        // binary64 words: hi + lo rounded once; low words (double-double
        // terms): the exact remainder, so that word + low word is the
        // double-double value
        if (mean)
            for (int a = 0; a < D; a++) {
                double w, r;
                two_sum(hacc[a].hi, hacc[a].lo, w, r);
                (*H)[(*hoff)[j] + a] = w;
                if (Hlo) (*Hlo)[(*hoff)[j] + a] = r;
            }
        double *Kj = K.data() + koff[j];
        double *Klj = Klo ? Klo->data() + koff[j] : nullptr;
        for (int a = 0; a < D; a++)
            for (int b = 0; b <= a; b++) {
                dd v = acc[(size_t)a * d + b];
                double w, r;
                two_sum(v.hi, v.lo, w, r);
                Kj[(size_t)a * D + b] = Kj[(size_t)b * D + a] = w;
                if (Klj) Klj[(size_t)a * D + b] = Klj[(size_t)b * D + a] = r;
            }
    }
    return TOR_OK;
}

tor_status upload_chain_tables(tor_ctx *ctx, const double *cov, int m, const double *mean = nullptr,
                               bool dd_terms = false) {
    std::vector<double> K, H, Klo, Hlo;
    std::vector<unsigned long long> koff, hoff;
    tor_status s = build_k_tables(cov, m, K, koff, mean, &H, &hoff, dd_terms ? &Klo : nullptr,
                                  dd_terms ? &Hlo : nullptr);
    if (s) return s;
    if (dd_terms) {
        if (ctx->klobuf.ensure(Klo.size() * sizeof(double)) != hipSuccess ||
            (mean && ctx->hlobuf.ensure(Hlo.size() * sizeof(double)) != hipSuccess))
            return fail(TOR_ENOMEM, "device allocation of the double-double K tables failed");
        HIP_TRY(hipMemcpyAsync(ctx->klobuf.p, Klo.data(), Klo.size() * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
        if (mean)
            HIP_TRY(hipMemcpyAsync(ctx->hlobuf.p, Hlo.data(), Hlo.size() * sizeof(double), hipMemcpyHostToDevice,
                                   ctx->stream));
    }
    if (mean) {
        if (ctx->hbuf.ensure(H.size() * sizeof(double)) != hipSuccess ||
            ctx->hoff.ensure(hoff.size() * sizeof(unsigned long long)) != hipSuccess)
            return fail(TOR_ENOMEM, "device allocation of the mean tables failed");
        HIP_TRY(hipMemcpyAsync(ctx->hbuf.p, H.data(), H.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->hoff.p, hoff.data(), hoff.size() * sizeof(unsigned long long),
                               hipMemcpyHostToDevice, ctx->stream));
    }
    if (ctx->kbuf.ensure(K.size() * sizeof(double)) != hipSuccess ||
        ctx->koff.ensure(koff.size() * sizeof(unsigned long long)) != hipSuccess)
        return fail(TOR_ENOMEM, "device allocation of the K tables failed");
    HIP_TRY(hipMemcpyAsync(ctx->kbuf.p, K.data(), K.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->koff.p, koff.data(), koff.size() * sizeof(unsigned long long),
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return TOR_OK;
}

tor_status check_sampler_args(const double *cov, int m, int n_post, const double *mean = nullptr,
                              bool displaced = false) {
    tor_status s = validate_cov(cov, m);
    if (s) return s;
    if (displaced && !mean) return fail(TOR_EINVAL, "mean is NULL");
    if (mean)
        for (int i = 0; i < 2 * m; i++)
            if (!std::isfinite(mean[i])) return fail(TOR_EINVAL, "mean[%d] is not finite", i);
    if (m > 1024) return fail(TOR_ETOOBIG, "m = %d > 1024 for the sampler", m);
    if (n_post > TOR_CHAIN_CLICKS) return fail(TOR_ETOOBIG, "n_post = %d > %d", n_post, TOR_CHAIN_CLICKS);
    if (n_post > m) return fail(TOR_EINVAL, "n_post > m");
    return TOR_OK;
}

tor_status run_chains(tor_ctx *ctx, int m, int n_post, uint64_t seed, long long begin, int nchains, bool trace,
                      bool displaced = false, bool dd_terms = false, bool steps = false) {
    const size_t nm = (size_t)nchains * (size_t)m;
    if (ctx->c_out.ensure(nm) != hipSuccess || ctx->c_status.ensure((size_t)nchains) != hipSuccess ||
        ctx->c_sub.ensure((size_t)nchains * sizeof(double)) != hipSuccess ||
        (trace && (ctx->c_tp.ensure(nm * sizeof(double)) != hipSuccess ||
                   ctx->c_tu.ensure(nm * sizeof(double)) != hipSuccess)) ||
        (steps && (ctx->c_tr.ensure(nm * sizeof(double)) != hipSuccess ||
                   ctx->c_tb.ensure(nm * sizeof(double)) != hipSuccess)))
        return fail(TOR_ENOMEM, "device allocation for %d chains failed", nchains);
    ChainParams P{};
    P.K = (const double *)ctx->kbuf.p;
    P.koff = (const unsigned long long *)ctx->koff.p;
    P.H = displaced ? (const double *)ctx->hbuf.p : nullptr;  // null selects the zero-mean kernels
    P.hoff = displaced ? (const unsigned long long *)ctx->hoff.p : nullptr;
    P.m = m;
    P.n_post = n_post;
    P.cap = n_post >= 0 ? n_post : ctx->chain_clicks;
    P.seed = seed;
    P.chain_begin = begin;
    P.nchains = nchains;
    P.outcome = (unsigned char *)ctx->c_out.p;
    P.status = (signed char *)ctx->c_status.p;
    P.trace_p = trace ? (double *)ctx->c_tp.p : nullptr;
    P.trace_u = trace ? (double *)ctx->c_tu.p : nullptr;
    P.subsets = (double *)ctx->c_sub.p;
    P.Klo = dd_terms ? (const double *)ctx->klobuf.p : nullptr;  // non-null selects double-double terms
    P.Hlo = dd_terms && displaced ? (const double *)ctx->hlobuf.p : nullptr;
    P.trace_r = steps ? (double *)ctx->c_tr.p : nullptr;
    P.trace_b = steps ? (double *)ctx->c_tb.p : nullptr;
    HIP_TRY(tor_launch_chains(P, 256 * 8, ctx->stream));
    return TOR_OK;
}

}  // namespace

namespace {

// The fixed-outcome chain with binary64 or double-double terms: the
// conditioning over the no-click steps in double-double with a device-side
// snapshot of the clicked block after every step, then every step's subset
// sum in shared launches (AUTO repeats in double-double the sums whose
// binary64 bound exceeds tol).  roots[k] holds snapshot k, qv the q of each
// no-click step, used[k] the term precision of step k.  With a mean vector
// every packed matrix carries the mean row first (displaced states): the
// conditioning moves the mean and q gains the mean-overlap factor.
tor_status chain_sums_dd(tor_ctx *ctx, const double *cov, const double *mean, int m, const std::vector<int> &g,
                         const std::vector<int> &seq, const int8_t *outcomes, int nn, tor_prec prec, double tol,
                         std::vector<std::vector<dd>> &roots, std::vector<SumIn> &in, std::vector<SumOut> &res,
                         std::vector<int> &used, std::vector<double> &qv) {
    const int nsteps = (int)seq.size(), nobs = nsteps, D = mean ? 1 : 0;
    const size_t EM = (size_t)EN(nobs, D);
    tor_status s = TOR_OK;
    // device buffer: matrix | acc (3) | q per no-click step (2 each) | snapshots | jobs
    std::vector<long long> snap_off(nsteps + 1), snap_n(nsteps + 1);
    size_t snap_tot = 0;
    {
        int c = 0;
        for (int k = 0; k < nsteps; k++) {
            if (outcomes[seq[k]] == 1) c++;
            snap_n[k] = c;
            snap_off[k] = (long long)snap_tot;
            snap_tot += (size_t)EN(c, D);
        }
    }
    const size_t o_acc = align_up(EM * sizeof(dd), 256);
    const size_t o_q = align_up(o_acc + 3 * sizeof(double), 256);
    const size_t o_snap = align_up(o_q + 2 * (size_t)std::max(nn, 1) * sizeof(double), 256);
    const size_t o_jobs = align_up(o_snap + snap_tot * sizeof(dd), 256);
    const size_t bytes = o_jobs + (size_t)std::max(nn, 1) * sizeof(CondJob);
    if (bytes > ctx->mem_budget) return fail(TOR_ENOMEM, "chain needs %.2f GB", bytes / 1e9);
    if (ctx->cond.ensure(bytes) != hipSuccess) return fail(TOR_ENOMEM, "device allocation failed");
    unsigned char *db = (unsigned char *)ctx->cond.p;
    dd *dmat = (dd *)db;
    std::vector<unsigned char> &stage = ctx->host_stage;
    if (stage.size() < bytes) stage.resize(bytes);
    dd *hm = (dd *)stage.data();
    if (D) hm[0] = dd_from(0.0);
    for (int a = 0; a < 2 * nobs; a++) {
        if (D) hm[pidx(a + 1, 0)] = dd_from(mean[g[a]]);
        for (int b = 0; b <= a; b++) hm[pidx(a + D, b + D)] = sigq(cov, m, g[a], g[b]);
    }
    const double a0[3] = {1.0, 0.0, 0.0};
    std::memcpy(stage.data() + o_acc, a0, sizeof a0);
    CondJob *hj = (CondJob *)(stage.data() + o_jobs);
    {
        int r = nobs, t = 0;
        for (int k = 0; k < nsteps; k++) {
            if (outcomes[seq[k]] == 1) continue;
            CondJob j{};
            j.mat = dmat;
            j.acc = (double *)(db + o_acc);
            j.qout = (double *)(db + o_q) + 2 * t;
            j.begin = 0;
            j.r = r;
            j.d = D;
            hj[t++] = j;
            r--;
        }
    }
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemcpyAsync(db, stage.data(), o_acc + 3 * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(db + o_jobs, stage.data() + o_jobs, (size_t)std::max(nn, 1) * sizeof(CondJob),
                           hipMemcpyHostToDevice, st));
    {
        int t = 0;
        for (int k = 0; k < nsteps; k++) {
            if (outcomes[seq[k]] == 0) {
                const CondJob &j = hj[t];
                const long long blocks =
                    std::max<long long>(1, (EN(j.r - 1, D) + TOR_COND_CHUNK - 1) / TOR_COND_CHUNK);
                HIP_TRY(tor_launch_condition((const CondJob *)(db + o_jobs) + t, 1, blocks, j.r, st));
                t++;
            }
            if (snap_n[k] > 0)
                HIP_TRY(hipMemcpyAsync(db + o_snap + snap_off[k] * sizeof(dd), dmat, sizeof(dd) * EN(snap_n[k], D),
                                       hipMemcpyDeviceToDevice, st));
        }
        ctx->stats.condition_launches += t;
    }
    HIP_TRY(hipMemcpyAsync(stage.data() + o_q, db + o_q, o_jobs - o_q, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    // the q of each no-click step, out of the staging buffer that the subset
    // sums below reuse
    qv.assign((const double *)(stage.data() + o_q), (const double *)(stage.data() + o_q) + 2 * (size_t)nn);
    // one subset sum per step over the clicks so far, all in shared launches
    std::vector<int> which;
    const dd *snaps = (const dd *)(stage.data() + o_snap);
    for (int k = 0; k < nsteps; k++) {
        in[k].n = (int)snap_n[k];
        in[k].D = D;
        if (snap_n[k] > 0) roots[k].assign(snaps + snap_off[k], snaps + snap_off[k] + EN(snap_n[k], D));
        else roots[k].assign((size_t)EN(0, D), dd_from(0.0));
        in[k].packed = &roots[k];
        which.push_back(k);
    }
    s = gpu_sums(ctx, in, which, prec == TOR_PREC_DD, res);
    if (s) return s;
    if (prec == TOR_PREC_AUTO) {
        std::vector<int> redo;
        for (int k = 0; k < nsteps; k++)
            if (in[k].n > 0 && !(bound_of(TOR_PREC_F64, in[k].n, res[k].T, res[k].A, quad_of(roots[k], in[k].n, D)) <= tol))
                redo.push_back(k);
        if (!redo.empty()) {
            s = gpu_sums(ctx, in, redo, true, res);
            if (s) return s;
            for (int k : redo) used[k] = TOR_PREC_DD;
        }
    }
    return TOR_OK;
}

// The fixed-outcome chain with quad-double terms: the conditioning over the
// no-click steps in quad-double with a snapshot of the clicked block after
// every step, then one quad-double subset sum per step.  roots[k] keeps the
// double-double rounding of snapshot k (for the final log det); qv the q of
// each no-click step.
tor_status chain_sums_qd(tor_ctx *ctx, const double *cov, const double *mean, int m, const std::vector<int> &g,
                         const std::vector<int> &seq, const int8_t *outcomes, int nn,
                         std::vector<std::vector<dd>> &roots, std::vector<SumIn> &in, std::vector<SumOut> &res,
                         std::vector<double> &qv) {
    const int nsteps = (int)seq.size(), nobs = nsteps, D = mean ? 1 : 0;  // D: the mean row first
    const size_t words = (size_t)EN(nobs, D);
    const size_t cols_off = align_up(words * sizeof(qd), 256);
    const size_t cols_words = 2 * (2 * (size_t)nobs - 2 + D) + 2;
    const size_t acc_off = align_up(cols_off + cols_words * sizeof(qd), 256);
    const size_t q_off = align_up(acc_off + 3 * sizeof(double), 256);
    const size_t job_off = align_up(q_off + 2 * (size_t)std::max(nn, 1) * sizeof(double), 256);
    const size_t total_bytes = job_off + (size_t)std::max(nn, 1) * sizeof(CondJobQ);
    if (total_bytes > ctx->mem_budget) return fail(TOR_ENOMEM, "chain needs %.2f GB", total_bytes / 1e9);
    if (ctx->cond.ensure(total_bytes) != hipSuccess) return fail(TOR_ENOMEM, "device allocation failed");
    unsigned char *db = (unsigned char *)ctx->cond.p;
    std::vector<unsigned char> stage(total_bytes);
    qd *hm = (qd *)stage.data();
    if (D) hm[0] = qd_from(0.0);
    for (int a = 0; a < 2 * nobs; a++) {
        if (D) hm[pidx(a + 1, 0)] = qd_from(mean[g[a]]);
        for (int b = 0; b <= a; b++) hm[pidx(a + D, b + D)] = qd_from_dd(sigq(cov, m, g[a], g[b]));
    }
    const double a0[3] = {1.0, 0.0, 0.0};
    std::memcpy(stage.data() + acc_off, a0, sizeof a0);
    CondJobQ *hj = (CondJobQ *)(stage.data() + job_off);
    for (int k = 0, t = 0, r = nobs; k < nsteps; k++) {
        if (outcomes[seq[k]] == 1) continue;
        CondJobQ j{};
        j.mat = db;
        j.acc = (double *)(db + acc_off);
        j.cols = db + cols_off;
        j.qout = (double *)(db + q_off) + 2 * t;
        j.r = r--;
        j.d = D;
        hj[t++] = j;
    }
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemcpyAsync(db, stage.data(), total_bytes, hipMemcpyHostToDevice, st));
    std::vector<std::vector<qd>> snaps(nsteps);
    std::vector<int> snap_n(nsteps);
    int c = 0, t = 0;
    for (int k = 0; k < nsteps; k++) {
        if (outcomes[seq[k]] == 1) {
            c++;
        } else {
            const long long blocks =
                std::max<long long>(1, (EN(hj[t].r - 1, D) + TOR_COND_CHUNK - 1) / TOR_COND_CHUNK);
            HIP_TRY(tor_launch_condition_qd((const CondJobQ *)(db + job_off) + t, 1, blocks, st));
            t++;
        }
        snap_n[k] = c;
        snaps[k].assign((size_t)EN(c, D), qd_from(0.0));
        if (c > 0)
            HIP_TRY(hipMemcpyAsync(snaps[k].data(), db, snaps[k].size() * sizeof(qd), hipMemcpyDeviceToHost, st));
    }
    qv.assign(2 * (size_t)nn, 0.0);
    if (nn > 0) HIP_TRY(hipMemcpyAsync(qv.data(), db + q_off, 2 * (size_t)nn * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    ctx->stats.condition_launches += 2 * (int64_t)t;
    for (int k = 0; k < nsteps; k++) {
        const int n = snap_n[k];
        in[k].n = n;
        roots[k].resize(snaps[k].size());
        for (size_t e = 0; e < snaps[k].size(); e++) roots[k][e] = qd_to_dd(snaps[k][e]);
        in[k].packed = &roots[k];
        in[k].D = D;
        tor_status s = gpu_sum_qd(ctx, snaps[k], n, res[k], D);
        if (s) return s;
    }
    return TOR_OK;
}

}  // namespace

extern "C" {

// gbs_sample and its displaced form (mean != NULL)
static tor_status sample_impl(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                              uint64_t seed, int32_t n_samples, uint8_t *samples, gbs_stats *stats) {
    if (!ctx) return fail(TOR_EINVAL, "ctx is NULL");
    if (n_samples < 0 || (n_samples > 0 && !samples)) return fail(TOR_EINVAL, "bad samples buffer");
    tor_status s = check_sampler_args(cov, m, n_post, mean, mean != nullptr);
    if (s) return s;
    HIP_TRY(hipSetDevice(ctx->device));
    auto t0 = std::chrono::steady_clock::now();
    const bool dd_terms = ctx->chain_prec == TOR_PREC_DD;
    s = upload_chain_tables(ctx, cov, m, mean, dd_terms);
    if (s) return s;
    const int NB = 16384;
    std::vector<unsigned char> out((size_t)NB * m);
    std::vector<signed char> st(NB);
    std::vector<double> sub(NB);
    long long begin = 0, consumed = 0, evaluated = 0, capped = 0;
    double subsets = 0.0;
    int got = 0;
    while (got < n_samples) {
        if (begin >= (1LL << 31)) return fail(TOR_EAGAIN, "no %d accepted samples within 2^31 chains", n_samples);
        s = run_chains(ctx, m, n_post, seed, begin, NB, false, mean != nullptr, dd_terms);
        if (s) return s;
        HIP_TRY(hipMemcpyAsync(out.data(), ctx->c_out.p, out.size(), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipMemcpyAsync(st.data(), ctx->c_status.p, st.size(), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipMemcpyAsync(sub.data(), ctx->c_sub.p, sub.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        evaluated += NB;
        for (int i = 0; i < NB && got < n_samples; i++) {
            consumed++;
            subsets += sub[i];
            if (st[i] == 2) capped++;
            if (st[i] == 1) {
                std::memcpy(samples + (size_t)got * m, out.data() + (size_t)i * m, (size_t)m);
                got++;
            }
        }
        begin += NB;
    }
    if (stats) {
        stats->chains_started = consumed;
        stats->chains_accepted = got;
        stats->chains_evaluated = evaluated;
        stats->chains_capped = capped;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->subsets = subsets;
    }
    return TOR_OK;
}

tor_status gbs_sample(tor_ctx *ctx, const double *cov, int32_t m, int32_t n_post, uint64_t seed,
                      int32_t n_samples, uint8_t *samples, gbs_stats *stats) {
    return sample_impl(ctx, cov, nullptr, m, n_post, seed, n_samples, samples, stats);
}

tor_status gbs_sample_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                                uint64_t seed, int32_t n_samples, uint8_t *samples, gbs_stats *stats) {
    if (!mean) return fail(TOR_EINVAL, "mean is NULL");
    return sample_impl(ctx, cov, mean, m, n_post, seed, n_samples, samples, stats);
}

// gbs_chain_fixed and its displaced form (mean != NULL)
static tor_status chain_fixed_impl(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                   const int8_t *outcomes, tor_prec prec, double tol, double *step_p,
                                   tor_result *total) {
    if (!ctx || !total) return fail(TOR_EINVAL, "NULL argument");
    if (prec != TOR_PREC_AUTO && prec != TOR_PREC_F64 && prec != TOR_PREC_DD && prec != TOR_PREC_QD)
        return fail(TOR_EINVAL, "bad precision %d", (int)prec);
    if (!(tol > 0.0)) tol = 1e-10;
    tor_status s = validate_cov_block(cov, m, outcomes);
    if (s) return s;
    const int D = mean ? 1 : 0;
    if (mean)
        for (int j = 0; j < m; j++)
            if (outcomes[j] >= 0 && !(std::isfinite(mean[2 * j]) && std::isfinite(mean[2 * j + 1])))
                return fail(TOR_EINVAL, "mean of mode %d is not finite", j);
    // measurement sequence: modes m-1 .. 0 with an outcome; order of the matrix:
    // clicked modes in measurement order, then the no-click modes in reverse
    // measurement order (each no-click step conditions on the last mode)
    std::vector<int> seq, clicks, noclicks;
    for (int j = m - 1; j >= 0; j--) {
        if (outcomes[j] < 0) continue;
        seq.push_back(j);
        if (outcomes[j] == 1) clicks.push_back(j);
        else noclicks.push_back(j);
    }
    const int nc = (int)clicks.size(), nn = (int)noclicks.size(), nobs = nc + nn;
    if (nc > TOR_MAX_CLICKS) return fail(TOR_ETOOBIG, "%d clicks > %d", nc, TOR_MAX_CLICKS);
    if (nobs > TOR_COND_MAX_MODES) return fail(TOR_ETOOBIG, "%d observed modes > %d", nobs, TOR_COND_MAX_MODES);
    HIP_TRY(hipSetDevice(ctx->device));
    if (step_p)
        for (int j = 0; j < m; j++) step_p[j] = 1.0;
    std::memset(total, 0, sizeof *total);
    if (nobs == 0) {
        total->p = 1.0;
        total->status = TOR_OK;
        return TOR_OK;
    }
    std::vector<int> g;  // quadrature index per row of the ordered matrix
    for (int c : clicks) {
        g.push_back(2 * c);
        g.push_back(2 * c + 1);
    }
    for (auto it = noclicks.rbegin(); it != noclicks.rend(); ++it) {
        g.push_back(2 * *it);
        g.push_back(2 * *it + 1);
    }
    const int nsteps = nobs;
    std::vector<std::vector<dd>> roots(nsteps);
    std::vector<SumIn> in(nsteps);
    std::vector<SumOut> res(nsteps);
    std::vector<int> used(nsteps, prec == TOR_PREC_QD ? TOR_PREC_QD : prec == TOR_PREC_DD ? TOR_PREC_DD : TOR_PREC_F64);
    std::vector<double> qv;
    if (prec == TOR_PREC_QD) {
        s = chain_sums_qd(ctx, cov, mean, m, g, seq, outcomes, nn, roots, in, res, qv);
    } else {
        s = chain_sums_dd(ctx, cov, mean, m, g, seq, outcomes, nn, prec, tol, roots, in, res, used, qv);
    }
    if (s) return s;
    // step probabilities: click T_k / T_{k-1}; no click q T_k / T_{k-1}
    const double *hq = qv.data();
    dd prev = dd_from(1.0), pvac = dd_from(1.0);
    double worst_bound = 0.0, worst_R = 0.0, log_pvac = 0.0;
    int worst_used = TOR_PREC_F64;
    for (int k = 0, t = 0; k < nsteps; k++) {
        const dd T = res[k].T;
        if (!std::isfinite(T.hi) || !std::isfinite(res[k].A)) return fail(TOR_ENOTPD, "a Schur pivot was not positive");
        dd num = T;
        if (outcomes[seq[k]] == 0) {
            const dd q = dd_make(hq[2 * t], hq[2 * t + 1]);
            num = dd_mul(q, T);
            pvac = dd_mul(pvac, q);
            log_pvac += std::log(q.hi) + std::log1p(q.lo / q.hi);
            t++;
        }
        if (step_p) step_p[seq[k]] = (num.hi + num.lo) / (prev.hi + prev.lo);
        if (in[k].n > 0) {
            // the step's sum is over the matrix after t conditioning steps
            const double cu = t * (prec == TOR_PREC_QD ? kUQD : kUDD);
            worst_bound =
                std::max(worst_bound, bound_of(used[k], in[k].n, T, res[k].A, quad_of(roots[k], in[k].n, D), cu));
            worst_R = std::max(worst_R, res[k].A / std::fabs(T.hi));
            worst_used = std::max(worst_used, used[k]);
        }
        prev = T;
    }
    // the whole pattern telescopes to P_vac(N) * T(clicks | N), as tor_probability
    const dd pr = dd_mul(pvac, prev);
    total->p = pr.hi + pr.lo;
    total->p_lo = pr.lo - (total->p - pr.hi);
    total->log_p = total->p > 0 ? log_pvac + std::log(prev.hi) + std::log1p(prev.lo / prev.hi) : -INFINITY;
    total->T = prev.hi;
    total->T_lo = prev.lo;
    total->abs_sum = res[nsteps - 1].A;
    total->cancel_ratio = worst_R;
    total->rel_err_bound = 2.0 * worst_bound;  // a step is a ratio of two sums
    total->log_pvac_n = log_pvac;
    if (nc > 0) {  // Tor of the final conditioned matrix (log det from its packed snapshot)
        std::vector<dd> full((size_t)4 * nc * nc);
        const std::vector<dd> &pk = roots[nsteps - 1];
        for (int a = 0; a < 2 * nc; a++)
            for (int b = 0; b <= a; b++)
                full[(size_t)a * 2 * nc + b] = full[(size_t)b * 2 * nc + a] = pk[pidx(a + D, b + D)];
        double ld = 0.0;
        if (f64_cholesky_logdet(full, 2 * nc, &ld)) total->tor = std::exp(0.5 * ld) * (prev.hi + prev.lo);
    } else {
        total->tor = 1.0;
    }
    total->n_clicks = nc;
    total->prec_used = worst_used;
    total->status = total->rel_err_bound <= tol ? TOR_OK : TOR_WARN_PRECISION;
    return total->status;
}

tor_status gbs_chain_fixed(tor_ctx *ctx, const double *cov, int32_t m, const int8_t *outcomes, tor_prec prec,
                           double tol, double *step_p, tor_result *total) {
    return chain_fixed_impl(ctx, cov, nullptr, m, outcomes, prec, tol, step_p, total);
}

tor_status gbs_chain_fixed_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                     const int8_t *outcomes, tor_prec prec, double tol, double *step_p,
                                     tor_result *total) {
    if (!mean) return fail(TOR_EINVAL, "mean is NULL");
    return chain_fixed_impl(ctx, cov, mean, m, outcomes, prec, tol, step_p, total);
}

// gbs_trace and its displaced form (mean != NULL)
static tor_status trace_impl(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                             uint64_t seed, int64_t chain_begin, int32_t nchains, double *p_click, double *uniform,
                             uint8_t *outcome, int8_t *status, double *cancel_ratio = nullptr,
                             double *err_bound = nullptr) {
    if (!ctx) return fail(TOR_EINVAL, "ctx is NULL");
    if (nchains < 0 || chain_begin < 0) return fail(TOR_EINVAL, "bad chain range");
    tor_status s = check_sampler_args(cov, m, n_post, mean, mean != nullptr);
    if (s) return s;
    if (nchains == 0) return TOR_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    const bool dd_terms = ctx->chain_prec == TOR_PREC_DD, steps = cancel_ratio || err_bound;
    s = upload_chain_tables(ctx, cov, m, mean, dd_terms);
    if (s) return s;
    s = run_chains(ctx, m, n_post, seed, chain_begin, nchains, true, mean != nullptr, dd_terms, steps);
    if (s) return s;
    const size_t nm = (size_t)nchains * m;
    if (cancel_ratio)
        HIP_TRY(hipMemcpyAsync(cancel_ratio, ctx->c_tr.p, nm * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (err_bound)
        HIP_TRY(hipMemcpyAsync(err_bound, ctx->c_tb.p, nm * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (p_click)
        HIP_TRY(hipMemcpyAsync(p_click, ctx->c_tp.p, nm * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (uniform)
        HIP_TRY(hipMemcpyAsync(uniform, ctx->c_tu.p, nm * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (outcome) HIP_TRY(hipMemcpyAsync(outcome, ctx->c_out.p, nm, hipMemcpyDeviceToHost, ctx->stream));
    if (status) HIP_TRY(hipMemcpyAsync(status, ctx->c_status.p, (size_t)nchains, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return TOR_OK;
}

tor_status gbs_trace(tor_ctx *ctx, const double *cov, int32_t m, int32_t n_post, uint64_t seed,
                     int64_t chain_begin, int32_t nchains, double *p_click, double *uniform, uint8_t *outcome,
                     int8_t *status) {
    return trace_impl(ctx, cov, nullptr, m, n_post, seed, chain_begin, nchains, p_click, uniform, outcome, status);
}

tor_status gbs_trace_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                               uint64_t seed, int64_t chain_begin, int32_t nchains, double *p_click,
                               double *uniform, uint8_t *outcome, int8_t *status) {
    if (!mean) return fail(TOR_EINVAL, "mean is NULL");
    return trace_impl(ctx, cov, mean, m, n_post, seed, chain_begin, nchains, p_click, uniform, outcome, status);
}

tor_status gbs_trace_steps(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                           uint64_t seed, int64_t chain_begin, int32_t nchains, double *p_click, double *uniform,
                           uint8_t *outcome, int8_t *status, double *cancel_ratio, double *err_bound) {
    return trace_impl(ctx, cov, mean, m, n_post, seed, chain_begin, nchains, p_click, uniform, outcome, status,
                      cancel_ratio, err_bound);
}

}  // extern "C"

// ------------------------------------------------------------------ server
//
// Continuous batching: each worker owns a context (its own stream and device
// buffers).  A free worker takes the oldest pending requests that fit its
// memory budget (and the batch cap), evaluates them as one fused batch, and
// publishes the results; requests that arrive meanwhile wait for the next free
// worker, so batches of different workers overlap on the device.  Every result
// is bitwise the same as the query evaluated alone (see tor_batch).

namespace {

struct ServerReq {
    Reduced red;     // patterns with no-click modes: conditioned by the worker
    Prepared prep;
    std::vector<int8_t> pattern;   // quad-double servers: the query itself, evaluated alone
    const tor_state *st = nullptr;
    std::chrono::steady_clock::time_point t_submit, t_done;
    tor_result res;
    bool done = false;
};

}  // namespace

struct tor_server {
    tor_ctx *parent = nullptr;
    tor_server_opts opts{};
    std::vector<tor_ctx *> wctx;
    std::vector<std::thread> threads;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, std::unique_ptr<ServerReq>> reqs;
    uint64_t next_ticket = 1;
    bool stopping = false;
    tor_server_stats stats{};
};

namespace {

void server_worker(tor_server *S, int w) {
    tor_ctx *ctx = S->wctx[w];
    (void)hipSetDevice(ctx->device);
    const size_t es = S->opts.prec == TOR_PREC_F64 ? sizeof(double) : sizeof(dd);
    for (;;) {
        std::vector<uint64_t> take;
        std::vector<Prepared> batch;
        std::vector<Reduced> red;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stopping || !S->pending.empty(); });
            if (S->pending.empty()) return;  // stopping and drained
            size_t bytes = 0;
            // quad-double queries are taken one at a time so that the workers share them
            const int most = S->opts.prec == TOR_PREC_QD ? 1 : S->opts.max_batch;
            while (!S->pending.empty() && (int)take.size() < most) {
                uint64_t t = S->pending.front();
                ServerReq &r = *S->reqs[t];
                size_t b = sum_bytes(r.red.n, task_modes_for(ctx, S->opts.prec == TOR_PREC_DD, r.red.n), es,
                                     r.red.D) +
                           cond_words(&r.red) * sizeof(dd);
                if (!take.empty() && bytes + b > S->opts.mem_budget_bytes) break;
                bytes += b;
                take.push_back(t);
                batch.push_back(std::move(r.prep));
                red.push_back(std::move(r.red));
                S->pending.pop_front();
            }
        }
        if (S->opts.prec == TOR_PREC_QD) {  // quad-double: the single-query paths, one at a time
            std::vector<std::pair<const tor_state *, std::vector<int8_t>>> qq;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                for (uint64_t t : take) qq.emplace_back(S->reqs[t]->st, std::move(S->reqs[t]->pattern));
            }
            std::vector<tor_result> out(take.size());
            for (size_t i = 0; i < qq.size(); i++) {
                const tor_state *st = qq[i].first;
                const int8_t *pat = qq[i].second.data();
                std::memset(&out[i], 0, sizeof out[i]);
                tor_status s = st->mean.empty()
                                   ? probability_qd(ctx, st->cov.data(), st->m, pat, S->opts.tol, &out[i], st)
                                   : probability_qd_disp(ctx, st->cov.data(), st->mean.data(), st->m, pat,
                                                         S->opts.tol, &out[i], st);
                if (s < 0) {
                    std::memset(&out[i], 0, sizeof out[i]);
                    out[i].status = s;
                }
            }
            auto now = std::chrono::steady_clock::now();
            {
                std::lock_guard<std::mutex> lk(S->mu);
                for (size_t i = 0; i < take.size(); i++) {
                    ServerReq &r = *S->reqs[take[i]];
                    r.res = out[i];
                    r.t_done = now;
                    r.done = true;
                }
                S->stats.batches += 1;
                S->stats.completed += (int64_t)take.size();
                S->stats.max_batch_seen = std::max<int64_t>(S->stats.max_batch_seen, (int64_t)take.size());
            }
            S->cv_done.notify_all();
            continue;
        }
        // no-click conditioning of the batch's full patterns, then their checks
        std::vector<Reduced *> rp;
        for (Reduced &x : red)
            if (x.cond) rp.push_back(&x);
        if (!rp.empty()) {
            tor_status cs = condition_on_gpu(ctx, rp);
            for (size_t i = 0; i < batch.size(); i++) {
                if (!red[i].cond && rp.end() == std::find(rp.begin(), rp.end(), &red[i])) continue;
                tor_status s = cs < 0 ? cs : prepare_reduced(red[i], batch[i]);
                if (s != TOR_OK) {
                    batch[i].status = s;
                    batch[i].n = 0;
                }
            }
        }
        std::vector<tor_result> out(batch.size());
        (void)evaluate_many(ctx, batch, S->opts.prec, S->opts.tol, out.data());
        auto now = std::chrono::steady_clock::now();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (size_t i = 0; i < take.size(); i++) {
                ServerReq &r = *S->reqs[take[i]];
                r.res = out[i];
                r.t_done = now;
                r.done = true;
            }
            S->stats.batches += 1;
            S->stats.completed += (int64_t)take.size();
            S->stats.max_batch_seen = std::max<int64_t>(S->stats.max_batch_seen, (int64_t)take.size());
        }
        S->cv_done.notify_all();
    }
}

tor_status take_result(tor_server *S, uint64_t ticket, tor_result *out, double *latency_s) {
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(TOR_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    ServerReq &r = *it->second;
    if (out) *out = r.res;
    if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    tor_status st = r.res.status;
    S->reqs.erase(it);
    return st;
}

}  // namespace

extern "C" {

tor_status tor_server_start(tor_ctx *ctx, const tor_server_opts *opts, tor_server **out) {
    if (!ctx || !out) return fail(TOR_EINVAL, "NULL argument");
    *out = nullptr;
    tor_server_opts o;
    o.workers = 2;
    o.max_pending = 1 << 16;
    o.mem_budget_bytes = (size_t)16 << 30;
    o.prec = TOR_PREC_DD;
    o.tol = 1e-10;
    o.max_batch = 4096;
    if (opts) {
        if (opts->workers > 0) o.workers = opts->workers;
        if (opts->max_pending > 0) o.max_pending = opts->max_pending;
        if (opts->mem_budget_bytes > 0) o.mem_budget_bytes = opts->mem_budget_bytes;
        o.prec = opts->prec;
        if (opts->tol > 0) o.tol = opts->tol;
        if (opts->max_batch > 0) o.max_batch = opts->max_batch;
    }
    if (o.workers > 16) return fail(TOR_EINVAL, "at most 16 workers");
    if (o.prec != TOR_PREC_AUTO && o.prec != TOR_PREC_F64 && o.prec != TOR_PREC_DD && o.prec != TOR_PREC_QD)
        return fail(TOR_EINVAL, "bad precision");
    tor_server *S = new (std::nothrow) tor_server();
    if (!S) return fail(TOR_ENOMEM, "host allocation failed");
    S->parent = ctx;
    S->opts = o;
    for (int w = 0; w < o.workers; w++) {
        tor_ctx *c = nullptr;
        tor_status st = tor_ctx_create(ctx->device, &c);
        if (st) {
            for (tor_ctx *x : S->wctx) tor_ctx_destroy(x);
            delete S;
            return st;
        }
        c->task_modes[0] = ctx->task_modes[0];
        c->task_modes[1] = ctx->task_modes[1];
        std::memcpy(c->tuned, ctx->tuned, sizeof c->tuned);
        c->wave_grid = ctx->wave_grid;
        c->mem_budget = std::max(ctx->mem_budget, o.mem_budget_bytes);
        S->wctx.push_back(c);
    }
    for (int w = 0; w < o.workers; w++) S->threads.emplace_back(server_worker, S, w);
    *out = S;
    return TOR_OK;
}

tor_status tor_submit(tor_server *S, const tor_state *st, const int8_t *pattern, uint64_t *ticket) {
    if (!S || !st || !pattern || !ticket) return fail(TOR_EINVAL, "NULL argument");
    auto t0 = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) return fail(TOR_EINVAL, "server is stopping");
        if ((int)S->pending.size() >= S->opts.max_pending) return fail(TOR_EAGAIN, "queue full");
    }
    std::unique_ptr<ServerReq> r(new (std::nothrow) ServerReq());
    if (!r) return fail(TOR_ENOMEM, "host allocation failed");
    r->t_submit = t0;
    tor_status s = reduce_for_state(st, pattern, r->red);  // validates the pattern
    if (s) return s;
    if (S->opts.prec == TOR_PREC_QD) {  // evaluated alone by a worker from the pattern itself
        r->pattern.assign(pattern, pattern + st->m);
        r->st = st;
        r->red = Reduced();
        std::lock_guard<std::mutex> lk(S->mu);
        if ((int)S->pending.size() >= S->opts.max_pending) return fail(TOR_EAGAIN, "queue full");
        uint64_t t = S->next_ticket++;
        S->reqs.emplace(t, std::move(r));
        S->pending.push_back(t);
        S->stats.submitted += 1;
        *ticket = t;
        S->cv_work.notify_one();
        return TOR_OK;
    }
    const int n = r->red.n, D = r->red.D;
    if (!r->red.cond) {  // marginal pattern: ready now (conditioned ones: in the worker)
        s = prepare_reduced(r->red, r->prep);
        if (s) return s;
        std::vector<dd>().swap(r->red.sig);
    }
    const size_t es = S->opts.prec == TOR_PREC_F64 ? sizeof(double) : sizeof(dd);
    if (sum_bytes(n, task_modes_for(S->wctx[0], S->opts.prec == TOR_PREC_DD, n), es, D) > S->wctx[0]->mem_budget)
        return fail(TOR_ENOMEM, "query with %d clicks exceeds the device memory budget", n);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if ((int)S->pending.size() >= S->opts.max_pending) return fail(TOR_EAGAIN, "queue full");
        uint64_t t = S->next_ticket++;
        S->reqs.emplace(t, std::move(r));
        S->pending.push_back(t);
        S->stats.submitted += 1;
        *ticket = t;
    }
    S->cv_work.notify_one();
    return TOR_OK;
}

tor_status tor_poll(tor_server *S, uint64_t ticket, tor_result *out, double *latency_s) {
    if (!S) return fail(TOR_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(TOR_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) return TOR_EAGAIN;
    return take_result(S, ticket, out, latency_s);
}

tor_status tor_wait(tor_server *S, uint64_t ticket, tor_result *out, double *latency_s) {
    if (!S) return fail(TOR_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(TOR_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    ServerReq *r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done; });
    return take_result(S, ticket, out, latency_s);
}

tor_status tor_server_get_stats(tor_server *S, tor_server_stats *out) {
    if (!S || !out) return fail(TOR_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->pending = (int64_t)S->pending.size();
    return TOR_OK;
}

tor_status tor_server_stop(tor_server *S) {
    if (!S) return fail(TOR_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->threads) t.join();
    for (tor_ctx *c : S->wctx) tor_ctx_destroy(c);
    delete S;
    return TOR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotuner
//
// Picks the wave-tier task size J (modes per task) for each tree size n by
// timing the candidates on a synthetic SPD matrix with the same structure as
// the workloads (2x2 mode blocks, moderate conditioning).  The choice depends
// only on (precision, n), so a query's result never depends on the other
// queries of a batch.

namespace {

std::vector<dd> synthetic_sigma(int n) {
    // sigma = I + B B^T / (2n) with B from a fixed linear congruential stream
    const int d = 2 * n;
    std::vector<double> B((size_t)d * d);
    unsigned s = 2024u;
    for (auto &b : B) {
        s = s * 1664525u + 1013904223u;
        b = ((s >> 8) & 0xffffff) / 16777216.0 - 0.5;
    }
    std::vector<dd> sig((size_t)d * d);
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double v = i == j ? 1.0 : 0.0;
            for (int k = 0; k < d; k++) v += B[(size_t)i * d + k] * B[(size_t)j * d + k] / (2.0 * n);
            sig[(size_t)i * d + j] = dd_from(v);
        }
    return sig;
}

// The context's tuning table as JSON: task sizes of the batched path
// ("dd:24": 10) and unit depths of the persistent kernel ("pst:24": 2).
tor_status write_tuning(const tor_ctx *ctx, const char *path) {
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(TOR_EINVAL, "cannot write %s", path);
    hipDeviceProp_t prop;
    (void)hipGetDeviceProperties(&prop, ctx->device);
    std::fprintf(f, "{\"arch\": \"%s\", \"task_modes\": {", prop.gcnArchName);
    bool first = true;
    for (int sl = 0; sl < 2; sl++)
        for (int n = 0; n <= TOR_MAX_CLICKS; n++)
            if (ctx->tuned[sl][n] > 0) {
                std::fprintf(f, "%s\"%s:%d\": %d", first ? "" : ", ", sl ? "dd" : "f64", n, ctx->tuned[sl][n]);
                first = false;
            }
    std::fprintf(f, "}, \"persistent_unit_levels\": {");
    first = true;
    for (int n = 0; n <= TOR_MAX_CLICKS; n++)
        if (ctx->ps_t1[n] > 0) {
            std::fprintf(f, "%s\"pst:%d\": %d", first ? "" : ", ", n, ctx->ps_t1[n] - 1);
            first = false;
        }
    std::fprintf(f, "}}\n");
    std::fclose(f);
    return TOR_OK;
}

}  // namespace

extern "C" {

tor_status tor_autotune(tor_ctx *ctx, tor_prec prec, int32_t n_lo, int32_t n_hi, const char *cache_path) {
    if (!ctx) return fail(TOR_EINVAL, "ctx is NULL");
    if (prec != TOR_PREC_F64 && prec != TOR_PREC_DD) return fail(TOR_EINVAL, "tune TOR_PREC_F64 or TOR_PREC_DD");
    if (n_lo < 1 || n_hi > TOR_MAX_CLICKS || n_lo > n_hi) return fail(TOR_EINVAL, "bad n range");
    HIP_TRY(hipSetDevice(ctx->device));
    const bool use_dd = prec == TOR_PREC_DD;
    const int slot = use_dd ? 1 : 0;
    for (int n = n_lo; n <= n_hi; n++) {
        Prepared p;
        tor_status s = prepare(synthetic_sigma(n), n, dd_from(1.0), 0.0, p);
        if (s) return s;
        std::vector<SumIn> in(1);
        in[0].packed = &p.packed;
        in[0].n = n;
        std::vector<int> which{0};
        std::vector<SumOut> out(1);
        int best = std::min(n, TOR_TASK_MAX);
        double best_t = 1e300;
        for (int J = std::min(n, TOR_TASK_MAX); J >= std::max(1, std::min(n, 6)); J--) {
            ctx->tuned[slot][n] = J;
            s = gpu_sums(ctx, in, which, use_dd, out);  // warm
            if (s) return s;
            const int reps = n <= 20 ? 5 : (n <= 26 ? 3 : 1);
            auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < reps; r++) {
                s = gpu_sums(ctx, in, which, use_dd, out);
                if (s) return s;
            }
            double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / reps;
            if (t < best_t) {
                best_t = t;
                best = J;
            }
            if (J == n) break;
        }
        ctx->tuned[slot][n] = best;
    }
    if (cache_path && *cache_path) return write_tuning(ctx, cache_path);
    return TOR_OK;
}

tor_status tor_load_tuning(tor_ctx *ctx, const char *cache_path) {
    if (!ctx || !cache_path) return fail(TOR_EINVAL, "NULL argument");
    FILE *f = std::fopen(cache_path, "r");
    if (!f) return fail(TOR_EINVAL, "cannot read %s", cache_path);
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, k);
    std::fclose(f);
    // entries look like "dd:24": 9
    int loaded = 0;
    for (size_t pos = 0; (pos = txt.find('"', pos)) != std::string::npos;) {
        size_t end = txt.find('"', pos + 1);
        if (end == std::string::npos) break;
        std::string key = txt.substr(pos + 1, end - pos - 1);
        pos = end + 1;
        if (key.rfind("pst:", 0) == 0) {  // persistent kernel: depth-first levels per unit
            const int n = std::atoi(key.c_str() + 4);
            const size_t colon = txt.find(':', pos);
            if (colon == std::string::npos) break;
            const int t = std::atoi(txt.c_str() + colon + 1);
            if (n >= 0 && n <= TOR_MAX_CLICKS && t >= 0 && t <= TOR_PS_LMAX) {
                ctx->ps_t1[n] = t + 1;
                loaded++;
            }
            continue;
        }
        int sl = key.rfind("dd:", 0) == 0 ? 1 : (key.rfind("f64:", 0) == 0 ? 0 : -1);
        if (sl < 0) continue;
        int n = std::atoi(key.c_str() + (sl ? 3 : 4));
        size_t colon = txt.find(':', pos);
        if (colon == std::string::npos) break;
        int J = std::atoi(txt.c_str() + colon + 1);
        if (n >= 0 && n <= TOR_MAX_CLICKS && J >= 1 && J <= TOR_TASK_MAX) {
            ctx->tuned[sl][n] = J;
            loaded++;
        }
    }
    if (!loaded) return fail(TOR_EINVAL, "no tuning entries in %s", cache_path);
    return TOR_OK;
}

tor_status tor_get_tuning(const tor_ctx *ctx, tor_prec prec, int32_t n, int32_t *task_modes) {
    if (!ctx || !task_modes) return fail(TOR_EINVAL, "NULL argument");
    if (n < 0 || n > TOR_MAX_CLICKS) return fail(TOR_EINVAL, "bad n");
    *task_modes = task_modes_for(ctx, prec == TOR_PREC_DD, n);
    return TOR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ persistent server

namespace {

// First-fit allocator of index ranges (the partial arena, the chain output buffer).
struct RangeAlloc {
    std::map<size_t, size_t> free_;  // offset -> length
    void reset(size_t total) {
        free_.clear();
        if (total) free_[0] = total;
    }
    size_t alloc(size_t len) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= len) {
                const size_t off = it->first, rest = it->second - len;
                free_.erase(it);
                if (rest) free_[off + len] = rest;
                return off;
            }
        return SIZE_MAX;
    }
    void release(size_t off, size_t len) {
        if (!len) return;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Schedule of an n-mode tree in the persistent kernel: the task modes J of the
// batched path (so that the trees, tasks and reduction order are the same)
// and the depth-first levels t of a unit (units = 2^(n - J - t)): tuned per n
// (tor_pserver_autotune), else leaving 4096 units.
void ps_schedule(const tor_ctx *ctx, int n, int &J, int &t) {
    J = task_modes_for(ctx, true, n);
    const int G = n - J;
    t = ctx->ps_t1[n] > 0 ? ctx->ps_t1[n] - 1 : std::max(0, G - 12);
    t = std::max(0, std::min({t, G, TOR_PS_LMAX}));
}

// Partials a request needs: one per task, then every reduction stage's.
size_t ps_parts(long long tasks) {
    size_t total = (size_t)tasks;
    for (long long c = tasks; c > 1;) {
        c = (c + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
        total += (size_t)c;
    }
    return total;
}

// The device copy of an inverted state's inverse in double-double words.
tor_status state_inverse_on_device(const tor_state *st) {
    tor_state *ms = const_cast<tor_state *>(st);
    std::lock_guard<std::mutex> lk(ms->dev_mu);
    if (ms->dinv.p) return TOR_OK;
    const size_t ent = (size_t)E(st->m);
    std::vector<dd> h(ent);
    for (size_t e = 0; e < ent; e++) h[e] = st->inv_prec == TOR_PREC_QD ? qd_to_dd(st->inv_q[e]) : st->inv[e];
    if (ms->dinv.ensure(ent * sizeof(dd)) != hipSuccess) return fail(TOR_ENOMEM, "device copy of the inverse failed");
    HIP_TRY(hipMemcpy(ms->dinv.p, h.data(), ent * sizeof(dd), hipMemcpyHostToDevice));
    g_data_gen++;
    return TOR_OK;
}

// The sampler's K_j tables of a zero-mean state on the device (made once).
tor_status state_chain_tables(const tor_state *st) {
    tor_state *ms = const_cast<tor_state *>(st);
    std::lock_guard<std::mutex> lk(ms->dev_mu);
    if (ms->dK.p) return TOR_OK;
    std::vector<double> K;
    std::vector<unsigned long long> koff;
    tor_status s = build_k_tables(st->cov.data(), st->m, K, koff);
    if (s) return s;
    // one buffer [koff | K] and one large copy (a small separate copy could
    // wait for the persistent kernel to leave a CU free)
    const size_t ob = align_up(koff.size() * sizeof(unsigned long long), 256);
    std::vector<unsigned char> blob(ob + K.size() * sizeof(double), 0);
    std::memcpy(blob.data(), koff.data(), koff.size() * sizeof(unsigned long long));
    std::memcpy(blob.data() + ob, K.data(), K.size() * sizeof(double));
    if (ms->dK.ensure(blob.size()) != hipSuccess) return fail(TOR_ENOMEM, "device allocation of the K tables failed");
    HIP_TRY(hipMemcpy(ms->dK.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
    ms->k_off_bytes = ob;
    g_data_gen++;
    return TOR_OK;
}

struct PsEntry {  // host bookkeeping of a ticket
    int type = TOR_PS_PROB;
    bool host_only = false;       // finished on the host (no clicks): res holds the result
    unsigned long long seq = 0;   // the request's index in the ring
    Prepared prep;                // probability: what the result's assembly needs
    size_t part_off = 0, part_len = 0;  // probability: partials in the arena
    size_t out_off = 0, out_len = 0;    // chains: outputs in the pinned buffer
    int m = 0, nchains = 0;
    tor_result res{};
    std::chrono::steady_clock::time_point t0;
};

}  // namespace

struct tor_pserver {
    tor_ctx *ctx = nullptr;
    int device = 0;
    hipStream_t kst = nullptr;
    PsHost *host = nullptr;
    PsReq *ring = nullptr;
    PsResult *res = nullptr;
    unsigned char *outbuf = nullptr;
    size_t outbuf_bytes = 0;
    DevBuf dev, scratch, arena;
    RangeAlloc parts, outs;
    PsParams params{};
    unsigned long long epoch = 0;  // launches so far: the newest launch's number
    int grid = 0;
    double tol = 1e-10;
    std::mutex mu;
    unsigned long long next_seq = 0;        // next request index to publish
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, PsEntry> live;
    uint64_t slot_ticket[TOR_PS_SLOTS] = {};  // ticket whose request holds the slot (0: free)
    unsigned long long slot_seq[TOR_PS_SLOTS] = {};  // the request last published into the slot
    // completion watcher: stamps the time each published request finishes
    std::thread watcher;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    unsigned long long watch_seq = 0;          // requests before it are stamped or read
    bool slot_done[TOR_PS_SLOTS] = {};         // the slot's request is finished (stamped)
    std::chrono::steady_clock::time_point slot_t_done[TOR_PS_SLOTS];
    tor_status kernel_error = TOR_OK;          // a failed relaunch seen by the watcher
    std::string kernel_error_msg;              // and its message
    tor_pserver_stats stats{};
};

namespace {

// Launch the persistent kernel unless it is running (S->mu held).  A launch
// that is closing (its workgroups are leaving) counts as not running: the next
// one is queued behind it on the kernel's stream.
tor_status ps_ensure_running(tor_pserver *S) {
    const hipError_t q = hipStreamQuery(S->kst);
    if (q == hipErrorNotReady) {
        if (__atomic_load_n(&S->host->seen_closing, __ATOMIC_ACQUIRE) != S->epoch) return TOR_OK;
    } else if (q != hipSuccess) {
        (void)hipGetLastError();
        return fail(TOR_EDEVICE, "persistent kernel failed: %s", hipGetErrorString(q));
    }
    HIP_TRY(hipSetDevice(S->device));
    S->params.epoch = ++S->epoch;
    HIP_TRY(tor_launch_pserver(S->params, S->grid, S->kst));
    S->stats.launches++;
    return TOR_OK;
}

// Claim the next ring slot and publish a filled request (S->mu held).
tor_status ps_publish(tor_pserver *S, PsReq &rq, PsEntry &&e, uint64_t *ticket) {
    const unsigned long long seq = S->next_seq;
    const int slot = (int)(seq % TOR_PS_SLOTS);
    rq.seq = (long long)seq;
    rq.gen = g_data_gen.load();
    PsReq *dst = &S->ring[slot];
    std::memcpy((char *)dst + sizeof(long long), (const char *)&rq + sizeof(long long), sizeof(PsReq) - sizeof(long long));
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(&dst->seq, (long long)seq, __ATOMIC_RELEASE);
    __atomic_store_n(&S->host->published, seq + 1, __ATOMIC_RELEASE);
    S->next_seq = seq + 1;
    e.seq = seq;
    e.t0 = std::chrono::steady_clock::now();
    const uint64_t t = S->next_ticket++;
    S->slot_ticket[slot] = t;
    S->slot_seq[slot] = seq;
    S->slot_done[slot] = false;
    S->live.emplace(t, std::move(e));
    *ticket = t;
    S->stats.submitted++;
    S->cv_work.notify_one();
    return ps_ensure_running(S);
}

// Stamp request seq finished if its completion word says so (S->mu held).  A
// request whose slot already holds a later one was read and released: it is
// finished, and the slot's flags belong to the later request.
bool ps_check(tor_pserver *S, unsigned long long seq) {
    const int slot = (int)(seq % TOR_PS_SLOTS);
    if (S->slot_seq[slot] != seq) return true;
    if (S->slot_done[slot]) return true;
    if (__atomic_load_n(&S->res[slot].done, __ATOMIC_ACQUIRE) != seq + 1) return false;
    S->slot_done[slot] = true;
    S->slot_t_done[slot] = std::chrono::steady_clock::now();
    return true;
}

// A ticket's request finished on the device (S->mu held)?
bool ps_done(tor_pserver *S, const PsEntry &e) { return e.host_only || ps_check(S, e.seq); }

// Completion time of a finished ticket (S->mu held).
std::chrono::steady_clock::time_point ps_t_done(const tor_pserver *S, const PsEntry &e) {
    return e.host_only ? e.t0 : S->slot_t_done[e.seq % TOR_PS_SLOTS];
}

// The completion watcher: stamps finished requests as their completion words
// arrive (so that latencies are the device's, not the reader's), wakes
// waiting readers, and launches the kernel again if it exited with requests
// outstanding.
void ps_watch(tor_pserver *S) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto last_check = std::chrono::steady_clock::now();
    while (!S->stopping) {
        if (S->watch_seq == S->next_seq) {
            S->cv_work.wait(lk);
            continue;
        }
        bool any = false;
        // a slot holding a later request than q means q was read already
        auto unstamped = [&](unsigned long long q) {
            const int slot = (int)(q % TOR_PS_SLOTS);
            return S->slot_seq[slot] == q && S->slot_ticket[slot] && !S->slot_done[slot];
        };
        for (unsigned long long q = S->watch_seq; q < S->next_seq; ++q)
            if (unstamped(q) && ps_check(S, q)) any = true;
        while (S->watch_seq < S->next_seq && !unstamped(S->watch_seq))  // past every stamped or read request
            S->watch_seq++;
        if (any) S->cv_done.notify_all();
        const auto now = std::chrono::steady_clock::now();
        if (now - last_check > std::chrono::milliseconds(1)) {
            last_check = now;
            if (S->watch_seq < S->next_seq && S->kernel_error == TOR_OK) {
                S->kernel_error = ps_ensure_running(S);
                if (S->kernel_error) {
                    S->kernel_error_msg = g_err;
                    S->cv_done.notify_all();
                }
            }
        }
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(2));
        lk.lock();
    }
}

void ps_release(tor_pserver *S, uint64_t ticket, PsEntry &e) {
    if (!e.host_only) {
        S->slot_ticket[e.seq % TOR_PS_SLOTS] = 0;
        S->parts.release(e.part_off, e.part_len);
        S->outs.release(e.out_off, e.out_len);
    }
    S->stats.completed++;
    S->live.erase(ticket);
}

}  // namespace

extern "C" {

tor_status tor_pserver_start(tor_ctx *ctx, const tor_pserver_opts *opts, tor_pserver **out) {
    if (!ctx || !out) return fail(TOR_EINVAL, "NULL argument");
    *out = nullptr;
    tor_pserver_opts o{};
    o.tol = 1e-10;
    o.mem_budget_bytes = (size_t)1 << 30;
    o.chain_buffer_bytes = (size_t)64 << 20;
    o.grid = 0;
    o.idle_ms = 50;
    if (opts) {
        if (opts->tol > 0) o.tol = opts->tol;
        if (opts->mem_budget_bytes > 0) o.mem_budget_bytes = opts->mem_budget_bytes;
        if (opts->chain_buffer_bytes > 0) o.chain_buffer_bytes = opts->chain_buffer_bytes;
        if (opts->grid < 0 || opts->idle_ms < 0) return fail(TOR_EINVAL, "negative grid or idle time");
        o.grid = opts->grid;
        if (opts->idle_ms > 0) o.idle_ms = opts->idle_ms;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<tor_pserver> S(new (std::nothrow) tor_pserver());
    if (!S) return fail(TOR_ENOMEM, "host allocation failed");
    S->ctx = ctx;
    S->device = ctx->device;
    S->tol = o.tol;
    const int occ = tor_pserver_occupancy(ctx->device);
    if (occ < 1) return fail(TOR_EDEVICE, "the persistent kernel does not fit the device");
    S->grid = o.grid > 0 ? std::min(o.grid, occ) : occ;
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (khz <= 0) return fail(TOR_EDEVICE, "no wall clock rate");
    auto cleanup = [&]() {
        if (S->kst) (void)hipStreamDestroy(S->kst);
        if (S->host) (void)hipHostFree(S->host);
        if (S->ring) (void)hipHostFree(S->ring);
        if (S->res) (void)hipHostFree(S->res);
        if (S->outbuf) (void)hipHostFree(S->outbuf);
        S->dev.release();
        S->scratch.release();
        S->arena.release();
        (void)hipGetLastError();
    };
    // host-coherent ring, results, control block and chain outputs
    if (hipHostMalloc((void **)&S->host, sizeof(PsHost), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&S->ring, sizeof(PsReq) * TOR_PS_SLOTS, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&S->res, sizeof(PsResult) * TOR_PS_SLOTS, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&S->outbuf, o.chain_buffer_bytes, hipHostMallocCoherent) != hipSuccess) {
        cleanup();
        return fail(TOR_ENOMEM, "pinned allocation of the request ring failed");
    }
    S->outbuf_bytes = o.chain_buffer_bytes;
    std::memset(S->host, 0, sizeof(PsHost));
    std::memset(S->ring, 0, sizeof(PsReq) * TOR_PS_SLOTS);
    for (int i = 0; i < TOR_PS_SLOTS; i++) S->ring[i].seq = -1;
    std::memset(S->res, 0, sizeof(PsResult) * TOR_PS_SLOTS);
    // device state, per-workgroup scratch and the partial arena
    const size_t scratch_bytes = (size_t)S->grid * TOR_PS_SCRATCH_WORDS * sizeof(dd);
    if (S->dev.ensure(sizeof(PsDev)) != hipSuccess || S->scratch.ensure(scratch_bytes) != hipSuccess ||
        S->arena.ensure(o.mem_budget_bytes) != hipSuccess) {
        cleanup();
        return fail(TOR_ENOMEM, "device allocation of the persistent server failed");
    }
    S->parts.reset(o.mem_budget_bytes / sizeof(Partial));
    S->outs.reset(o.chain_buffer_bytes);
    if (hipStreamCreateWithFlags(&S->kst, hipStreamNonBlocking) != hipSuccess) {
        cleanup();
        return fail(TOR_EDEVICE, "hipStreamCreate failed");
    }
    {
        std::vector<unsigned char> init(sizeof(PsDev), 0);
        PsDev *d = reinterpret_cast<PsDev *>(init.data());
        for (int i = 0; i < TOR_PS_SLOTS; i++) d->next[i] = (unsigned long long)i << 32;
        if (hipMemcpy(S->dev.p, init.data(), init.size(), hipMemcpyHostToDevice) != hipSuccess) {
            cleanup();
            return fail(TOR_EDEVICE, "initialising the persistent server failed");
        }
    }
    PsParams &P = S->params;
    P.host = S->host;
    P.ring = S->ring;
    P.res = S->res;
    P.dev = (PsDev *)S->dev.p;
    P.scratch = (dd *)S->scratch.p;
    P.scratch_stride = TOR_PS_SCRATCH_WORDS;
    P.idle_ticks = (long long)o.idle_ms * khz;
    P.refresh_ticks = std::max(1LL, (long long)khz * 2 / 1000);  // 2 us
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (ps_ensure_running(S.get()) != TOR_OK) {
            std::string msg = g_err;
            cleanup();
            return fail(TOR_EDEVICE, "%s", msg.c_str());
        }
    }
    S->watcher = std::thread(ps_watch, S.get());
    *out = S.release();
    return TOR_OK;
}

tor_status tor_pserver_submit(tor_pserver *S, const tor_state *st, const int8_t *pattern, uint64_t *ticket) {
    if (!S || !st || !pattern || !ticket) return fail(TOR_EINVAL, "NULL argument");
    if (st->ctx != S->ctx) return fail(TOR_EINVAL, "state belongs to another context");
    if (!st->mean.empty()) return fail(TOR_EINVAL, "displaced states are served by tor_submit");
    const int m = st->m;
    bool zero = false;
    for (int i = 0; i < m; i++) {
        if (pattern[i] < -1 || pattern[i] > 1) return fail(TOR_EINVAL, "pattern[%d] = %d", i, (int)pattern[i]);
        zero |= pattern[i] == 0;
    }
    const bool jac = zero && is_full_pattern(pattern, m);
    if (zero && !(jac && st->inv_prec))
        return fail(TOR_EINVAL, "a pattern with no-click modes needs a full pattern of an inverted state "
                                "(tor_state_invert), or tor_submit");
    HIP_TRY(hipSetDevice(S->device));
    Reduced red;
    tor_status s = jac ? reduce_pattern_jacobi(st, pattern, red) : reduce_pattern(st->cov.data(), m, pattern, red);
    if (s) return s;
    PsEntry e;
    e.type = TOR_PS_PROB;
    s = prepare_reduced(red, e.prep);
    if (s) return s;
    const int n = red.n;
    if (n == 0) {  // nothing to sum: the result is known on the host
        SumOut so;
        finalize(e.prep, so, TOR_PREC_DD, S->tol, &e.res);
        e.host_only = true;
        e.t0 = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lk(S->mu);
        *ticket = S->next_ticket++;
        S->live.emplace(*ticket, std::move(e));
        S->stats.submitted++;
        return TOR_OK;
    }
    s = jac ? state_inverse_on_device(st) : state_on_device(st);
    if (s) return s;
    int J, t;
    PsReq rq{};
    rq.type = TOR_PS_PROB;
    rq.n = n;
    rq.m = m;
    rq.jac = jac ? 1 : 0;
    rq.cov = (const double *)st->dcov.p;
    rq.inv = jac ? (const dd *)st->dinv.p : nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    ps_schedule(S->ctx, n, J, t);
    const int G = n - J, g = G - t;
    rq.J = J;
    rq.g = g;
    rq.t = t;
    rq.units = 1LL << g;
    rq.tasks = 1LL << G;
    int k = 0;
    for (int i = 0; i < m; i++)
        if (pattern[i] == 1) rq.C[k++] = i;
    if (S->slot_ticket[S->next_seq % TOR_PS_SLOTS]) return fail(TOR_EAGAIN, "request ring full");
    e.part_len = ps_parts(rq.tasks);
    e.part_off = S->parts.alloc(e.part_len);
    if (e.part_off == SIZE_MAX) {
        e.part_len = 0;
        return fail(TOR_EAGAIN, "not admitted: partial sums of %zu bytes do not fit", ps_parts(rq.tasks) * sizeof(Partial));
    }
    rq.part = (Partial *)S->arena.p + e.part_off;
    S->stats.units += rq.units;
    return ps_publish(S, rq, std::move(e), ticket);
}

tor_status tor_pserver_submit_chains(tor_pserver *S, const tor_state *st, int32_t n_post, uint64_t seed,
                                     int64_t chain_begin, int32_t nchains, uint64_t *ticket) {
    if (!S || !st || !ticket) return fail(TOR_EINVAL, "NULL argument");
    if (st->ctx != S->ctx) return fail(TOR_EINVAL, "state belongs to another context");
    if (!st->mean.empty()) return fail(TOR_EINVAL, "displaced states are sampled by gbs_sample_displaced");
    if (nchains < 1 || chain_begin < 0) return fail(TOR_EINVAL, "bad chain range");
    const int m = st->m;
    if (m > 1024) return fail(TOR_ETOOBIG, "m = %d > 1024 for the sampler", m);
    if (n_post > TOR_CHAIN_MAX - 1) return fail(TOR_ETOOBIG, "n_post = %d > %d", n_post, TOR_CHAIN_MAX - 1);
    if (n_post > m) return fail(TOR_EINVAL, "n_post > m");
    HIP_TRY(hipSetDevice(S->device));
    tor_status s = state_chain_tables(st);
    if (s) return s;
    PsEntry e;
    e.type = TOR_PS_CHAINS;
    e.m = m;
    e.nchains = nchains;
    e.out_len = (size_t)nchains * (size_t)(m + 1);
    PsReq rq{};
    rq.type = TOR_PS_CHAINS;
    rq.m = m;
    rq.units = nchains;
    ChainParams &P = rq.cp;
    P.koff = (const unsigned long long *)st->dK.p;
    P.K = (const double *)((const unsigned char *)st->dK.p + st->k_off_bytes);
    P.H = nullptr;
    P.hoff = nullptr;
    P.m = m;
    P.n_post = n_post;
    P.cap = n_post >= 0 ? n_post : std::min(S->ctx->chain_clicks, TOR_CHAIN_MAX - 1);
    P.seed = seed;
    P.chain_begin = chain_begin;
    P.nchains = nchains;
    P.trace_p = nullptr;
    P.trace_u = nullptr;
    P.subsets = nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->slot_ticket[S->next_seq % TOR_PS_SLOTS]) return fail(TOR_EAGAIN, "request ring full");
    e.out_off = S->outs.alloc(e.out_len);
    if (e.out_off == SIZE_MAX) {
        e.out_len = 0;
        return fail(TOR_EAGAIN, "not admitted: chain outputs do not fit the pinned buffer");
    }
    P.outcome = S->outbuf + e.out_off;
    P.status = (signed char *)(S->outbuf + e.out_off + (size_t)nchains * m);
    S->stats.units += nchains;
    return ps_publish(S, rq, std::move(e), ticket);
}

tor_status tor_pserver_poll(tor_pserver *S, uint64_t ticket, int32_t wait, tor_result *out, double *latency_s) {
    if (!S || !out) return fail(TOR_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        {
            auto it = S->live.find(ticket);
            if (it == S->live.end()) return fail(TOR_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
            PsEntry &e = it->second;
            if (e.type != TOR_PS_PROB) return fail(TOR_EINVAL, "ticket %llu is a sampling request", (unsigned long long)ticket);
            if (ps_done(S, e)) {
                if (!e.host_only) {
                    const PsResult &r = S->res[e.seq % TOR_PS_SLOTS];
                    SumOut so;
                    so.T = dd_make(r.t_hi, r.t_lo);
                    so.A = r.a;
                    if (!std::isfinite(so.T.hi) || !std::isfinite(so.A)) {
                        std::memset(&e.res, 0, sizeof e.res);
                        e.res.status = TOR_ENOTPD;
                    } else {
                        finalize(e.prep, so, TOR_PREC_DD, S->tol, &e.res);
                    }
                }
                *out = e.res;
                if (latency_s) *latency_s = std::chrono::duration<double>(ps_t_done(S, e) - e.t0).count();
                const tor_status st = e.res.status;
                ps_release(S, ticket, e);
                return st;
            }
            if (S->kernel_error) return fail(S->kernel_error, "persistent kernel: %s", S->kernel_error_msg.c_str());
            if (!wait) return TOR_EAGAIN;
            S->cv_done.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

tor_status tor_pserver_poll_chains(tor_pserver *S, uint64_t ticket, int32_t wait, uint8_t *outcomes,
                                   int8_t *status, double *latency_s) {
    if (!S) return fail(TOR_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        {
            auto it = S->live.find(ticket);
            if (it == S->live.end()) return fail(TOR_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
            PsEntry &e = it->second;
            if (e.type != TOR_PS_CHAINS) return fail(TOR_EINVAL, "ticket %llu is a probability query", (unsigned long long)ticket);
            if (ps_done(S, e)) {
                const unsigned char *o = S->outbuf + e.out_off;
                if (outcomes) std::memcpy(outcomes, o, (size_t)e.nchains * e.m);
                if (status) std::memcpy(status, o + (size_t)e.nchains * e.m, (size_t)e.nchains);
                if (latency_s) *latency_s = std::chrono::duration<double>(ps_t_done(S, e) - e.t0).count();
                ps_release(S, ticket, e);
                return TOR_OK;
            }
            if (S->kernel_error) return fail(S->kernel_error, "persistent kernel: %s", S->kernel_error_msg.c_str());
            if (!wait) return TOR_EAGAIN;
            S->cv_done.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

tor_status tor_pserver_get_stats(tor_pserver *S, tor_pserver_stats *out) {
    if (!S || !out) return fail(TOR_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->pending = (int64_t)S->live.size();
    out->running = hipStreamQuery(S->kst) == hipErrorNotReady ? 1 : 0;
    (void)hipGetLastError();
    // the kernel's counters as it last mirrored them into host memory (a
    // device copy could wait for the kernel to leave a CU free)
    out->device_cursor = (int64_t)__atomic_load_n(&S->host->seen_cur, __ATOMIC_ACQUIRE);
    out->device_published = (int64_t)__atomic_load_n(&S->host->seen_pub, __ATOMIC_ACQUIRE);
    out->workgroups = S->grid;
    out->workgroups_started = (int32_t)__atomic_load_n(&S->host->seen_started, __ATOMIC_ACQUIRE);
    out->workgroups_peak = (int32_t)__atomic_load_n(&S->host->seen_peak, __ATOMIC_ACQUIRE);
    return TOR_OK;
}

tor_status tor_pserver_stop(tor_pserver *S) {
    if (!S) return fail(TOR_EINVAL, "NULL argument");
    (void)hipSetDevice(S->device);
    tor_status first = TOR_OK;
    // finish every published request (their results are dropped if not polled)
    {
        std::unique_lock<std::mutex> lk(S->mu);
        for (;;) {
            bool pending = false;
            for (auto &kv : S->live)
                if (!ps_done(S, kv.second)) pending = true;
            if (!pending) break;
            if (S->kernel_error) {
                first = S->kernel_error;
                break;
            }
            S->cv_done.wait_for(lk, std::chrono::milliseconds(1));
        }
        S->stopping = true;
        S->cv_work.notify_all();
    }
    S->watcher.join();
    __atomic_store_n(&S->host->stop, 1u, __ATOMIC_RELEASE);
    const hipError_t e = hipStreamSynchronize(S->kst);
    if (e != hipSuccess && first == TOR_OK) first = fail(TOR_EDEVICE, "persistent kernel: %s", hipGetErrorString(e));
    (void)hipStreamDestroy(S->kst);
    (void)hipHostFree(S->host);
    (void)hipHostFree(S->ring);
    (void)hipHostFree(S->res);
    (void)hipHostFree(S->outbuf);
    S->dev.release();
    S->scratch.release();
    S->arena.release();
    (void)hipGetLastError();
    delete S;
    return first;
}

}  // extern "C"

extern "C" {

tor_status tor_pserver_autotune(tor_pserver *S, int32_t n_lo, int32_t n_hi, const char *cache_path) {
    if (!S) return fail(TOR_EINVAL, "NULL argument");
    if (n_lo < 1 || n_hi > TOR_MAX_CLICKS || n_lo > n_hi) return fail(TOR_EINVAL, "bad n range");
    tor_ctx *ctx = S->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    // a synthetic 32-mode state (sigma = I + B B^T / 64, SPD), marginal queries
    // of n clicks drawn by a fixed generator.  For each unit depth: the time of
    // one query alone (latency) and the time per query of a burst of 32
    // submitted together (throughput under load), medians of three.  The
    // choice: the best throughput among the depths whose latency is within
    // 1.5x (+ 20 us) of the best latency.
    constexpr int M = TOR_MAX_CLICKS, BURST = 32;
    const char *vb = std::getenv("TOR_TUNE_VERBOSE");  // print each measurement to stderr
    const bool verbose = vb && *vb && *vb != '0';
    const std::vector<dd> sig = synthetic_sigma(M);
    std::vector<double> cov(sig.size());
    for (size_t i = 0; i < sig.size(); i++) cov[i] = sig[i].hi;
    tor_state *st = nullptr;
    tor_status s = tor_state_create(ctx, cov.data(), M, &st);
    if (s) return s;
    unsigned lcg = 7u;
    auto run = [&](const std::vector<std::vector<int8_t>> &pats, int count, double &secs) -> tor_status {
        auto t0 = std::chrono::steady_clock::now();
        uint64_t tk[BURST];
        for (int q = 0; q < count; q++) {
            tor_status e = tor_pserver_submit(S, st, pats[q].data(), &tk[q]);
            if (e < 0) return e;
        }
        for (int q = 0; q < count; q++) {
            tor_result r;
            tor_status e = tor_pserver_poll(S, tk[q], 1, &r, nullptr);
            if (e < 0) return e;
        }
        secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return TOR_OK;
    };
    for (int n = n_lo; n <= n_hi; n++) {
        std::vector<std::vector<int8_t>> pats(BURST, std::vector<int8_t>(M, -1));
        for (auto &p : pats)
            for (int k = 0; k < n;) {
                lcg = lcg * 1664525u + 1013904223u;
                const int i = (int)((lcg >> 8) % M);
                if (p[i] != 1) {
                    p[i] = 1;
                    k++;
                }
            }
        const int J = task_modes_for(ctx, true, n), G = n - J, TMAX = std::min(G, TOR_PS_LMAX);
        std::vector<double> lat(TMAX + 1), per(TMAX + 1);
        for (int t = 0; t <= TMAX; t++) {
            ctx->ps_t1[n] = t + 1;
            double a[3], b[3];
            for (int rep = 0; rep < 4; rep++) {  // one warm-up pass, three timed
                double one, burst;
                s = run(pats, 1, one);
                if (s == TOR_OK) s = run(pats, BURST, burst);
                if (s < 0) {
                    tor_state_destroy(st);
                    return s;
                }
                if (rep) {
                    a[rep - 1] = one;
                    b[rep - 1] = burst / BURST;
                }
            }
            std::sort(a, a + 3);
            std::sort(b, b + 3);
            lat[t] = a[1];
            per[t] = b[1];
            if (verbose)
                std::fprintf(stderr, "pserver autotune n=%d J=%d t=%d units=%lld alone %.3f ms, per query in a burst %.3f ms\n",
                             n, J, t, 1LL << (G - t), lat[t] * 1e3, per[t] * 1e3);
        }
        const double lmin = *std::min_element(lat.begin(), lat.end());
        int best = 0;
        for (int t = 0; t <= TMAX; t++)
            if (lat[t] <= 1.5 * lmin + 20e-6 && (lat[best] > 1.5 * lmin + 20e-6 || per[t] < per[best])) best = t;
        ctx->ps_t1[n] = best + 1;
    }
    tor_state_destroy(st);
    if (cache_path && *cache_path) return write_tuning(ctx, cache_path);
    return TOR_OK;
}

}  // extern "C"

