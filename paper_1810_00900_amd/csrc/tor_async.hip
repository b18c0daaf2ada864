// Stream-ordered batches: click patterns and results in device memory.
//
// The host cannot see the patterns, so the plan the host planner makes for
// tor_batch (tor_api.hip, gpu_group) is made here on the device, for the same
// per-query trees: task size J(n), 2^(n-J) tasks after n - J HBM levels, the
// same reduction chunks in the same order.  A query's result therefore does
// not depend on the planner that scheduled it or on the other queries.
//
//   async_scan_kernel      one wave per query: clicked modes, validation
//   async_plan_kernel      one workgroup: sizes, admission into the
//                          workspace, job tables of every launch (block scans
//                          over queries in query order)
//   async_gather_kernel    one wave per query: the root Sigma_C = sigma_Q[C]
//                          (row a2 for marginal patterns) and log det Sigma_C
//   (expand, wave and reduce kernels with device-side launch dimensions)
//   async_finalize_kernel  one thread per query: tor_result (row a6)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor.h"
#include "tor_kernels.h"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

// ---------------------------------------------------------------- scan

__global__ __launch_bounds__(64) void async_scan_kernel(const int8_t *__restrict__ pats, AsyncPlan P) {
    const int lane = threadIdx.x;
    for (int q = blockIdx.x; q < P.nq; q += gridDim.x) {
        const int8_t *row = pats + (size_t)q * (size_t)P.m;
        int count = 0;
        bool bad = false, noclick = false, unobs = false;
        for (int base = 0; base < P.m; base += 64) {
            const int k = base + lane;
            const int v = k < P.m ? (int)row[k] : 1;  // lanes past the end count as observed
            const bool one = v == 1 && k < P.m;
            if (v == 0) noclick = true;
            else if (v == -1) unobs = true;
            else if (v != 1) bad = true;
            const unsigned long long mask = __ballot(one);
            const int pos = count + __popcll(mask & ((1ULL << lane) - 1ULL));
            if (one && pos < TOR_MAX_N) P.q[q].C[pos] = k;
            count += __popcll(mask);
        }
        bad = __any(bad);
        noclick = __any(noclick);
        unobs = __any(unobs);
        if (lane == 0) {
            AsyncQuery &Q = P.q[q];
            // a full pattern (no unobserved mode) of an inverted state takes the
            // complementary-minor route; other no-click patterns are not taken
            const bool jac = noclick && !unobs && P.inv != nullptr;
            Q.n = count;
            Q.jac = jac ? 1 : 0;
            Q.status = (bad || (noclick && !jac)) ? TOR_EINVAL : (count > TOR_MAX_N ? TOR_ETOOBIG : TOR_OK);
        }
    }
}

// ---------------------------------------------------------------- plan

constexpr int kPlanThreads = 1024;

// Exclusive scan of one value per thread over the workgroup; *total receives
// the sum.  lds holds kPlanThreads + 1 entries.
__device__ long long block_excl_scan(long long x, long long *lds, long long *total) {
    const int t = threadIdx.x;
    lds[t] = x;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const long long y = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += y;
        __syncthreads();
    }
    const long long incl = lds[t];
    *total = lds[kPlanThreads - 1];
    __syncthreads();
    return incl - x;
}

// Exclusive prefix sums of value(q) over queries in query order: thread t owns
// a contiguous chunk of queries; write(q, prefix) for every q.  Returns the total.
template <class V, class W>
__device__ long long scan_queries(int nq, V value, W write, long long *lds) {
    const int t = threadIdx.x;
    const int chunk = (nq + kPlanThreads - 1) / kPlanThreads;
    const int lo = min(nq, t * chunk), hi = min(nq, lo + chunk);
    long long s = 0;
    for (int q = lo; q < hi; q++) s += value(q);
    long long total;
    long long ex = block_excl_scan(s, lds, &total);
    for (int q = lo; q < hi; q++) {
        const long long v = value(q);
        write(q, ex);
        ex += v;
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// reduction-stage input counts of a tree with nt tasks: cnt[0] = nt, cnt[s+1] =
// ceil(cnt[s] / chunk); stage s runs while cnt[s] > 1
__device__ __forceinline__ long long stage_count(long long nt, int s) {
    long long c = nt;
    for (int k = 0; k < s; k++) c = ceil_div(c, TOR_REDUCE_CHUNK);
    return c;
}

__device__ __forceinline__ NodeDesc *level_ptr(const AsyncPlan &P, int q, const AsyncQuery &Q, int d) {
    if (d == 0) return P.roots + q;
    return ((d & 1) ? P.descB : P.descA) + Q.desc_off;
}

__global__ __launch_bounds__(kPlanThreads) void async_plan_kernel(AsyncPlan P) {
    __shared__ long long lds[kPlanThreads + 1];
    const int nq = P.nq;
    AsyncQuery *Qs = P.q;
    // sizes of every query's tree
    for (int q = threadIdx.x; q < nq; q += kPlanThreads) {
        AsyncQuery &Q = Qs[q];
        Q.J = Q.G = 0;
        Q.nt = Q.entries = Q.pb = 0;
        Q.nstage = 0;
        Q.pool_off = Q.desc_off = Q.pb_off = Q.final_off = 0;
        Q.final_buf = 0;
        Q.log_det = 0.0;
        Q.quad = 0.0;
        Q.jscale = 1.0;
        Q.log_pvac = Q.jac ? -0.5 * (P.log_det_sigq + P.mu_k_mu) : 0.0;
        if (Q.status != TOR_OK || Q.n == 0) continue;
        const int n = Q.n;
        const int J = min(n, P.J_of_n[n]);
        const int G = n - J;
        long long entries = EN(n, P.D);
        for (int d = 0; d < G; d++) entries += (1LL << d) * (long long)EN(n - d - 1, P.D);
        Q.J = J;
        Q.G = G;
        Q.nt = 1LL << G;
        Q.entries = entries;
        long long pb = 0;
        int ns = 0;
        for (int s = 0; s < TOR_ASYNC_STAGES; s++) {
            const long long c = stage_count(Q.nt, s);
            if (c <= 1) break;
            pb += ceil_div(c, TOR_REDUCE_CHUNK);
            ns++;
        }
        Q.pb = pb;
        Q.nstage = ns;
        if (stage_count(Q.nt, ns) > 1) Q.status = TOR_ETOOBIG;  // more stages than planned for
    }
    __syncthreads();
    // admission in query order: a query runs if everything up to it fits
    scan_queries(nq, [&](int q) { return Qs[q].entries; }, [&](int q, long long x) { Qs[q].pool_off = x; }, lds);
    scan_queries(nq, [&](int q) { return Qs[q].nt; }, [&](int q, long long x) { Qs[q].desc_off = x; }, lds);
    scan_queries(nq, [&](int q) { return Qs[q].pb; }, [&](int q, long long x) { Qs[q].pb_off = x; }, lds);
    for (int q = threadIdx.x; q < nq; q += kPlanThreads) {
        AsyncQuery &Q = Qs[q];
        if (Q.status != TOR_OK || Q.n == 0) continue;
        if (Q.pool_off + Q.entries > P.pool_cap || Q.desc_off + Q.nt > P.desc_cap || Q.pb_off + Q.pb > P.pb_cap) {
            Q.status = TOR_ENOMEM;
            continue;
        }
        NodeDesc r;
        r.off = (unsigned long long)Q.pool_off;
        r.coef_hi = 1.0;
        r.coef_lo = 0.0;
        r.acoef = 1.0;
        P.roots[q] = r;
        // the partial that ends up holding the tree's sum
        if (Q.nstage == 0) {
            Q.final_buf = 0;
            Q.final_off = Q.desc_off;
        } else {
            long long off = Q.pb_off;
            for (int s = 0; s + 1 < Q.nstage; s++) off += ceil_div(stage_count(Q.nt, s), TOR_REDUCE_CHUNK);
            Q.final_buf = 1;
            Q.final_off = off;
        }
    }
    __syncthreads();
    auto live = [&](int q) { return Qs[q].status == TOR_OK && Qs[q].n > 0; };
    // tree kind of a query: 1 for the information-form trees of an inverted
    // displaced state's full patterns, else 0; the tables are kind-major
    auto kind = [&](int q) { return P.nkinds > 1 && Qs[q].jac ? 1 : 0; };
    const int stride = P.gcap + TOR_TASK_MAX + 1;  // launch dimensions per kind
    for (int k = 0; k < P.nkinds; k++) {  // a tree kind's expand and wave tables
    // HBM levels: depth d expands every tree with more than d levels
    for (int d = 0; d < P.gcap; d++) {
        const long long cnt = scan_queries(
            nq, [&](int q) { return (long long)(live(q) && kind(q) == k && Qs[q].G > d); },
            [&](int q, long long pos) {
                const AsyncQuery &Q = Qs[q];
                if (!(live(q) && kind(q) == k && Q.G > d)) return;
                long long base = Q.pool_off + EN(Q.n, P.D);
                for (int t = 0; t < d; t++) base += (1LL << t) * (long long)EN(Q.n - t - 1, P.D);
                ExpandJob j;
                j.par = level_ptr(P, q, Q, d);
                j.chi = level_ptr(P, q, Q, d + 1);
                j.child_base = (unsigned long long)base;
                j.r = Q.n - d;
                j.d = P.D;
                P.exp_jobs[((size_t)k * P.gcap + d) * nq + pos] = j;
            },
            lds);
        if (threadIdx.x == 0) {
            P.dims[k * stride + d].njobs = cnt;
            P.dims[k * stride + d].total = cnt << d;
        }
    }
    // wave tier: one launch per task size (descending J, query order within)
    for (int J = P.jmax; J >= 1; J--) {
        auto in = [&](int q) { return live(q) && kind(q) == k && Qs[q].J == J; };
        const long long cnt = scan_queries(
            nq, [&](int q) { return (long long)in(q); }, [&](int q, long long pos) { Qs[q].slot = pos; }, lds);
        const long long tot = scan_queries(
            nq, [&](int q) { return in(q) ? Qs[q].nt : 0LL; },
            [&](int q, long long begin) {
                if (!in(q)) return;
                const AsyncQuery &Q = Qs[q];
                WaveJob w;
                w.tasks = level_ptr(P, q, Q, Q.G);
                w.out = P.partA + Q.desc_off;
                w.begin = begin;
                P.wave_jobs[((size_t)k * (TOR_TASK_MAX + 1) + J) * nq + Q.slot] = w;
            },
            lds);
        if (threadIdx.x == 0) {
            P.dims[k * stride + P.gcap + J].njobs = cnt;
            P.dims[k * stride + P.gcap + J].total = tot;
        }
    }
    }  // kinds
    // reduction stages: stage s sums chunks of stage s - 1 (stage 0: the tasks)
    for (int s = 0; s < TOR_ASYNC_STAGES; s++) {
        auto in = [&](int q) { return live(q) && Qs[q].nstage > s; };
        const long long cnt = scan_queries(
            nq, [&](int q) { return (long long)in(q); }, [&](int q, long long pos) { Qs[q].slot = pos; }, lds);
        const long long blocks = scan_queries(
            nq, [&](int q) { return in(q) ? ceil_div(stage_count(Qs[q].nt, s), TOR_REDUCE_CHUNK) : 0LL; },
            [&](int q, long long bb) {
                if (!in(q)) return;
                const AsyncQuery &Q = Qs[q];
                long long out_off = Q.pb_off;
                for (int k = 0; k < s; k++) out_off += ceil_div(stage_count(Q.nt, k), TOR_REDUCE_CHUNK);
                ReduceJob r;
                if (s == 0) {
                    r.in = P.partA + Q.desc_off;
                } else {
                    r.in = P.partB + out_off - ceil_div(stage_count(Q.nt, s - 1), TOR_REDUCE_CHUNK);
                }
                r.out = P.partB + out_off;
                r.count = stage_count(Q.nt, s);
                r.block_begin = bb;
                P.red_jobs[(size_t)s * nq + Q.slot] = r;
            },
            lds);
        if (threadIdx.x == 0) {
            P.dims[P.nkinds * stride + s].njobs = cnt;
            P.dims[P.nkinds * stride + s].total = blocks;
        }
    }
}

// ---------------------------------------------------------------- roots

// The root of each admitted tree: Sigma_C = sigma_Q[C] (sigma_Q = sigma + I/2,
// the diagonal exact in double-double) in packed lower storage, and
// log det Sigma_C from a binary64 Cholesky (the same operations in the same
// order as the host's, one row per lane); a non-positive pivot gives ENOTPD.
// Displaced states: the root has the mean row [0, mu_C] first, and the
// forward solve with the Cholesky factor gives mu_C^T Sigma_C^-1 mu_C for the
// error bound (as the host computes it).  A full pattern of an inverted state
// (jac) gathers G = sigma_Q^-1 over C instead; its binary64 log det G gives
// log det Sigma_C = -log det G, log P_vac(N) and the factor (-1)^n det(G)^1/2
// that turns the tree's sum of G into the sum of Sigma_C.
template <class S>
__global__ __launch_bounds__(64) void async_gather_kernel(const double *__restrict__ cov, AsyncPlan P) {
    __shared__ double L[2 * TOR_MAX_N][2 * TOR_MAX_N];
    __shared__ double z[2 * TOR_MAX_N];
    __shared__ double piv;
    __shared__ int ok;
    const int lane = threadIdx.x;
    const size_t ld = 2 * (size_t)P.m;
    for (int q = blockIdx.x; q < P.nq; q += gridDim.x) {
        AsyncQuery &Q = P.q[q];
        const bool run = Q.status == TOR_OK && Q.n > 0;  // uniform over the block
        if (!run) continue;
        const int n = Q.n, d = 2 * n, o = P.D;
        S *root = (S *)P.pool + Q.pool_off;
        for (int e = lane; e < EN(n, o); e += 64) {
            int a, b;
            unpack(e, a, b);
            if (o && b == 0) {  // mean column (0 at the corner); h = K mu for the information form
                const int ga = a == 0 ? 0 : 2 * Q.C[(a - 1) >> 1] + ((a - 1) & 1);
                if (a == 0) root[e] = from_pair<S>(0.0, 0.0);
                else if (Q.jac) root[e] = from_pair<S>(((const dd *)P.inv_h)[ga].hi, ((const dd *)P.inv_h)[ga].lo);
                else root[e] = from_pair<S>(P.mean[ga], 0.0);
                continue;
            }
            a -= o;
            b -= o;
            const int ga = 2 * Q.C[a >> 1] + (a & 1), gb = 2 * Q.C[b >> 1] + (b & 1);
            const int r = ga > gb ? ga : gb, c = ga > gb ? gb : ga;
            dd x;
            if (Q.jac) {
                x = ((const dd *)P.inv)[pidx(r, c)];
            } else {
                const double v = cov[(size_t)r * ld + (size_t)c];
                if (ga == gb) two_sum(v, 0.5, x.hi, x.lo);
                else x = dd_from(v);
            }
            root[pidx(a + o, b + o)] = from_pair<S>(x.hi, x.lo);
            L[a][b] = x.hi + x.lo;
        }
        if (lane == 0) ok = 1;
        __syncthreads();
        double logdet = 0.0;
        for (int j = 0; j < d; j++) {
            if (lane == 0) {
                double s = L[j][j];
                for (int t = 0; t < j; t++) s -= L[j][t] * L[j][t];
                if (!(s > 0.0)) ok = 0;
                piv = sqrt(s);
                L[j][j] = piv;
                logdet += log(s);
            }
            __syncthreads();
            for (int i = j + 1 + lane; i < d; i += 64) {
                double v = L[i][j];
                for (int t = 0; t < j; t++) v -= L[i][t] * L[j][t];
                L[i][j] = v / piv;
            }
            __syncthreads();
        }
        if (lane == 0) {
            Q.log_det = Q.jac ? -logdet : logdet;
            if (!ok) Q.status = TOR_ENOTPD;
            if (Q.jac && ok && !o) {
                Q.jscale = ((n & 1) ? -1.0 : 1.0) * exp(0.5 * logdet);
                Q.log_pvac = -0.5 * (P.log_det_sigq + logdet);
            }
            if (o && ok) {  // z = L^-1 mu_C (h_C for the information form), quad = |z|^2
                double quad = 0.0;
                for (int a = 0; a < d; a++) {
                    const int ga = 2 * Q.C[a >> 1] + (a & 1);
                    double v = Q.jac ? ((const dd *)P.inv_h)[ga].hi + ((const dd *)P.inv_h)[ga].lo : P.mean[ga];
                    for (int t = 0; t < a; t++) v -= L[a][t] * z[t];
                    z[a] = v / L[a][a];
                    quad += z[a] * z[a];
                }
                Q.quad = quad;
                if (Q.jac) {  // T(Sigma_C) = (-1)^n det(G)^1/2 exp(-quad / 2) T_h(G)
                    Q.jscale = ((n & 1) ? -1.0 : 1.0) * exp(0.5 * logdet - 0.5 * quad);
                    Q.log_pvac = -0.5 * (P.log_det_sigq + logdet) - 0.5 * P.mu_k_mu + 0.5 * quad;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- results

__global__ void async_finalize_kernel(AsyncPlan P, double tol, int prec_used, tor_result *__restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.nq) return;
    const AsyncQuery &Q = P.q[q];
    tor_result r;
    r.p = r.p_lo = r.log_p = r.tor = r.T = r.T_lo = r.abs_sum = r.cancel_ratio = r.rel_err_bound = 0.0;
    r.log_pvac_n = 0.0;
    r.n_clicks = r.prec_used = 0;
    r.reserved = 0;
    r.status = Q.status;
    if (Q.status != TOR_OK) {
        out[q] = r;
        return;
    }
    dd T = dd_from(1.0);
    double A = 1.0;
    if (Q.n > 0) {
        const Partial p = (Q.final_buf ? P.partB : P.partA)[Q.final_off];
        T = dd_make(p.t_hi, p.t_lo);
        A = p.a;
    }
    if (!isfinite(T.hi) || !isfinite(A)) {
        r.status = TOR_ENOTPD;
        out[q] = r;
        return;
    }
    // marginal pattern: P_vac(N) = 1, p = T.  Full pattern of an inverted
    // state: p = (-1)^n det(sigma_Q)^-1/2 T(G) (as the host forms it), and the
    // reported sums are those of Sigma_C, T(Sigma_C) = jscale T(G).
    dd pr;
    if (Q.jac) {
        const double sg = (Q.n & 1) ? -1.0 : 1.0;
        pr = dd_mul(dd_make(sg * P.det_rsqrt_hi, sg * P.det_rsqrt_lo), T);
        T = dd_mul_d(T, Q.jscale);
        A *= fabs(Q.jscale);
    } else {
        pr = dd_mul(dd_from(1.0), T);
    }
    r.p = pr.hi + pr.lo;
    r.p_lo = pr.lo - (r.p - pr.hi);
    r.log_p = r.p > 0 ? Q.log_pvac + log(T.hi) + log1p(T.lo / T.hi) : -INFINITY;
    r.log_pvac_n = Q.log_pvac;
    r.T = T.hi;
    r.T_lo = T.lo;
    r.tor = exp(0.5 * Q.log_det) * (T.hi + T.lo);
    r.abs_sum = A;
    r.cancel_ratio = A / fabs(T.hi);
    const double u = prec_used == TOR_PREC_DD ? 4.930380657631324e-32 : 1.1102230246251565e-16;
    // the host's bound: the tree's n u plus, for a full pattern of an inverted
    // state, the roundoff of the sweeps that formed the inverse
    const double cu = Q.jac ? P.inv_cond_u : 0.0;
    r.rel_err_bound = 16.0 * ((Q.n > 1 ? Q.n : 1) * u + cu) * (A / fabs(T.hi)) * (1.0 + Q.quad);
    r.n_clicks = Q.n;
    r.prec_used = prec_used;
    r.status = r.rel_err_bound <= tol ? TOR_OK : TOR_WARN_PRECISION;
    out[q] = r;
}

}  // namespace tor

hipError_t tor_launch_async_prologue(const int8_t *d_patterns, const double *d_cov, const AsyncPlan &P,
                                     hipStream_t st) {
    if (P.nq < 1) return hipSuccess;
    const unsigned g = (unsigned)(P.nq < 65536 ? P.nq : 65536);
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::async_scan_kernel, dim3(g), dim3(64), 0, st, d_patterns, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::async_plan_kernel, dim3(1), dim3(tor::kPlanThreads), 0, st, P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    (void)hipGetLastError();  // report only this launch's error
    if (P.is_dd) hipLaunchKernelGGL(tor::async_gather_kernel<dd>, dim3(g), dim3(64), 0, st, d_cov, P);
    else hipLaunchKernelGGL(tor::async_gather_kernel<double>, dim3(g), dim3(64), 0, st, d_cov, P);
    return hipGetLastError();
}

hipError_t tor_launch_async_finalize(const AsyncPlan &P, double tol, int prec_used, void *d_out, hipStream_t st) {
    if (P.nq < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::async_finalize_kernel, dim3((unsigned)((P.nq + 255) / 256)), dim3(256), 0, st, P, tol,
                       prec_used, (tor_result *)d_out);
    return hipGetLastError();
}
