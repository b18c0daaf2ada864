// Single-launch subset sums of small zero-mean trees (n <= TOR_FUSED_MAX_N).
//
// The batched path evaluates a tree in a chain of launches: one expansion
// launch per HBM level, the wave tier, the reduction stages and a gather.  For
// a tree of 2^20 subsets that chain, not the arithmetic, sets the time.  Here
// one launch does all of it.  The tree's 2^(n - J) wave-tier tasks are split
// into units of 2^t consecutive tasks; a one-wave workgroup takes a unit:
//   1. it copies Sigma_C (packed lower) into LDS and takes the unit's g = n - J
//      - t decisions there, each include decision an in-place Schur update of
//      the last mode's 2x2 pivot block (Sec. II, Eq. MatrixUpdate) and a factor
//      q = det(pivot)^-1/2 on the path coefficient -- the expansion's update,
//      operation for operation, so the unit's node is bitwise the batched
//      path's node at that depth;
//   2. it walks the unit's last t decisions depth first in its own global
//      scratch and sums each task's subtree with the wave tier;
//   3. completion counters order the reduction: the workgroup that finishes
//      the last unit of a block of TOR_REDUCE_CHUNK tasks sums that block (the
//      first reduction stage), and the one that finishes the last block sums
//      the block sums (the second stage) and writes (T, A) to host memory.
// Task partials, block sums and their order are those of the batched path, so
// results are bitwise equal to it for the same task size J.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor_kernels.h"
#include "tor_tree.hpp"
#include "tor_wave.hpp"

#pragma clang fp contract(off)

namespace tor {

// The wave-tier working set of a J-mode task: the nine-mode set plus set-aside
// pivot columns for J = 10, 11.
template <class S, int J> struct FzTask {
    using type = WaveSmem<S, J, 0>;
};
template <class S> struct FzTask<S, 10> {
    using type = TopSmem<S, 0, 1>;
};
template <class S> struct FzTask<S, 11> {
    using type = TopSmem<S, 0, 2>;
};

// Byte offset of the prefix matrix and of the reduction arrays in the shared
// region: after the wave tier's packed-index table, which is filled once per
// workgroup and kept.
constexpr int kFzOffset = 512;

template <class S, int J> union FzLds {
    typename FzTask<S, J>::type task;
    struct {
        unsigned char pad[kFzOffset];
        S m[EN(TOR_FUSED_MAX_N, 0)];
    } pre;
    struct {
        unsigned char pad[kFzOffset];
        dd T[256];
        double A[256];
    } red;
};
static_assert(sizeof(unsigned short) * ab_n(0) <= kFzOffset, "the index table lies before the prefix");

struct FzPath {  // node of each depth-first level (wave-uniform)
    const void *node[TOR_FUSED_TMAX + 1];
    dd c[TOR_FUSED_TMAX + 1];
    double a[TOR_FUSED_TMAX + 1];
};

template <class S, int J> struct FzOcc {
    static constexpr int value =
        sizeof(FzLds<S, J>) + sizeof(FzPath) + 2 * (2 * TOR_FUSED_MAX_N - 2) * sizeof(S) + 512 <= 20480 ? 2 : 1;
};

// Ordering of a wave's global stores before its own lanes' later loads of them.
__device__ __forceinline__ void fz_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The two scaled pivot columns of the r-mode node m's last mode into vt.
template <class S>
__device__ __forceinline__ Pivot<S> fz_columns(const S *m, int r, S *vt, int lane) {
    const int R = 2 * r, RC = R - 2;
    const Pivot<S> pv = make_pivot_m<S, 0>(m, R - 2, R - 1);
    for (int c = lane; c < RC; c += 64) {
        const S c0 = m[pidx(R - 2, c)];
        vt[c] = mul_s(c0, pv.s1);
        vt[RC + c] = mul_s(sub_mul(m[pidx(R - 1, c)], pv.l, c0), pv.s2);
    }
    wave_sync();
    return pv;
}

// Include child of the r-mode node `in` written to `out` (in == out: in place;
// an entry of the child needs only itself and the pivot columns).  A lane
// takes four of its entries per pass, every operand loaded before the first
// store, so that four independent double-double chains overlap (one wave per
// SIMD has no other work to hide their latency).
template <class S>
__device__ __forceinline__ void fz_entry(const S *in, const S *vt, int RC, int e, S &x, S &va, S &vb, S &wa, S &wb) {
    int a, b;
    unpack(e, a, b);
    x = in[e];
    va = vt[a];
    vb = vt[b];
    wa = vt[RC + a];
    wb = vt[RC + b];
}

template <class S>
__device__ __forceinline__ Pivot<S> fz_include(const S *in, int r, S *out, S *vt, int lane) {
    const int RC = 2 * r - 2, EC = EN(r - 1, 0);
    const Pivot<S> pv = fz_columns<S>(in, r, vt, lane);
    int e = lane;
    for (; e + 192 < EC; e += 256) {
        S x[4], va[4], vb[4], wa[4], wb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) fz_entry<S>(in, vt, RC, e + 64 * k, x[k], va[k], vb[k], wa[k], wb[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = sub_dot2(x[k], va[k], vb[k], wa[k], wb[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) out[e + 64 * k] = x[k];
    }
    for (; e < EC; e += 64) {
        S x, va, vb, wa, wb;
        fz_entry<S>(in, vt, RC, e, x, va, vb, wa, wb);
        out[e] = sub_dot2(x, va, vb, wa, wb);
    }
    return pv;
}

template <class S, int J>
__device__ __forceinline__ void fz_task(FzLds<S, J> &L, const S *node, dd c, double a, int lane, dd &T, double &A) {
    if constexpr (J <= 9) wave_task<S, J, 0>(L.task, node, c, a, lane, T, A);
    else wave_task_top<S, J, 0>(L.task, node, c, a, lane, T, A);
}

// Sum of in[0 .. count), count <= TOR_REDUCE_CHUNK, in the order of one block
// of the batched reduction: 256 strided sequential sums (four per lane), then
// a fixed pairwise tree.
// All of a lane's partials are loaded before the first addition (the block
// is read once, in one round trip, right after the claim); the additions then
// run in the block's order.
template <class S, int J>
__device__ __forceinline__ Partial fz_block_sum(const Partial *in, long long count, FzLds<S, J> &L, int lane) {
    constexpr int PER = TOR_REDUCE_CHUNK / 256;  // partials per strided sum
    Partial pp[4][PER];
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const long long k = lane + 64 * w + 256 * i;
            if (k < count) pp[w][i] = in[k];
        }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        dd T = dd_from(0.0);
        double A = 0.0;
#pragma unroll
        for (int i = 0; i < PER; ++i)
            if (lane + 64 * w + 256 * i < count) {
                T = dd_add(T, dd_make(pp[w][i].t_hi, pp[w][i].t_lo));
                A += pp[w][i].a;
            }
        L.red.T[lane + 64 * w] = T;
        L.red.A[lane + 64 * w] = A;
    }
    wave_sync();
    for (int s = 128; s > 0; s >>= 1) {
        for (int v = lane; v < s; v += 64) {
            L.red.T[v] = dd_add(L.red.T[v], L.red.T[v + s]);
            L.red.A[v] = L.red.A[v] + L.red.A[v + s];
        }
        wave_sync();
    }
    Partial p;
    p.t_hi = L.red.T[0].hi;
    p.t_lo = L.red.T[0].lo;
    p.a = L.red.A[0];
    p.pad = 0.0;
    wave_sync();
    return p;
}

// Lane 0 adds one to *ctr (device scope, after every earlier store of the
// wave is released); every lane gets the value before the add.
__device__ __forceinline__ unsigned fz_count(unsigned *ctr, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    unsigned old = 0;
    if (lane == 0) old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = (unsigned)__shfl((int)old, 0);
    return old;
}

__device__ __forceinline__ void fz_claimed(unsigned *ctr, int lane) {
    if (lane == 0) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // ready for the next launch
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void fz_result(Partial *res, const Partial &p, int lane) {
    if (lane == 0) *res = p;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: the host reads it after the stream
}

template <class S, int J>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FzOcc<S, J>::value))) void fused_tree_kernel(
    const FusedJob *__restrict__ jobs, int njobs, long long units, S *__restrict__ ws, long long ws_stride) {
    __shared__ FzLds<S, J> L;
    __shared__ FzPath path;
    __shared__ S vt[2 * (2 * TOR_FUSED_MAX_N - 2)];
    const int lane = threadIdx.x;
    wave_tree_init<0>(reinterpret_cast<unsigned short *>(&L), lane);  // the table at offset 0 of every task set
    S *const wsb = ws + (long long)blockIdx.x * ws_stride;
    for (long long U = blockIdx.x; U < units; U += gridDim.x) {
        const int j = find_job(jobs, njobs, U);
        const FusedJob jb = jobs[j];
        const long long u = U - jb.begin;
        const int n = jb.n, g = jb.g, t = jb.t, r0 = n - g;  // r0 = J + t: modes of the unit's node
        // 1. the unit's g decisions in LDS, most significant bit first
        S *pm = L.pre.m;
        const S *root = (const S *)jb.root;
        for (int e = lane; e < EN(n, 0); e += 64) pm[e] = root[e];
        wave_sync();
        dd c = dd_from(1.0);
        double a = 1.0;
        for (int k = 0, r = n; k < g; ++k, --r) {
            if ((u >> (g - 1 - k)) & 1) {
                const Pivot<S> pv = fz_include<S>(pm, r, pm, vt, lane);
                wave_sync();
                c = dd_neg(coef_mul(c, pv.q));
                a = a * hi_of(pv.q);
            }
        }
        const long long EW = EN(r0, 0);
        for (int e = lane; e < EW; e += 64) wsb[e] = pm[e];
        fz_sync();
        if (lane == 0) {
            path.node[0] = wsb;
            path.c[0] = c;
            path.a[0] = a;
        }
        wave_sync();
        // 2. the unit's 2^t tasks depth first (levels from the first decision
        //    where q differs from q - 1)
        for (long long q = 0; q < (1LL << t); ++q) {
            const int f = q == 0 ? 0 : t - 1 - __builtin_ctzll((unsigned long long)q);
            for (int k = f; k < t; ++k) {
                const S *par = (const S *)path.node[k];
                const dd pc = path.c[k];
                const double pa = path.a[k];
                wave_sync();
                if ((q >> (t - 1 - k)) & 1) {
                    S *out = wsb + (1 + k) * EW;
                    const Pivot<S> pv = fz_include<S>(par, r0 - k, out, vt, lane);
                    fz_sync();
                    if (lane == 0) {
                        path.node[k + 1] = out;
                        path.c[k + 1] = dd_neg(coef_mul(pc, pv.q));
                        path.a[k + 1] = pa * hi_of(pv.q);
                    }
                } else if (lane == 0) {
                    path.node[k + 1] = par;
                    path.c[k + 1] = pc;
                    path.a[k + 1] = pa;
                }
                wave_sync();
            }
            dd T;
            double A;
            fz_task<S, J>(L, (const S *)path.node[t], path.c[t], path.a[t], lane, T, A);
            if (lane == 0) {
                Partial p;
                p.t_hi = T.hi;
                p.t_lo = T.lo;
                p.a = A;
                p.pad = 0.0;
                jb.part[(u << t) + q] = p;
            }
            wave_sync();
        }
        // 3. completion and the two reduction stages
        const long long tasks = 1LL << (g + t);
        if (tasks == 1) {  // a single task: no reduction stage
            fz_sync();
            fz_result(jb.res, jb.part[0], lane);
            continue;
        }
        const long long blk = (u << t) / TOR_REDUCE_CHUNK;
        const long long blk_tasks = tasks < TOR_REDUCE_CHUNK ? tasks : TOR_REDUCE_CHUNK;
        const long long nblk = (tasks + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
        if (fz_count(&jb.ctr[1 + blk], lane) + 1 != (unsigned)(blk_tasks >> t)) continue;
        fz_claimed(&jb.ctr[1 + blk], lane);
        const Partial s1 = fz_block_sum<S, J>(jb.part + blk * TOR_REDUCE_CHUNK, blk_tasks, L, lane);
        if (nblk == 1) {
            fz_result(jb.res, s1, lane);
            continue;
        }
        if (lane == 0) jb.part[tasks + blk] = s1;
        if (fz_count(&jb.ctr[0], lane) + 1 != (unsigned)nblk) continue;
        fz_claimed(&jb.ctr[0], lane);
        fz_result(jb.res, fz_block_sum<S, J>(jb.part + tasks, nblk, L, lane), lane);
    }
}

template <class S, int J>
static hipError_t launch_fused_J(const FusedJob *jobs, int njobs, long long units, void *ws, long long ws_stride,
                                 int grid, hipStream_t st) {
    if (units < 1 || grid < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL((fused_tree_kernel<S, J>), dim3((unsigned)grid), dim3(64), 0, st, jobs, njobs, units,
                       (S *)ws, ws_stride);
    return hipGetLastError();
}

template <class S>
static hipError_t launch_fused_S(int J, const FusedJob *jobs, int njobs, long long units, void *ws,
                                 long long ws_stride, int grid, hipStream_t st) {
    switch (J) {
    case 1: return launch_fused_J<S, 1>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 2: return launch_fused_J<S, 2>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 3: return launch_fused_J<S, 3>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 4: return launch_fused_J<S, 4>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 5: return launch_fused_J<S, 5>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 6: return launch_fused_J<S, 6>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 7: return launch_fused_J<S, 7>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 8: return launch_fused_J<S, 8>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 9: return launch_fused_J<S, 9>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 10: return launch_fused_J<S, 10>(jobs, njobs, units, ws, ws_stride, grid, st);
    case 11: return launch_fused_J<S, 11>(jobs, njobs, units, ws, ws_stride, grid, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tor

hipError_t tor_launch_fused(int is_dd, int J, const FusedJob *jobs, int njobs, long long units, void *ws,
                            long long ws_stride, int grid, hipStream_t st) {
    return is_dd ? tor::launch_fused_S<dd>(J, jobs, njobs, units, ws, ws_stride, grid, st)
                 : tor::launch_fused_S<double>(J, jobs, njobs, units, ws, ws_stride, grid, st);
}
