// Wave-tier kernels of the subset tree (the LDS and register tiers), templated
// on the scalar S (binary64 or double-double), the task size J (modes per
// workgroup task) and the mean-row mode D (0: zero-mean state; 1: displaced
// state, the packed matrix carries the mean vector as its first row; -1: the
// information form, the first row holds sigma_Q^-1 mu and the pivots carry
// exp(+|w|^2 / 2)).  Each
// translation unit that includes this header instantiates the launchers it
// needs, so the zero-mean and displaced kernels compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "tor_kernels.h"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

// Waves per SIMD the wave tier asks the register allocator for: two where five
// or more one-wave workgroups fit the CU's 160 KiB of LDS, so that some SIMD
// can hold a second wave to hide the first one's latency; else one.  The
// double-double leaf with a mean row (one more packed row per node) does not
// fit the 256 registers of two waves without spilling, so it asks for one.
template <class S, int J, int D> struct WaveOcc {
    static constexpr int value = (D != 0 && sizeof(S) > sizeof(double)) ? 1
                                 : (sizeof(WaveSmem<S, J, D>) + 1024) * 5 <= 163840 ? 2 : 1;
};

// One wave-tier task of J <= 9 modes: the node's matrix at root (global
// memory) with path coefficient (c, a); every lane returns the task's (T, A).
template <class S, int J, int D>
__device__ __forceinline__ void wave_task(WaveSmem<S, J, D> &sm, const S *root, dd c, double a, int lane, dd &T,
                                          double &A) {
    for (int e = lane; e < EN(J, MR(D)); e += 64) sm.mat[e] = root[e];
    wave_tree<S, J, D>(sm, c, a, lane, T, A);
    wave_reduce(T, A);
}

template <class S, int J, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WaveOcc<S, J, D>::value))) void wave_kernel(
    const WaveJob *__restrict__ jobs, int njobs, long long total, const S *__restrict__ pool,
    const LaunchDims *__restrict__ dyn) {
    __shared__ WaveSmem<S, J, D> sm;
    const int lane = threadIdx.x;
    if (dyn) {
        njobs = (int)dyn->njobs;
        total = dyn->total;
    }
    wave_tree_init<D>(sm.ab, lane);
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int j = find_job(jobs, njobs, t);
        const long long lt = t - jobs[j].begin;
        NodeDesc d = jobs[j].tasks[lt];
        dd T;
        double A;
        wave_task<S, J, D>(sm, pool + d.off, dd_make(d.coef_hi, d.coef_lo), d.acoef, lane, T, A);
        if (lane == 0) {
            Partial p;
            p.t_hi = T.hi;
            p.t_lo = T.lo;
            p.a = A;
            p.pad = 0.0;
            jobs[j].out[lt] = p;
        }
        wave_sync();
    }
}

// Tasks of 10 or 11 modes: the top one or two decisions are taken in LDS,
// depth first, above the nine-mode tree.  At a 10-mode node the pivot columns
// of its last mode are set aside, the exclude child (the leading nine-mode
// block, in place) is summed by the nine-mode tree, then the include child is
// formed in place over that block (the HBM tier's update) and summed the same
// way.  An 11-mode task sums its exclude child (the leading 10-mode block) so,
// then rebuilds its include child from the task's matrix, still in HBM, and
// sums that.  Each top level saves one HBM level for a few hundred bytes of LDS.
template <class S, int D, int NT> struct TopSmem {  // NT = J - 9 set-aside column pairs
    WaveSmem<S, 9, D> w;
    S vtop[NT][2 * (2 * TOR_TASK_MAX - 2 + MR(D))];
};

// pivot of the last mode of the r-mode node m[] and its two scaled columns
template <class S, int r, int D>
__device__ __forceinline__ Pivot<S> top_columns(const S *m, S *v, int lane) {
    constexpr int R = 2 * r + MR(D), RC = R - 2;
    // every lane forms the pivot (same value everywhere, no LDS round trip)
    const Pivot<S> pv = make_pivot_m<S, D>(m, R - 2, R - 1);
    for (int c = lane; c < RC; c += 64) {
        S m0 = m[pidx(R - 2, c)];
        v[c] = mul_s(m0, pv.s1);
        v[RC + c] = mul_s(sub_mul(m[pidx(R - 1, c)], pv.l, m0), pv.s2);
    }
    return pv;
}

// dst[e] = src[e] - v1(a) v1(b) - v2(a) v2(b) for the (r-1)-mode child, e < EN(r-1, MR(D))
template <class S, int r, int D>
__device__ __forceinline__ void top_update(const S *src, S *dst, const S *v, int lane) {
    constexpr int RC = 2 * r - 2 + MR(D);
    for (int e = lane; e < EN(r - 1, MR(D)); e += 64) {
        int a, b;
        unpack(e, a, b);
        dst[e] = sub_dot2(src[e], v[a], v[b], v[RC + a], v[RC + b]);
    }
}

// the 10-mode node in sm.w.mat[0 .. EN(10, MR(D))); adds this lane's share to (T, A)
template <class S, int D, int NT>
__device__ __forceinline__ void top10(TopSmem<S, D, NT> &sm, dd c, double a, int lane, dd &T, double &A) {
    S *v = sm.vtop[0];
    const Pivot<S> pv = top_columns<S, 10, D>(sm.w.mat, v, lane);
    wave_sync();
    dd t;
    double x;
    wave_tree<S, 9, D>(sm.w, c, a, lane, t, x);
    T = dd_add(T, t);
    A += x;
    wave_sync();
    top_update<S, 10, D>(sm.w.mat, sm.w.mat, v, lane);
    wave_sync();
    wave_tree<S, 9, D>(sm.w, dd_neg(coef_mul(c, pv.q)), a * hi_of(pv.q), lane, t, x);
    T = dd_add(T, t);
    A += x;
}

// One wave-tier task of J = 10 or 11 modes (the node's matrix at root, which
// stays readable: the 11-mode task rebuilds its include child from it); every
// lane returns the task's (T, A).
template <class S, int J, int D>
__device__ __forceinline__ void wave_task_top(TopSmem<S, D, J - 9> &sm, const S *root, dd c0, double a0, int lane,
                                              dd &T, double &A) {
    static_assert(J == 10 || J == 11, "top levels: one or two");
    static_assert(WaveCfg<S, 9, D>::MAT >= EN(J, MR(D)), "the task's matrix must fit the nine-mode working set");
    for (int e = lane; e < EN(J, MR(D)); e += 64) sm.w.mat[e] = root[e];
    wave_sync();
    T = dd_from(0.0);
    A = 0.0;
    if constexpr (J == 10) {
        top10<S, D, J - 9>(sm, c0, a0, lane, T, A);
    } else {
        S *v = sm.vtop[1];
        const Pivot<S> pv = top_columns<S, 11, D>(sm.w.mat, v, lane);
        wave_sync();
        top10<S, D, J - 9>(sm, c0, a0, lane, T, A);
        wave_sync();
        top_update<S, 11, D>(root, sm.w.mat, v, lane);
        wave_sync();
        top10<S, D, J - 9>(sm, dd_neg(coef_mul(c0, pv.q)), a0 * hi_of(pv.q), lane, T, A);
    }
    wave_reduce(T, A);
}

template <class S, int J, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WaveOcc<S, 9, D>::value))) void wave_kernel_top(
    const WaveJob *__restrict__ jobs, int njobs, long long total, const S *__restrict__ pool,
    const LaunchDims *__restrict__ dyn) {
    __shared__ TopSmem<S, D, J - 9> sm;
    const int lane = threadIdx.x;
    if (dyn) {
        njobs = (int)dyn->njobs;
        total = dyn->total;
    }
    wave_tree_init<D>(sm.w.ab, lane);
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int j = find_job(jobs, njobs, t);
        const long long lt = t - jobs[j].begin;
        NodeDesc d = jobs[j].tasks[lt];
        dd T;
        double A;
        wave_task_top<S, J, D>(sm, pool + d.off, dd_make(d.coef_hi, d.coef_lo), d.acoef, lane, T, A);
        if (lane == 0) {
            Partial p;
            p.t_hi = T.hi;
            p.t_lo = T.lo;
            p.a = A;
            p.pad = 0.0;
            jobs[j].out[lt] = p;
        }
        wave_sync();
    }
}

// With dyn (a plan made on the device) njobs and total are read from dyn by the
// kernel and grid_cap is the grid itself.
template <class S, int J, int D>
static hipError_t launch_wave_J(const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                                hipStream_t st, const LaunchDims *dyn) {
    long long g = dyn ? grid_cap : (total < grid_cap ? total : grid_cap);
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL((wave_kernel<S, J, D>), dim3((unsigned)g), dim3(64), 0, st, jobs, njobs, total,
                       (const S *)pool, dyn);
    return hipGetLastError();
}

template <class S, int J, int D>
static hipError_t launch_wave_top(const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                                  hipStream_t st, const LaunchDims *dyn) {
    long long g = dyn ? grid_cap : (total < grid_cap ? total : grid_cap);
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL((wave_kernel_top<S, J, D>), dim3((unsigned)g), dim3(64), 0, st, jobs, njobs, total,
                       (const S *)pool, dyn);
    return hipGetLastError();
}

template <class S, int D>
static hipError_t launch_wave_S(int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                                int grid_cap, hipStream_t st, const LaunchDims *dyn) {
    switch (J) {
    case 1: return launch_wave_J<S, 1, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 2: return launch_wave_J<S, 2, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 3: return launch_wave_J<S, 3, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 4: return launch_wave_J<S, 4, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 5: return launch_wave_J<S, 5, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 6: return launch_wave_J<S, 6, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 7: return launch_wave_J<S, 7, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 8: return launch_wave_J<S, 8, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 9: return launch_wave_J<S, 9, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 10: return launch_wave_top<S, 10, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    case 11: return launch_wave_top<S, 11, D>(jobs, njobs, total, pool, grid_cap, st, dyn);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tor
