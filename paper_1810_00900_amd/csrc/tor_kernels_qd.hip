// Quad-double term tier of the subset tree: the same three tiers as the
// binary64 and double-double kernels (HBM expansion, LDS wave tree, register
// leaves), with every matrix entry, pivot quantity, path coefficient and sum
// in quad-double (qd.hpp).  For sums whose cancellation ratio R is beyond
// double-double terms (full click patterns conditioned on hundreds of
// no-click modes): the relative error bound 16 n u R becomes 16 n 2^-208 R.
//
// The path coefficient of a node lives in its pool slot, one word before the
// packed matrix, so descriptors keep the layout of the other tiers.  D = 1: a
// displaced state, the packed matrices carry the mean row first (the pivots'
// overlap factors exp(-|w|^2 / 2) by the quad-double exp); D = -1: the
// information form of an inverted displaced state's full patterns (the first
// row holds sigma_Q^-1 mu, the factors are exp(+|w|^2 / 2)).
#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "qd.hpp"
#include "tor_kernels.h"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

// One 64-lane workgroup per task of J <= 8 modes (LDS 50 KB at J = 8: three
// workgroups per CU, one wave per SIMD for the register leaf).
template <int J, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1))) void wave_kernel_qd(
    const WaveJob *__restrict__ jobs, int njobs, long long total, const qd *__restrict__ pool) {
    __shared__ WaveSmem<qd, J, D> sm;
    const int lane = threadIdx.x;
    wave_tree_init<D>(sm.ab, lane);
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int j = find_job(jobs, njobs, t);
        const long long lt = t - jobs[j].begin;
        const NodeDesc d = jobs[j].tasks[lt];
        const qd *root = pool + d.off;
        for (int e = lane; e < EN(J, MR(D)); e += 64) sm.mat[e] = root[e];
        const qd c = root[-1];
        qd T;
        double A;
        wave_tree<qd, J, D>(sm, c, d.acoef, lane, T, A);
        wave_reduce(T, A);
        if (lane == 0) {
            PartialQ p;
            p.t0 = T.x0;
            p.t1 = T.x1;
            p.t2 = T.x2;
            p.t3 = T.x3;
            p.a = A;
            p.pad0 = p.pad1 = p.pad2 = 0.0;
            reinterpret_cast<PartialQ *>(jobs[j].out)[lt] = p;
        }
        wave_sync();
    }
}

// One wave per parent node (four per 256-thread workgroup): the include child
// goes to the pool with its coefficient -c q in the word before it.
template <int D>
__global__ __launch_bounds__(256) void expand_kernel_qd(const ExpandJob *__restrict__ jobs, int log2npar,
                                                        long long total, qd *__restrict__ pool) {
    __shared__ qd vs[4][2][2 * TOR_MAX_N + MR(D)];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    qd *v0 = vs[w][0], *v1 = vs[w][1];
    for (long long f = (long long)blockIdx.x * 4 + w; f < total; f += (long long)gridDim.x * 4) {
        const ExpandJob job = jobs[f >> log2npar];
        const long long i = f & ((1LL << log2npar) - 1);
        const int r = job.r, R = 2 * r + MR(D), RC = R - 2, EC = EN(r - 1, MR(D));
        const NodeDesc d = job.par[i];
        const qd *base = pool + d.off;
        const Pivot<qd> pv = make_pivot_m<qd, D>(base, R - 2, R - 1);
        const unsigned long long coff = job.child_base + (unsigned long long)i * (unsigned long long)(EC + 1) + 1;
        if (lane == 0) {
            job.chi[2 * i] = d;
            NodeDesc c;
            c.off = coff;
            c.coef_hi = 0.0;
            c.coef_lo = 0.0;
            c.acoef = d.acoef * hi_of(pv.q);
            job.chi[2 * i + 1] = c;
            pool[coff - 1] = qd_neg(qd_mul(base[-1], pv.q));
        }
        for (int c = lane; c < RC; c += 64) {
            const qd m0 = base[pidx(R - 2, c)];
            v0[c] = qd_mul(m0, pv.s1);
            v1[c] = qd_mul(qd_sub_mul(base[pidx(R - 1, c)], pv.l, m0), pv.s2);
        }
        wave_sync();
        qd *outp = pool + coff;
        for (int e = lane; e < EC; e += 64) {
            int a, b;
            unpack(e, a, b);
            outp[e] = qd_sub_dot2(base[e], v0[a], v0[b], v1[a], v1[b]);
        }
        wave_sync();
    }
}

// Fixed-order block sums of per-task partials (as reduce_kernel, in qd).
__global__ __launch_bounds__(256) void reduce_kernel_qd(const ReduceJobQ *__restrict__ jobs, int njobs,
                                                        long long total_blocks) {
    __shared__ qd sT[256];
    __shared__ double sA[256];
    for (long long gb = blockIdx.x; gb < total_blocks; gb += gridDim.x) {
        int lo_j = 0, hi_j = njobs - 1;
        while (lo_j < hi_j) {
            int mid = (lo_j + hi_j + 1) >> 1;
            if (jobs[mid].block_begin <= gb) lo_j = mid;
            else hi_j = mid - 1;
        }
        const ReduceJobQ job = jobs[lo_j];
        const long long b = gb - job.block_begin;
        const long long lo = b * TOR_REDUCE_CHUNK;
        const long long hi = lo + TOR_REDUCE_CHUNK < job.count ? lo + TOR_REDUCE_CHUNK : job.count;
        qd T = qd_from(0.0);
        double A = 0.0;
        for (long long k = lo + threadIdx.x; k < hi; k += blockDim.x) {
            const PartialQ p = job.in[k];
            T = qd_add(T, qd_make(p.t0, p.t1, p.t2, p.t3));
            A += p.a;
        }
        sT[threadIdx.x] = T;
        sA[threadIdx.x] = A;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                sT[threadIdx.x] = qd_add(sT[threadIdx.x], sT[threadIdx.x + s]);
                sA[threadIdx.x] = sA[threadIdx.x] + sA[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            PartialQ p;
            p.t0 = sT[0].x0;
            p.t1 = sT[0].x1;
            p.t2 = sT[0].x2;
            p.t3 = sT[0].x3;
            p.a = sA[0];
            p.pad0 = p.pad1 = p.pad2 = 0.0;
            job.out[b] = p;
        }
        __syncthreads();
    }
}

// Vacuum conditioning in qd, two kernels per step.  First one block per job
// forms the pivot of the job's last mode and writes the two scaled pivot
// columns to the job's scratch (and multiplies the job's P_vac by q).
__global__ __launch_bounds__(256) void condition_cols_qd(const CondJobQ *__restrict__ jobs) {
    const CondJobQ job = jobs[blockIdx.x];
    const int r = job.r, R = 2 * r + (job.d ? 1 : 0), RC = R - 2;
    const qd *M = static_cast<const qd *>(job.mat);
    qd *cols = static_cast<qd *>(job.cols);
    const Pivot<qd> pv = job.d ? make_pivot_m<qd, 1>(M, R - 2, R - 1) : make_pivot_m<qd, 0>(M, R - 2, R - 1);
    for (int c = threadIdx.x; c < RC; c += blockDim.x) {
        const qd m0 = M[pidx(R - 2, c)];
        cols[c] = qd_mul(m0, pv.s1);
        cols[RC + c] = qd_mul(qd_sub_mul(M[pidx(R - 1, c)], pv.l, m0), pv.s2);
    }
    if (threadIdx.x == 0) {
        const dd q = qd_to_dd(pv.q);
        const dd p = dd_mul(dd_make(job.acc[0], job.acc[1]), q);
        job.acc[0] = p.hi;
        job.acc[1] = p.lo;
        job.acc[2] += log(q.hi) + log1p(q.lo / q.hi);
        if (job.qout) {
            job.qout[0] = q.hi;
            job.qout[1] = q.lo;
        }
    }
}

// Then the in-place rank-2 update of the leading block, TOR_COND_CHUNK
// entries per block (the last two rows, read by the first kernel, are not
// written).
__global__ __launch_bounds__(256) void condition_update_qd(const CondJobQ *__restrict__ jobs, int njobs) {
    const int j = find_job(jobs, njobs, (long long)blockIdx.x);
    const CondJobQ job = jobs[j];
    const long long blk = (long long)blockIdx.x - job.begin;
    const int r = job.r, RC = 2 * r - 2 + (job.d ? 1 : 0);
    qd *M = static_cast<qd *>(job.mat);
    const qd *cols = static_cast<const qd *>(job.cols);
    const int EC = job.d ? EN(r - 1, 1) : EN(r - 1, 0);
    const int e0 = (int)(blk * TOR_COND_CHUNK);
    const int e1 = e0 + TOR_COND_CHUNK < EC ? e0 + TOR_COND_CHUNK : EC;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        int a, b;
        unpack(e, a, b);
        M[e] = qd_sub_dot2(M[e], cols[a], cols[b], cols[RC + a], cols[RC + b]);
    }
}

template <int J, int D>
static hipError_t launch_qd_J(const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                              hipStream_t st) {
    const long long g = total < grid_cap ? total : grid_cap;
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL((wave_kernel_qd<J, D>), dim3((unsigned)g), dim3(64), 0, st, jobs, njobs, total,
                       (const qd *)pool);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_qd_D(int J, const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                              hipStream_t st) {
    switch (J) {
    case 1: return launch_qd_J<1, D>(jobs, njobs, total, pool, grid_cap, st);
    case 2: return launch_qd_J<2, D>(jobs, njobs, total, pool, grid_cap, st);
    case 3: return launch_qd_J<3, D>(jobs, njobs, total, pool, grid_cap, st);
    case 4: return launch_qd_J<4, D>(jobs, njobs, total, pool, grid_cap, st);
    case 5: return launch_qd_J<5, D>(jobs, njobs, total, pool, grid_cap, st);
    case 6: return launch_qd_J<6, D>(jobs, njobs, total, pool, grid_cap, st);
    case 7: return launch_qd_J<7, D>(jobs, njobs, total, pool, grid_cap, st);
    case 8: return launch_qd_J<8, D>(jobs, njobs, total, pool, grid_cap, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tor

hipError_t tor_launch_wave_qd(int J, const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                              hipStream_t st, int disp) {
    if (disp < 0) return tor::launch_qd_D<-1>(J, jobs, njobs, total, pool, grid_cap, st);
    return disp ? tor::launch_qd_D<1>(J, jobs, njobs, total, pool, grid_cap, st)
                : tor::launch_qd_D<0>(J, jobs, njobs, total, pool, grid_cap, st);
}

hipError_t tor_launch_expand_qd(const ExpandJob *jobs, int njobs, int log2npar, void *pool, int grid_cap,
                                hipStream_t st, int disp) {
    const long long total = (long long)njobs << log2npar;
    const long long blocks = (total + 3) / 4;
    const long long g = blocks < grid_cap ? blocks : grid_cap;
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    if (disp < 0)
        hipLaunchKernelGGL(tor::expand_kernel_qd<-1>, dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (qd *)pool);
    else if (disp)
        hipLaunchKernelGGL(tor::expand_kernel_qd<1>, dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (qd *)pool);
    else
        hipLaunchKernelGGL(tor::expand_kernel_qd<0>, dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (qd *)pool);
    return hipGetLastError();
}

hipError_t tor_launch_reduce_qd(const ReduceJobQ *jobs, int njobs, long long total_blocks, hipStream_t st) {
    const long long g = total_blocks < (1LL << 20) ? total_blocks : (1LL << 20);
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::reduce_kernel_qd, dim3((unsigned)g), dim3(256), 0, st, jobs, njobs, total_blocks);
    return hipGetLastError();
}

hipError_t tor_launch_condition_qd(const CondJobQ *jobs, int njobs, long long total_blocks, hipStream_t st) {
    if (njobs < 1 || total_blocks < 1) return hipSuccess;
    if (total_blocks > (1LL << 31) - 1) return hipErrorInvalidValue;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::condition_cols_qd, dim3((unsigned)njobs), dim3(256), 0, st, jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tor::condition_update_qd, dim3((unsigned)total_blocks), dim3(256), 0, st, jobs, njobs);
    return hipGetLastError();
}
