// GPU kernels for the signed subset sum of threshold-detector GBS.
//
// Given an SPD matrix Sigma (2n x 2n; modes are 2x2 blocks) the kernels compute
//
//     T = sum_{Y subset of [n]} (-1)^{|Y|} det(Sigma[Y])^{-1/2},
//     A = sum_{Y subset of [n]}            det(Sigma[Y])^{-1/2},
//
// which is the click probability of Sec. II of arXiv:1810.00900 (the click POVM
// as a difference of Gaussian operators, summed by linearity) after the no-click
// modes have been conditioned away (Eq. MatrixUpdate).  A is the sum of the
// magnitudes of the terms; A / |T| is the cancellation ratio.
//
// The subsets are enumerated as a binary tree over the modes, deciding the last
// mode first (the paper also measures mode l first).  At a node with matrix M
// (r modes) the "exclude" child is the leading principal block of M (no work:
// in packed row-major lower storage it is a prefix of M) and the "include" child
// is the Schur complement of the last mode's 2x2 pivot block, i.e. the paper's
// vacuum-conditioning update Eq. MatrixUpdate, with factor
// q = det(pivot)^{-1/2} (the q_k of Eq. (prob) at zero mean).  Then
//     T(M) = T(exclude) - q * T(include),   A(M) = A(exclude) + q * A(include).
// Every term det(Sigma[Y])^{-1/2} is the product of the q's along its path (a
// block Cholesky factorisation of Sigma[Y] shared with every subset that has
// the same prefix).
//
// Three tiers:
//   expand  (HBM)   top levels, one 64-lane wave per node (up to 16 while a
//                   level has few nodes), children written to a pool in HBM
//                   (breadth-first, one launch per level);
//   wave    (LDS)   a 64-lane workgroup takes one node with J modes and expands
//                   J - TL more levels breadth-first in LDS (64 leaves);
//   leaf    (VGPR)  each lane finishes a TL-mode node depth-first in registers.
// Scalars S are binary64 ("f64 tier") or double-double ("dd tier"); T, A and the
// path coefficients are always accumulated in double-double.  Reductions are in
// a fixed order, so results are bitwise reproducible.  This file holds the
// zero-mean wave kernels, the expansion, conditioning and reduction kernels;
// the displaced-state wave kernels are in tor_kernels_disp.hip and the
// quad-double tier in tor_kernels_qd.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor_kernels.h"
#include "tor_tree.hpp"
#include "tor_wave.hpp"

#pragma clang fp contract(off)

namespace tor {

// ---------------------------------------------------------------- HBM tier


// One wave per parent node (four per 256-thread workgroup): the include child
// (rank-2 Schur update of the last mode) goes to the pool, the exclude child
// keeps the parent's offset.  Waves run independently (no workgroup barrier).
// D = 1: displaced state (mean row first in every packed matrix); D = -1: the
// information form (the first row holds sigma_Q^-1 mu; see make_pivot_m).
// The pivot columns and the first kExpandPre entries of each lane are loaded
// before the pivot is formed, so that one HBM round trip serves all three
// (the child region never overlaps a parent's).  On the top levels, where
// there are few nodes, 2^log2split waves share a node: each forms the pivot
// and the columns and writes every 2^log2split-th 64-entry chunk of the child.
constexpr int kExpandPre = 4;
template <class S, int D>
__global__ __launch_bounds__(256) void expand_kernel(const ExpandJob *__restrict__ jobs, int log2npar,
                                                     long long total, S *__restrict__ pool,
                                                     const LaunchDims *__restrict__ dyn, int log2split) {
    if (dyn) total = dyn->njobs << log2npar;
    __shared__ S vs[4][2][2 * TOR_MAX_N + MR(D)];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    S *v0 = vs[w][0], *v1 = vs[w][1];
    const int nsplit = 1 << log2split;
    const long long work = total << log2split;
    for (long long g = (long long)blockIdx.x * 4 + w; g < work; g += (long long)gridDim.x * 4) {
        const long long f = g >> log2split;
        const int first = lane + 64 * (int)(g & (nsplit - 1));  // this wave's first entry
        const ExpandJob job = jobs[f >> log2npar];
        const long long i = f & ((1LL << log2npar) - 1);
        const int r = job.r, R = 2 * r + MR(D), RC = R - 2, EC = EN(r - 1, MR(D));
        NodeDesc d = job.par[i];
        const S *base = pool + d.off;
        S pre[kExpandPre], c0 = S(), c1 = S();
#pragma unroll
        for (int k = 0; k < kExpandPre; k++)
            if (first + 64 * nsplit * k < EC) pre[k] = base[first + 64 * nsplit * k];
        if (lane < RC) {  // RC <= 2 * TOR_MAX_N - 1 < 64
            c0 = base[pidx(R - 2, lane)];
            c1 = base[pidx(R - 1, lane)];
        }
        Pivot<S> pv = make_pivot_m<S, D>(base, R - 2, R - 1);
        unsigned long long coff = job.child_base + (unsigned long long)i * (unsigned long long)EC;
        if (first == 0) {
            job.chi[2 * i] = d;
            NodeDesc c;
            c.off = coff;
            dd cf = dd_neg(coef_mul(dd_make(d.coef_hi, d.coef_lo), pv.q));
            c.coef_hi = cf.hi;
            c.coef_lo = cf.lo;
            c.acoef = d.acoef * hi_of(pv.q);
            job.chi[2 * i + 1] = c;
        }
        if (lane < RC) {
            v0[lane] = mul_s(c0, pv.s1);
            v1[lane] = mul_s(sub_mul(c1, pv.l, c0), pv.s2);
        }
        wave_sync();
        S *outp = pool + coff;
#pragma unroll
        for (int k = 0; k < kExpandPre; k++) {
            const int e = first + 64 * nsplit * k;
            if (e < EC) {
                int a, b;
                unpack(e, a, b);
                outp[e] = sub_dot2(pre[k], v0[a], v0[b], v1[a], v1[b]);
            }
        }
        for (int e = first + 64 * nsplit * kExpandPre; e < EC; e += 64 * nsplit) {
            int a, b;
            unpack(e, a, b);
            outp[e] = sub_dot2(base[e], v0[a], v0[b], v1[a], v1[b]);
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------- no-click conditioning

// One step of the vacuum conditioning (Eq. MatrixUpdate) for every query of
// the launch: the last mode of the query's matrix (packed lower, r modes, the
// no-click modes last) is conditioned on vacuum -- the Schur complement of its
// 2x2 pivot block replaces the leading block in place, the include-child
// update of the subset tree -- and the query's vacuum probability is
// multiplied by q = det(pivot)^-1/2.  Each 256-thread block takes
// TOR_COND_CHUNK entries of one query; it forms the pivot and the scaled pivot
// columns its entries need in LDS (the last two rows, which the step does not
// write).  Blocks of one step write disjoint entries.  A displaced query
// (job.d = 1) carries its mean as row 0: the same update conditions the mean,
// and q gains the overlap factor of the pivot mode's mean.
__global__ __launch_bounds__(256) void condition_kernel(const CondJob *__restrict__ jobs, int njobs) {
    extern __shared__ dd cols[];
    const int j = find_job(jobs, njobs, (long long)blockIdx.x);
    const CondJob job = jobs[j];
    const long long blk = (long long)blockIdx.x - job.begin;
    const int r = job.r, R = 2 * r + job.d, RC = R - 2;
    dd *M = job.mat;
    const Pivot<dd> pv = job.d ? make_pivot_m<dd, 1>(M, R - 2, R - 1) : make_pivot_m<dd, 0>(M, R - 2, R - 1);
    const int EC = job.d ? EN(r - 1, 1) : EN(r - 1, 0);
    const int e0 = (int)(blk * TOR_COND_CHUNK);
    const int e1 = e0 + TOR_COND_CHUNK < EC ? e0 + TOR_COND_CHUNK : EC;
    int amax = -1, bl;  // largest row among this block's entries (none when r = 1)
    if (e1 > e0) unpack(e1 - 1, amax, bl);
    for (int c = threadIdx.x; c <= amax; c += blockDim.x) {
        const dd m0 = M[pidx(R - 2, c)];
        cols[c] = dd_mul(m0, pv.s1);
        cols[RC + c] = dd_mul(sub_mul(M[pidx(R - 1, c)], pv.l, m0), pv.s2);
    }
    __syncthreads();
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        int a, b;
        unpack(e, a, b);
        M[e] = dd_sub_dot2(M[e], cols[a], cols[b], cols[RC + a], cols[RC + b]);
    }
    if (blk == 0 && threadIdx.x == 0) {
        const dd p = dd_mul(dd_make(job.acc[0], job.acc[1]), pv.q);
        job.acc[0] = p.hi;
        job.acc[1] = p.lo;
        job.acc[2] += log(pv.q.hi) + log1p(pv.q.lo / pv.q.hi);
        if (job.qout) {
            job.qout[0] = pv.q.hi;
            job.qout[1] = pv.q.lo;
        }
    }
}

// ---------------------------------------------------------------- blocked conditioning

template <class F>
__device__ __forceinline__ int find_cond_job(const CondBlockJob *jobs, int njobs, long long t, F begin) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (begin(jobs[mid]) <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Panel of one block of b modes of a query (rows Rb .. R - 1, Rb = R - 2b).
// Every workgroup of the job walks the block's b steps on the 2b x 2b pivot
// block (and the mean column of a displaced query) in LDS, exactly as the
// per-mode kernel conditions those entries, keeping each step's pivot and the
// scaled pivot columns of the block's own rows; then each thread takes one
// column x < Rb: its 2b panel entries in registers, the b steps applied in
// order, each step's two scaled pivot columns at x written to V.  Rows are
// counted from the end (k = R - 1 - row), so a step's pivot rows are
// k = 2t, 2t + 1 and the rows it updates k > 2t + 1.
template <int D>
__device__ __forceinline__ void cond_panel(const CondBlockJob &job, long long wg) {
    constexpr int B = TOR_COND_BLOCK, NB = 2 * B;
    __shared__ dd blk[NB * (NB + 1) / 2];  // pivot block, packed by reversed row index
    __shared__ dd mc[NB];                  // mean column (D = 1)
    __shared__ Pivot<dd> piv[B];
    __shared__ dd vd[B][2][NB];            // scaled pivot columns at the block's rows
    const int b = job.b, nb = 2 * b, R = 2 * job.r + D, Rb = R - nb;
    dd *M = job.mat;
    const int tid = threadIdx.x;
    // the block's steps, every thread of the workgroup taking a share of each
    // step's entries (two workgroup barriers per step)
    constexpr int NT = 256;  // threads per workgroup (the launch's block size)
    __shared__ unsigned short lk[NB * (NB + 1) / 2];  // packed index -> (l, k) of the block
    for (int e = tid; e < NB * (NB + 1) / 2; e += NT) {
        int l, k;
        unpack(e, l, k);
        lk[e] = (unsigned short)(l | (k << 8));
    }
    // entry (k, l) of the block (rows R - 1 - k, R - 1 - l, k <= l) at pidx(l, k)
    for (int e = tid; e < nb * (nb + 1) / 2; e += NT) {
        int l, k;
        unpack(e, l, k);
        blk[e] = M[pidx(R - 1 - k, R - 1 - l)];
    }
    if (D)
        for (int k = tid; k < nb; k += NT) mc[k] = M[pidx(R - 1 - k, 0)];
    __syncthreads();
    for (int t = 0; t < b; ++t) {
        const int k1 = 2 * t, k0 = 2 * t + 1;  // rows R_t - 1 and R_t - 2 of this step
        // block (k, l) with k <= l is row R - 1 - k, column R - 1 - l: the
        // entry (row p0, column p0) is blk[pidx(k0, k0)], (p1, p0) is
        // blk[pidx(k0, k1)] (row k1 = p1 > column k0 = p0 means k1 < k0)
        const Pivot<dd> pv = make_pivot_v<dd, D>(blk[pidx(k0, k0)], blk[pidx(k0, k1)], blk[pidx(k1, k1)],
                                                 D ? mc[k0] : blk[0], D ? mc[k1] : blk[0]);
        for (int k = k0 + 1 + tid; k < nb; k += NT) {  // column c = R - 1 - k < p0
            const dd m0 = blk[pidx(k, k0)];
            vd[t][0][k] = dd_mul(m0, pv.s1);
            vd[t][1][k] = dd_mul(sub_mul(blk[pidx(k, k1)], pv.l, m0), pv.s2);
        }
        if (tid == 0) piv[t] = pv;
        __syncthreads();
        // the block's remaining entries and mean column, as the per-mode
        // update: all loads of a thread's (at most 3) entries first
        const int rem = nb - (k0 + 1), nrem = rem * (rem + 1) / 2;
        constexpr int PER = (NB * (NB + 1) / 2 + NT - 1) / NT;
        dd xe[PER], a1[PER], b1[PER], a2[PER], b2[PER];
        int dst[PER];
        // (past the last entry a thread reads entry 0, (k0 + 1, k0 + 1), and
        // stores nothing; there is none in the last step)
#pragma unroll
        for (int u = 0; u < PER && nrem > 0; ++u) {
            const int e = tid + NT * u;
            const bool ok = e < nrem;
            const unsigned short w = lk[ok ? e : 0];
            const int l = (w & 0xff) + k0 + 1, k = (w >> 8) + k0 + 1;  // k <= l
            dst[u] = ok ? pidx(l, k) : -1;
            xe[u] = blk[pidx(l, k)];
            a1[u] = vd[t][0][k];
            b1[u] = vd[t][0][l];
            a2[u] = vd[t][1][k];
            b2[u] = vd[t][1][l];
        }
        // (each entry is read and written by its own thread only)
#pragma unroll
        for (int u = 0; u < PER && nrem > 0; ++u) {
            const dd y = dd_sub_dot2(xe[u], a1[u], b1[u], a2[u], b2[u]);
            if (dst[u] >= 0) blk[dst[u]] = y;
        }
        if (D) {
            const dd w1 = dd_mul(mc[k0], pv.s1), w2 = dd_mul(sub_mul(mc[k1], pv.l, mc[k0]), pv.s2);
            for (int k = k0 + 1 + tid; k < nb; k += NT)
                mc[k] = dd_sub_dot2(mc[k], vd[t][0][k], w1, vd[t][1][k], w2);
        }
        __syncthreads();
    }
    if (wg == 0 && tid == 0)  // the per-mode kernel's accumulation, in step order
        for (int t = 0; t < b; ++t) {
            const dd q = piv[t].q;
            const dd p = dd_mul(dd_make(job.acc[0], job.acc[1]), q);
            job.acc[0] = p.hi;
            job.acc[1] = p.lo;
            job.acc[2] += log(q.hi) + log1p(q.lo / q.hi);
        }
    __syncthreads();
    // column x of the rest, TOR_COND_TPC threads per column: thread s of a
    // column holds its panel entries k = PE s .. PE s + PE - 1 (rows
    // R - 1 - k) in registers.  At step t the holder of the step's pivot rows
    // (2t, 2t + 1) forms the two scaled pivot columns at x, writes them to V
    // and passes them to the column's other threads (lane shuffles); every
    // thread then applies the step to its entries below the pivot rows.  Each
    // entry takes the same operations in the same order as with one thread
    // per column.
    constexpr int TPC = TOR_COND_TPC, PE = NB / TPC;
    static_assert(NB % TPC == 0 && PE % 2 == 0, "a step's two pivot rows lie in one thread's entries");
    const int s = tid % TPC, lane = tid & 63;
    for (int pass = 0; pass < job.passes; ++pass) {  // column groups of this workgroup
        const long long x = (wg * job.passes + pass) * (blockDim.x / TPC) + tid / TPC;
        const bool live = x < Rb;
        dd P[PE];
#pragma unroll
        for (int i = 0; i < PE; ++i) {
            const int k = PE * s + i;
            P[i] = live && k < nb ? M[pidx(R - 1 - k, (int)x)] : dd_from(0.0);
        }
#pragma unroll
        for (int t = 0; t < B; ++t) {
            if (t < b) {
                const Pivot<dd> pv = piv[t];
                const int holder = (2 * t) / PE, i0 = (2 * t) % PE;
                dd v1 = dd_from(0.0), v2 = dd_from(0.0);
                if (s == holder) {
                    const dd m0 = P[i0 + 1];
                    v1 = dd_mul(m0, pv.s1);
                    v2 = dd_mul(sub_mul(P[i0], pv.l, m0), pv.s2);
                    if (live) {
                        job.V[(long long)(2 * t) * job.ld + x] = v1;
                        job.V[(long long)(2 * t + 1) * job.ld + x] = v2;
                    }
                }
                const int src = (lane & ~(TPC - 1)) | holder;
                v1.hi = __shfl(v1.hi, src);
                v1.lo = __shfl(v1.lo, src);
                v2.hi = __shfl(v2.hi, src);
                v2.lo = __shfl(v2.lo, src);
#pragma unroll
                for (int i = 0; i < PE; ++i) {
                    const int k = PE * s + i;
                    if (k >= 2 * t + 2 && k < nb) P[i] = dd_sub_dot2(P[i], vd[t][0][k], v1, vd[t][1][k], v2);
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void cond_panel_kernel(const CondBlockJob *__restrict__ jobs, int njobs) {
    const int j = find_cond_job(jobs, njobs, (long long)blockIdx.x,
                                [](const CondBlockJob &q) { return q.begin_panel; });
    const CondBlockJob job = jobs[j];
    const long long wg = (long long)blockIdx.x - job.begin_panel;
    if (job.d) cond_panel<1>(job, wg);
    else cond_panel<0>(job, wg);
}

// The rest of the matrix (rows and columns below Rb) in 32 x 32 tiles of the
// lower triangle: each entry takes the block's b rank-2 updates in step order
// from the recorded columns (staged in LDS for the tile's rows and columns).
__global__ __launch_bounds__(256) void cond_bulk_kernel(const CondBlockJob *__restrict__ jobs, int njobs) {
    constexpr int B = TOR_COND_BLOCK;
    __shared__ dd Vr[B][2][32], Vc[B][2][32];
    const int j = find_cond_job(jobs, njobs, (long long)blockIdx.x,
                                [](const CondBlockJob &q) { return q.begin_bulk; });
    const CondBlockJob job = jobs[j];
    const long long tt = (long long)blockIdx.x - job.begin_bulk;
    const int b = job.b, Rb = 2 * (job.r - b) + job.d;
    // tile (I, J), J <= I, numbered row by row
    long long I = (long long)((sqrt(8.0 * (double)tt + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > tt) --I;
    while ((I + 1) * (I + 2) / 2 <= tt) ++I;
    const long long J = tt - I * (I + 1) / 2;
    const int a0 = (int)(32 * I), c0 = (int)(32 * J);
    for (int idx = threadIdx.x; idx < b * 64; idx += blockDim.x) {
        const int t = idx >> 6, w = (idx >> 5) & 1, l = idx & 31;
        const dd *v = job.V + (long long)(2 * t + w) * job.ld;
        Vr[t][w][l] = a0 + l < Rb ? v[a0 + l] : dd_from(0.0);
        Vc[t][w][l] = c0 + l < Rb ? v[c0 + l] : dd_from(0.0);
    }
    __syncthreads();
    dd *M = job.mat;
    // a thread's four entries share their column: the column's two values
    // of a step are read once for all four, whose update chains interleave
    // (each entry still takes the b updates in step order)
    const int cl = threadIdx.x & 31, c = c0 + cl;
    dd xq[4];
    long long eq[4];
    bool okq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int a = a0 + (threadIdx.x >> 5) + 8 * q;
        okq[q] = a < Rb && c <= a;
        eq[q] = (long long)a * (a + 1) / 2 + c;
        xq[q] = okq[q] ? M[eq[q]] : dd_from(0.0);
    }
    for (int t = 0; t < b; ++t) {
        const dd c1 = Vc[t][0][cl], c2 = Vc[t][1][cl];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int al = (threadIdx.x >> 5) + 8 * q;
            xq[q] = dd_sub_dot2(xq[q], Vr[t][0][al], c1, Vr[t][1][al], c2);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (okq[q]) M[eq[q]] = xq[q];
}

// ---------------------------------------------------------------- reduction

// One reduction stage: block b of a job sums in[b*chunk, min((b+1)*chunk, count))
// in a fixed order (thread-strided sequential sums, then a fixed LDS tree).
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceJob *__restrict__ jobs, int njobs,
                                                     long long total_blocks, const LaunchDims *__restrict__ dyn) {
    __shared__ dd sT[256];
    __shared__ double sA[256];
    if (dyn) {
        njobs = (int)dyn->njobs;
        total_blocks = dyn->total;
    }
    for (long long gb = blockIdx.x; gb < total_blocks; gb += gridDim.x) {
        int lo_j = 0, hi_j = njobs - 1;
        while (lo_j < hi_j) {
            int mid = (lo_j + hi_j + 1) >> 1;
            if (jobs[mid].block_begin <= gb) lo_j = mid;
            else hi_j = mid - 1;
        }
        const ReduceJob job = jobs[lo_j];
        const long long b = gb - job.block_begin;
        long long lo = b * TOR_REDUCE_CHUNK;
        long long hi = lo + TOR_REDUCE_CHUNK < job.count ? lo + TOR_REDUCE_CHUNK : job.count;
        dd T = dd_from(0.0);
        double A = 0.0;
        for (long long k = lo + threadIdx.x; k < hi; k += blockDim.x) {
            Partial p = job.in[k];
            T = dd_add(T, dd_make(p.t_hi, p.t_lo));
            A += p.a;
        }
        sT[threadIdx.x] = T;
        sA[threadIdx.x] = A;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                sT[threadIdx.x] = dd_add(sT[threadIdx.x], sT[threadIdx.x + s]);
                sA[threadIdx.x] = sA[threadIdx.x] + sA[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            Partial p;
            p.t_hi = sT[0].hi;
            p.t_lo = sT[0].lo;
            p.a = sA[0];
            p.pad = 0.0;
            job.out[b] = p;
        }
        __syncthreads();
    }
}

__global__ void gather_kernel(const Partial *const *__restrict__ src, int n, Partial *__restrict__ dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = *src[i];
}

// ---------------------------------------------------------------- launchers

}  // namespace tor

hipError_t tor_launch_wave(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                           int grid_cap, hipStream_t st, const LaunchDims *dyn, int disp) {
    if (disp < 0) return tor_launch_wave_info(is_dd, J, jobs, njobs, total, pool, grid_cap, st, dyn);
    if (disp) return tor_launch_wave_disp(is_dd, J, jobs, njobs, total, pool, grid_cap, st, dyn);
    return is_dd ? tor::launch_wave_S<dd, 0>(J, jobs, njobs, total, pool, grid_cap, st, dyn)
                 : tor::launch_wave_S<double, 0>(J, jobs, njobs, total, pool, grid_cap, st, dyn);
}

hipError_t tor_launch_expand(int is_dd, const ExpandJob *jobs, int njobs, int log2npar, void *pool, int grid_cap,
                             hipStream_t st, const LaunchDims *dyn, int disp) {
    long long total = (long long)njobs << log2npar;
    // few nodes (host-planned levels only): up to 16 waves per node
    int log2split = 0;
    while (!dyn && log2split < 4 && (total << log2split) < 8192) log2split++;
    long long blocks = ((total << log2split) + 3) / 4;
    long long g = dyn ? grid_cap : (blocks < grid_cap ? blocks : grid_cap);
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    if (is_dd && disp < 0)
        hipLaunchKernelGGL((tor::expand_kernel<dd, -1>), dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (dd *)pool, dyn, log2split);
    else if (!is_dd && disp < 0)
        hipLaunchKernelGGL((tor::expand_kernel<double, -1>), dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar,
                           total, (double *)pool, dyn, log2split);
    else if (is_dd && disp)
        hipLaunchKernelGGL((tor::expand_kernel<dd, 1>), dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (dd *)pool, dyn, log2split);
    else if (is_dd)
        hipLaunchKernelGGL((tor::expand_kernel<dd, 0>), dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (dd *)pool, dyn, log2split);
    else if (disp)
        hipLaunchKernelGGL((tor::expand_kernel<double, 1>), dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar,
                           total, (double *)pool, dyn, log2split);
    else
        hipLaunchKernelGGL((tor::expand_kernel<double, 0>), dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar,
                           total, (double *)pool, dyn, log2split);
    return hipGetLastError();
}

hipError_t tor_launch_reduce(const ReduceJob *jobs, int njobs, long long total_blocks, hipStream_t st,
                             const LaunchDims *dyn) {
    long long g = total_blocks < (1LL << 20) ? total_blocks : (1LL << 20);
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::reduce_kernel, dim3((unsigned)g), dim3(256), 0, st, jobs, njobs, total_blocks, dyn);
    return hipGetLastError();
}

hipError_t tor_launch_condition(const CondJob *jobs, int njobs, long long total_blocks, int rmax, hipStream_t st) {
    if (total_blocks < 1) return hipSuccess;
    if (rmax < 1 || rmax > TOR_COND_MAX_MODES || total_blocks > (1LL << 31) - 1) return hipErrorInvalidValue;
    const size_t lds = sizeof(dd) * 2 * (2 * (size_t)rmax - 1) + 16;  // 2 columns of 2 rmax - 1 rows (mean row)
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::condition_kernel, dim3((unsigned)total_blocks), dim3(256), lds, st, jobs, njobs);
    return hipGetLastError();
}

hipError_t tor_launch_cond_panel(const CondBlockJob *jobs, int njobs, long long total_blocks, hipStream_t st) {
    if (total_blocks < 1) return hipSuccess;
    if (total_blocks > (1LL << 31) - 1) return hipErrorInvalidValue;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::cond_panel_kernel, dim3((unsigned)total_blocks), dim3(256), 0, st, jobs, njobs);
    return hipGetLastError();
}

hipError_t tor_launch_cond_bulk(const CondBlockJob *jobs, int njobs, long long total_blocks, hipStream_t st) {
    if (total_blocks < 1) return hipSuccess;
    if (total_blocks > (1LL << 31) - 1) return hipErrorInvalidValue;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::cond_bulk_kernel, dim3((unsigned)total_blocks), dim3(256), 0, st, jobs, njobs);
    return hipGetLastError();
}

hipError_t tor_launch_gather(const Partial *const *src, int n, Partial *dst, hipStream_t st) {
    if (n < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n, dst);
    return hipGetLastError();
}
