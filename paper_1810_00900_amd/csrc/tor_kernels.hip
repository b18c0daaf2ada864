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
//   expand  (HBM)   top levels, one workgroup per node, children written to a
//                   pool in HBM (breadth-first, one launch per level);
//   wave    (LDS)   a 64-lane workgroup takes one node with J modes and expands
//                   J - TL more levels breadth-first in LDS (64 leaves);
//   leaf    (VGPR)  each lane finishes a TL-mode node depth-first in registers.
// Scalars S are binary64 ("f64 tier") or double-double ("dd tier"); T, A and the
// path coefficients are always accumulated in double-double.  Reductions are in
// a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor_kernels.h"

#pragma clang fp contract(off)

namespace tor {

__host__ __device__ constexpr int E(int r) { return r * (2 * r + 1); }
__host__ __device__ constexpr int pidx(int a, int b) { return a * (a + 1) / 2 + b; }

// packed lower-triangle index -> (row, column)
__device__ __forceinline__ void unpack(int e, int &a, int &b) {
    int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    if ((r + 1) * (r + 2) / 2 <= e) r++;
    if (r * (r + 1) / 2 > e) r--;
    a = r;
    b = e - r * (r + 1) / 2;
}

template <class S> __device__ __forceinline__ S szero();
template <> __device__ __forceinline__ double szero<double>() { return 0.0; }
template <> __device__ __forceinline__ dd szero<dd>() { return dd_make(0.0, 0.0); }

__device__ __forceinline__ double sub_mul(double x, double a, double b) { return fma(-a, b, x); }
__device__ __forceinline__ dd sub_mul(dd x, dd a, dd b) { return dd_sub(x, dd_mul(a, b)); }

// Pivot quantities of the last mode of an r-mode node:
//   alpha = M[p0,p0], beta = M[p1,p0], gamma = M[p1,p1]
//   s1 = alpha^-1/2, l = beta/alpha, D2 = gamma - l beta, s2 = D2^-1/2,
//   q = s1 s2 = det(pivot)^-1/2.
// With v1(c) = M[p0,c] s1 and v2(c) = (M[p1,c] - l M[p0,c]) s2 the Schur
// complement is M[a,b] - v1(a) v1(b) - v2(a) v2(b).
template <class S> struct Pivot {
    S s1, l, s2, q;
};

template <class S>
__device__ __forceinline__ Pivot<S> make_pivot(S al, S be, S ga) {
    Pivot<S> p;
    p.s1 = rsqrt_s(al);
    p.l = mul_s(be, mul_s(p.s1, p.s1));
    S d2 = sub_mul(ga, p.l, be);
    p.s2 = rsqrt_s(d2);
    p.q = mul_s(p.s1, p.s2);
    return p;
}

__device__ __forceinline__ dd coef_mul(dd c, double q) { return dd_mul_d(c, q); }
__device__ __forceinline__ dd coef_mul(dd c, dd q) { return dd_mul(c, q); }

// ---------------------------------------------------------------- leaf tier

template <class S, int R> struct Leaf {
    static __device__ __forceinline__ void run(const S *M, dd &T, double &A) {
        constexpr int p0 = 2 * R - 2, p1 = 2 * R - 1, RC = 2 * R - 2;
        dd T0;
        double A0;
        Leaf<S, R - 1>::run(M, T0, A0);  // exclude: the prefix of M
        Pivot<S> pv = make_pivot(M[pidx(p0, p0)], M[pidx(p1, p0)], M[pidx(p1, p1)]);
        S v1[RC], v2[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            S m0 = M[pidx(p0, c)];
            v1[c] = mul_s(m0, pv.s1);
            v2[c] = mul_s(sub_mul(M[pidx(p1, c)], pv.l, m0), pv.s2);
        }
        S C[E(R - 1)];
#pragma unroll
        for (int a = 0; a < RC; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b)
                C[pidx(a, b)] = sub_dot2(M[pidx(a, b)], v1[a], v1[b], v2[a], v2[b]);
        dd T1;
        double A1;
        Leaf<S, R - 1>::run(C, T1, A1);
        T = dd_sub_mul(T0, pv.q, T1);
        A = A0 + hi_of(pv.q) * A1;
    }
};

template <class S> struct Leaf<S, 1> {
    static __device__ __forceinline__ void run(const S *M, dd &T, double &A) {
        S q = rsqrt_s(det2(M[0], M[1], M[2]));
        T = dd_sub(dd_from(1.0), to_dd(q));
        A = 1.0 + hi_of(q);
    }
};

template <class S> struct Leaf<S, 0> {
    static __device__ __forceinline__ void run(const S *, dd &T, double &A) {
        T = dd_from(1.0);
        A = 1.0;
    }
};

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double shfl_xor_d(double x, int m) { return __shfl_xor(x, m, 64); }

// fixed butterfly over the 64 lanes; every lane ends with the same value
__device__ __forceinline__ void wave_reduce(dd &T, double &A) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        dd o = dd_make(shfl_xor_d(T.hi, m), shfl_xor_d(T.lo, m));
        double oa = shfl_xor_d(A, m);
        // order the operands by lane so both partners compute the same sum
        bool low = (threadIdx.x & m) == 0;
        T = low ? dd_add(T, o) : dd_add(o, T);
        A = low ? A + oa : oa + A;
    }
}

// ---------------------------------------------------------------- wave tier

template <class S, int J> struct WaveCfg {
    static constexpr int TL = J < 3 ? J : 3;
    static constexpr int TW = J - TL;
    static constexpr int NL = 1 << TW;  // leaves (<= 64)
    // LDS slot offsets: slot base for include children created at level k
    static constexpr int soff(int k) {
        int o = E(J);
        for (int kk = 0; kk < k; ++kk) o += (1 << kk) * E(J - kk - 1);
        return o;
    }
    static constexpr int MAT = soff(TW);
    static constexpr int vmax() {
        int m = 1;
        for (int k = 0; k < TW; ++k) {
            int v = (1 << k) * 2 * (2 * (J - k) - 2);
            if (v > m) m = v;
        }
        return m;
    }
    static constexpr int VMAX = vmax();
    static constexpr int NPIV = NL / 2 > 0 ? NL / 2 : 1;
};

template <class S, int J, int K> struct WaveLevel {
    using C = WaveCfg<S, J>;
    static __device__ __forceinline__ void run(S *mat, S *vbuf, Pivot<S> *piv, int *loc, dd *coef,
                                               double *acoef, int lane) {
        if constexpr (K < C::TW) {
            constexpr int r = J - K, R = 2 * r, NK = 1 << K, RC = R - 2, EC = E(r - 1);
            // phase 0: pivot of each node, coefficients and slots of the include children
            if (lane < NK) {
                const S *base = mat + loc[lane];
                Pivot<S> pv = make_pivot(base[pidx(R - 2, R - 2)], base[pidx(R - 1, R - 2)],
                                         base[pidx(R - 1, R - 1)]);
                piv[lane] = pv;
                coef[NK + lane] = dd_neg(coef_mul(coef[lane], pv.q));
                acoef[NK + lane] = acoef[lane] * hi_of(pv.q);
                loc[NK + lane] = C::soff(K) + lane * EC;
            }
            __syncthreads();
            // phase 1: the two scaled pivot columns of every node
            for (int it = lane; it < NK * RC; it += 64) {
                int i = it / RC, c = it - i * RC;
                const S *base = mat + loc[i];
                Pivot<S> pv = piv[i];
                S m0 = base[pidx(R - 2, c)];
                vbuf[i * 2 * RC + c] = mul_s(m0, pv.s1);
                vbuf[i * 2 * RC + RC + c] = mul_s(sub_mul(base[pidx(R - 1, c)], pv.l, m0), pv.s2);
            }
            __syncthreads();
            // phase 2: rank-2 updates into the include children's slots
            for (int it = lane; it < NK * EC; it += 64) {
                int i = it / EC, e = it - i * EC;
                int a, b;
                unpack(e, a, b);
                const S *base = mat + loc[i];
                const S *v = vbuf + i * 2 * RC;
                mat[C::soff(K) + i * EC + e] = sub_dot2(base[e], v[a], v[b], v[RC + a], v[RC + b]);
            }
            __syncthreads();
            WaveLevel<S, J, K + 1>::run(mat, vbuf, piv, loc, coef, acoef, lane);
        }
    }
};

// index of the last job whose begin <= t (jobs sorted by begin, jobs[0].begin == 0)
template <class Job>
__device__ __forceinline__ int find_job(const Job *jobs, int njobs, long long t) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class S, int J>
__global__ __launch_bounds__(64) void wave_kernel(const WaveJob *__restrict__ jobs, int njobs, long long total,
                                                  const S *__restrict__ pool) {
    using C = WaveCfg<S, J>;
    __shared__ S mat[C::MAT];
    __shared__ S vbuf[C::VMAX];
    __shared__ Pivot<S> piv[C::NPIV];
    __shared__ int loc[C::NL];
    __shared__ dd coef[C::NL];
    __shared__ double acoef[C::NL];
    const int lane = threadIdx.x;
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int j = find_job(jobs, njobs, t);
        const long long lt = t - jobs[j].begin;
        NodeDesc d = jobs[j].tasks[lt];
        const S *root = pool + d.off;
        for (int e = lane; e < E(J); e += 64) mat[e] = root[e];
        if (lane == 0) {
            loc[0] = 0;
            coef[0] = dd_make(d.coef_hi, d.coef_lo);
            acoef[0] = d.acoef;
        }
        __syncthreads();
        WaveLevel<S, J, 0>::run(mat, vbuf, piv, loc, coef, acoef, lane);
        dd T = dd_from(0.0);
        double A = 0.0;
        if (lane < C::NL) {
            S M[E(C::TL)];
            const S *base = mat + loc[lane];
#pragma unroll
            for (int e = 0; e < E(C::TL); ++e) M[e] = base[e];
            dd Tl;
            double Al;
            Leaf<S, C::TL>::run(M, Tl, Al);
            T = dd_mul(coef[lane], Tl);
            A = acoef[lane] * Al;
        }
        wave_reduce(T, A);
        if (lane == 0) {
            Partial p;
            p.t_hi = T.hi;
            p.t_lo = T.lo;
            p.a = A;
            p.pad = 0.0;
            jobs[j].out[lt] = p;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- HBM tier

template <class S>
__global__ __launch_bounds__(256) void expand_kernel(const ExpandJob *__restrict__ jobs, int log2npar,
                                                     long long total, S *__restrict__ pool) {
    __shared__ S v[2][2 * TOR_MAX_N];
    for (long long f = blockIdx.x; f < total; f += gridDim.x) {
        const ExpandJob job = jobs[f >> log2npar];
        const long long i = f & ((1LL << log2npar) - 1);
        const int r = job.r, R = 2 * r, RC = R - 2, EC = E(r - 1);
        NodeDesc d = job.par[i];
        const S *base = pool + d.off;
        Pivot<S> pv = make_pivot(base[pidx(R - 2, R - 2)], base[pidx(R - 1, R - 2)], base[pidx(R - 1, R - 1)]);
        unsigned long long coff = job.child_base + (unsigned long long)i * (unsigned long long)EC;
        if (threadIdx.x == 0) {
            job.chi[2 * i] = d;
            NodeDesc c;
            c.off = coff;
            dd cf = dd_neg(coef_mul(dd_make(d.coef_hi, d.coef_lo), pv.q));
            c.coef_hi = cf.hi;
            c.coef_lo = cf.lo;
            c.acoef = d.acoef * hi_of(pv.q);
            job.chi[2 * i + 1] = c;
        }
        for (int c = threadIdx.x; c < RC; c += blockDim.x) {
            S m0 = base[pidx(R - 2, c)];
            v[0][c] = mul_s(m0, pv.s1);
            v[1][c] = mul_s(sub_mul(base[pidx(R - 1, c)], pv.l, m0), pv.s2);
        }
        __syncthreads();
        S *outp = pool + coff;
        for (int e = threadIdx.x; e < EC; e += blockDim.x) {
            int a, b;
            unpack(e, a, b);
            outp[e] = sub_dot2(base[e], v[0][a], v[0][b], v[1][a], v[1][b]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- reduction

// One reduction stage: block b of a job sums in[b*chunk, min((b+1)*chunk, count))
// in a fixed order (thread-strided sequential sums, then a fixed LDS tree).
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceJob *__restrict__ jobs, int njobs,
                                                     long long total_blocks) {
    __shared__ dd sT[256];
    __shared__ double sA[256];
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

template <class S, int J>
static hipError_t launch_wave_J(const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                                hipStream_t st) {
    long long g = total < grid_cap ? total : grid_cap;
    if (g < 1) return hipSuccess;
    hipLaunchKernelGGL((wave_kernel<S, J>), dim3((unsigned)g), dim3(64), 0, st, jobs, njobs, total,
                       (const S *)pool);
    return hipGetLastError();
}

template <class S>
static hipError_t launch_wave_S(int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                                int grid_cap, hipStream_t st) {
    switch (J) {
    case 1: return launch_wave_J<S, 1>(jobs, njobs, total, pool, grid_cap, st);
    case 2: return launch_wave_J<S, 2>(jobs, njobs, total, pool, grid_cap, st);
    case 3: return launch_wave_J<S, 3>(jobs, njobs, total, pool, grid_cap, st);
    case 4: return launch_wave_J<S, 4>(jobs, njobs, total, pool, grid_cap, st);
    case 5: return launch_wave_J<S, 5>(jobs, njobs, total, pool, grid_cap, st);
    case 6: return launch_wave_J<S, 6>(jobs, njobs, total, pool, grid_cap, st);
    case 7: return launch_wave_J<S, 7>(jobs, njobs, total, pool, grid_cap, st);
    case 8: return launch_wave_J<S, 8>(jobs, njobs, total, pool, grid_cap, st);
    case 9: return launch_wave_J<S, 9>(jobs, njobs, total, pool, grid_cap, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tor

hipError_t tor_launch_wave(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                           int grid_cap, hipStream_t st) {
    return is_dd ? tor::launch_wave_S<dd>(J, jobs, njobs, total, pool, grid_cap, st)
                 : tor::launch_wave_S<double>(J, jobs, njobs, total, pool, grid_cap, st);
}

hipError_t tor_launch_expand(int is_dd, const ExpandJob *jobs, int njobs, int log2npar, void *pool, int grid_cap,
                             hipStream_t st) {
    long long total = (long long)njobs << log2npar;
    long long g = total < grid_cap ? total : grid_cap;
    if (g < 1) return hipSuccess;
    if (is_dd)
        hipLaunchKernelGGL(tor::expand_kernel<dd>, dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (dd *)pool);
    else
        hipLaunchKernelGGL(tor::expand_kernel<double>, dim3((unsigned)g), dim3(256), 0, st, jobs, log2npar, total,
                           (double *)pool);
    return hipGetLastError();
}

hipError_t tor_launch_reduce(const ReduceJob *jobs, int njobs, long long total_blocks, hipStream_t st) {
    long long g = total_blocks < (1LL << 20) ? total_blocks : (1LL << 20);
    if (g < 1) return hipSuccess;
    hipLaunchKernelGGL(tor::reduce_kernel, dim3((unsigned)g), dim3(256), 0, st, jobs, njobs, total_blocks);
    return hipGetLastError();
}

hipError_t tor_launch_gather(const Partial *const *src, int n, Partial *dst, hipStream_t st) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(tor::gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n, dst);
    return hipGetLastError();
}
