// Per-state inverse of sigma_Q = sigma + I/2 on the GPU, for full patterns
// (every mode observed).  With K = sigma_Q^-1 and G = K[C] (the clicked
// modes' block), Jacobi's complementary-minor identity gives
// det(sigma_Q[S]) = det(sigma_Q) det(K[S^c]) for every set of modes S, so the
// vacuum probabilities of Eq. (prob) over S = Y + N, N the no-click modes, are
// det(sigma_Q)^-1/2 det(G[C \ Y])^-1/2 and
//   p(C, N) = (-1)^n det(sigma_Q)^-1/2 T(G),
// the subset sum of the gathered block G: the conditioning on N (Eq.
// MatrixUpdate iterated over N) is done once per state instead of once per
// query.
//
// The inverse is formed by symmetric sweeps, one per mode, each on the mode's
// 2x2 block P (the current Schur complement, positive definite):
//   A[i, j] <- A[i, j] - A[i, P] P^-1 A[P, j]    (i, j outside P)
//   A[i, P] <- A[i, P] P^-1,   P <- -P^-1
// written with the pivot quantities of the subset tree (P = L L^T, s1 =
// alpha^-1/2, l = beta / alpha, s2 = (gamma - l beta)^-1/2, v1 = A[i, p0] s1,
// v2 = (A[i, p1] - l A[i, p0]) s2): the first line is the tree's rank-2
// update A - v1 v1^T - v2 v2^T; A[i, P] P^-1 = (v1 s1 - v2 l s2, v2 s2); and
// -P^-1 = [[-(s1^2 + l^2 s2^2), l s2^2], [l s2^2, -s2^2]].  After all sweeps A
// holds -sigma_Q^-1 (negated in place at the end), and the product of the
// blocks' det^-1/2 is det(sigma_Q)^-1/2.  Two launches per mode: the pivot
// columns go to a scratch buffer first because the update rewrites them.
// sigma_Q is packed on the device from the state's device copy of sigma.
#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "qd.hpp"
#include "tor_invert.h"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

__device__ __forceinline__ dd acc_word(dd q) { return q; }
__device__ __forceinline__ dd acc_word(qd q) { return qd_to_dd(q); }

// packed index of the symmetric entry (i, j) in either order
__device__ __forceinline__ int sym_idx(int i, int j) { return i >= j ? pidx(i, j) : pidx(j, i); }

template <class S>
__global__ __launch_bounds__(256) void sweep_cols_kernel(const S *__restrict__ A, int d, int k, S *__restrict__ cols,
                                                         S *__restrict__ piv, double *__restrict__ acc) {
    const int p0 = 2 * k, p1 = 2 * k + 1;
    const Pivot<S> pv = make_pivot(A[pidx(p0, p0)], A[pidx(p1, p0)], A[pidx(p1, p1)]);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d) {
        if (i == p0 || i == p1) {
            cols[i] = from_pair<S>(0.0, 0.0);
            cols[d + i] = from_pair<S>(0.0, 0.0);
        } else {
            const S x = A[sym_idx(i, p0)];
            const S y = A[sym_idx(i, p1)];
            cols[i] = mul_s(x, pv.s1);
            cols[d + i] = mul_s(sub_mul(y, pv.l, x), pv.s2);
        }
    }
    if (i == 0) {
        piv[0] = pv.s1;
        piv[1] = pv.s2;
        piv[2] = mul_s(pv.l, pv.s2);
        const dd q = acc_word(pv.q);
        const dd p = dd_mul(dd_make(acc[0], acc[1]), q);
        acc[0] = p.hi;
        acc[1] = p.lo;
        acc[2] += log(q.hi) + log1p(q.lo / q.hi);
    }
}

template <class S>
__global__ __launch_bounds__(256) void sweep_update_kernel(S *__restrict__ A, int d, int k, int entries,
                                                           const S *__restrict__ cols, const S *__restrict__ piv) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= entries) return;
    int a, b;
    unpack(e, a, b);
    const int p0 = 2 * k, p1 = 2 * k + 1;
    const bool ia = a == p0 || a == p1, ib = b == p0 || b == p1;
    const S *v1 = cols, *v2 = cols + d;
    if (!ia && !ib) {
        A[e] = sub_dot2(A[e], v1[a], v1[b], v2[a], v2[b]);
    } else if (ia && ib) {  // -P^-1
        const S zero = from_pair<S>(0.0, 0.0);
        if (b == p1) A[e] = sub_mul(zero, piv[1], piv[1]);            // (p1, p1): -s2^2
        else if (a == p1) A[e] = mul_s(piv[2], piv[1]);               // (p1, p0): l s2^2
        else A[e] = sub_dot2(zero, piv[0], piv[0], piv[2], piv[2]);  // (p0, p0)
    } else {                 // A[i, P] P^-1
        const int i = ia ? b : a, p = ia ? a : b;
        if (p == p0) A[e] = sub_mul(mul_s(piv[0], v1[i]), piv[2], v2[i]);
        else A[e] = mul_s(piv[1], v2[i]);
    }
}

__device__ __forceinline__ void put_word(dd *A, int e, dd x) { A[e] = x; }
__device__ __forceinline__ void put_word(qd *A, int e, dd x) { A[e] = qd_from_dd(x); }
__device__ __forceinline__ dd negate(dd x) { return dd_neg(x); }
__device__ __forceinline__ qd negate(qd x) { return qd_neg(x); }

// sigma_Q = sigma + I/2 in packed lower storage from the row-major 2m x 2m
// covariance on the device (the diagonal exact in double-double); entry 0's
// thread also starts the determinant accumulator (product 1, log 0).
template <class S>
__global__ __launch_bounds__(256) void pack_sigq_kernel(const double *__restrict__ cov, int d, int entries,
                                                        S *__restrict__ A, double *__restrict__ acc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= entries) return;
    int a, b;
    unpack(e, a, b);
    const double v = cov[(size_t)a * (size_t)d + (size_t)b];
    dd x;
    if (a == b) two_sum(v, 0.5, x.hi, x.lo);
    else x = dd_from(v);
    put_word(A, e, x);
    if (e == 0) {
        acc[0] = 1.0;
        acc[1] = 0.0;
        acc[2] = 0.0;
    }
}

// the sweeps leave -sigma_Q^-1: negate in place
template <class S> __global__ __launch_bounds__(256) void negate_kernel(S *__restrict__ A, int entries) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < entries) A[e] = negate(A[e]);
}

template <class S>
static hipError_t launch_sweep(void *A, int m, int k, void *cols, void *piv, double *acc, hipStream_t st) {
    const int d = 2 * m;
    const long long entries = (long long)d * (d + 1) / 2;
    (void)hipGetLastError();  // report only these launches' errors
    hipLaunchKernelGGL((sweep_cols_kernel<S>), dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st,
                       (const S *)A, d, k, (S *)cols, (S *)piv, acc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((sweep_update_kernel<S>), dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st, (S *)A,
                       d, k, (int)entries, (const S *)cols, (const S *)piv);
    return hipGetLastError();
}

}  // namespace tor

hipError_t tor_launch_sweep(int is_qd, void *A, int m, int k, void *cols, void *piv, double *acc, hipStream_t st) {
    if (m < 1 || m > TOR_INVERT_MAX_MODES || k < 0 || k >= m) return hipErrorInvalidValue;
    return is_qd ? tor::launch_sweep<qd>(A, m, k, cols, piv, acc, st)
                 : tor::launch_sweep<dd>(A, m, k, cols, piv, acc, st);
}

hipError_t tor_launch_pack_sigq(int is_qd, const double *cov, int m, void *A, double *acc, hipStream_t st) {
    if (m < 1 || m > TOR_INVERT_MAX_MODES) return hipErrorInvalidValue;
    const int d = 2 * m, entries = d * (d + 1) / 2;
    (void)hipGetLastError();
    if (is_qd)
        hipLaunchKernelGGL((tor::pack_sigq_kernel<qd>), dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st, cov,
                           d, entries, (qd *)A, acc);
    else
        hipLaunchKernelGGL((tor::pack_sigq_kernel<dd>), dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st, cov,
                           d, entries, (dd *)A, acc);
    return hipGetLastError();
}

hipError_t tor_launch_negate(int is_qd, void *A, int m, hipStream_t st) {
    if (m < 1 || m > TOR_INVERT_MAX_MODES) return hipErrorInvalidValue;
    const int d = 2 * m, entries = d * (d + 1) / 2;
    (void)hipGetLastError();
    if (is_qd)
        hipLaunchKernelGGL((tor::negate_kernel<qd>), dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st,
                           (qd *)A, entries);
    else
        hipLaunchKernelGGL((tor::negate_kernel<dd>), dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st,
                           (dd *)A, entries);
    return hipGetLastError();
}
