// Exact chain-rule sampling of threshold-detector GBS on the GPU.
//
// A sample is drawn mode by mode in ascending order (the paper's algorithm
// measures one mode at a time, Sec. II; any order is exact).  At mode j, with
// clicked set C and no-click set N among the modes before j, the probability of
// no click is p(C, N + j) / p(C, N).  Because every mode before j is in C or N,
// the vacuum-conditioned matrix of C + {j} is the inverse of
// G = K_j[C + j], K_j = (sigma_Q[0..j])^-1 (a Jacobi complementary-minor
// identity), and the subset sum over Sigma = G^-1 equals +-det(G)^{1/2} times the
// same sum over G.  Deciding j first in the tree over G splits it into
// X0 = T(G[C]) and X1 = q_j T(G / G_jj); then P(no click at j) = X0 / X1.  So a
// chain carries only its click list; the K_j are shared by all chains.
//
// One 64-lane workgroup runs one chain at a time: per mode it gathers G into
// LDS, evaluates the split subset tree (the wave tier; modes above 9 by a loop
// over the top decisions with rank-2 Schur updates in LDS), draws the coin from
// Philox4x32-10 keyed by (seed, chain, mode), and stops early when the
// postselection on n clicks can no longer be met.
//
// Displaced states (mean mu): in the same information form every vacuum
// probability P_vac(S) = det(sigma_Q[S])^-1/2 exp(-mu_S^T sigma_Q[S]^-1 mu_S / 2)
// becomes, with K = K_j and h = K mu[0..j], a common factor times
// det(K[Sbar])^-1/2 exp(+h_Sbar^T K[Sbar]^-1 h_Sbar / 2), Sbar the complement
// of S in modes 0..j (the quadratic form of a marginal in information form is
// the full one minus the complement's).  The common factors cancel in the
// ratio, so the same split tree runs over G with h[C + j] as a leading mean
// row and pivot factors exp(+|w|^2 / 2) (tree mode D = -1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor_kernels.h"
#include "tor_chain.hpp"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

// KMAX: largest step tree (clicks so far + 1) the kernel's LDS holds; two
// instances, so that chains with few clicks keep the smaller footprint.
// D = 0: zero-mean state; D = -1: displaced state (mean row h = K_j mu).
template <class S, int KMAX, int D>
__global__ __launch_bounds__(64) void chain_kernel(ChainParams P) {
    constexpr int O = MR(D);  // mean rows
    __shared__ __align__(16) unsigned char raw[ChainLds<S, D>::wave_bytes];
    // G in its own buffer; its two Schur complements in the nine-mode tree's
    // slot area (past the nine-mode matrix) when they fit, else beside G
    constexpr int EK = EN(KMAX, O), E9 = EN(9, O), MAT = WaveCfg<S, 9, D>::MAT;
    constexpr bool IN_SLOTS = E9 + 2 * EK <= MAT;
    __shared__ S gbuf[IN_SLOTS ? 1 : 3][EK];
    S *g12;
    if constexpr (IN_SLOTS) g12 = reinterpret_cast<WaveSmem<S, 9, D> *>(raw)->mat + E9;
    else g12 = gbuf[IN_SLOTS ? 0 : 1];  // gbuf[1], gbuf[2]
    __shared__ S vt[4 * KMAX];
    __shared__ int Cl[KMAX + 1];
    const int lane = threadIdx.x;
    wave_tree_init<D>(reinterpret_cast<WaveSmem<S, 9, D> *>(raw)->ab, lane);
    for (int ci = blockIdx.x; ci < P.nchains; ci += gridDim.x) {
        run_chain<S, KMAX, D>(P, ci, raw, gbuf[0], g12, vt, Cl, lane);
        wave_sync();
    }
}

}  // namespace tor

hipError_t tor_launch_chains(const ChainParams &P, int grid_cap, hipStream_t st) {
    int g = P.nchains < grid_cap ? P.nchains : grid_cap;
    if (g < 1) return hipSuccess;
    (void)hipGetLastError();  // report only this launch's error
    const bool small = P.cap + 1 <= TOR_CHAIN_MAX;
    if (P.Klo) {  // double-double terms
        if (P.H && small)
            hipLaunchKernelGGL((tor::chain_kernel<dd, TOR_CHAIN_MAX, -1>), dim3((unsigned)g), dim3(64), 0, st, P);
        else if (P.H)
            hipLaunchKernelGGL((tor::chain_kernel<dd, TOR_CHAIN_MAX_BIG, -1>), dim3((unsigned)g), dim3(64), 0, st, P);
        else if (small)
            hipLaunchKernelGGL((tor::chain_kernel<dd, TOR_CHAIN_MAX, 0>), dim3((unsigned)g), dim3(64), 0, st, P);
        else
            hipLaunchKernelGGL((tor::chain_kernel<dd, TOR_CHAIN_MAX_BIG, 0>), dim3((unsigned)g), dim3(64), 0, st, P);
        return hipGetLastError();
    }
    if (P.H && small)
        hipLaunchKernelGGL((tor::chain_kernel<double, TOR_CHAIN_MAX, -1>), dim3((unsigned)g), dim3(64), 0, st, P);
    else if (P.H)
        hipLaunchKernelGGL((tor::chain_kernel<double, TOR_CHAIN_MAX_BIG, -1>), dim3((unsigned)g), dim3(64), 0, st, P);
    else if (small)
        hipLaunchKernelGGL((tor::chain_kernel<double, TOR_CHAIN_MAX, 0>), dim3((unsigned)g), dim3(64), 0, st, P);
    else
        hipLaunchKernelGGL((tor::chain_kernel<double, TOR_CHAIN_MAX_BIG, 0>), dim3((unsigned)g), dim3(64), 0, st, P);
    return hipGetLastError();
}
