// The chain-rule sampler's per-chain work (one 64-lane wave), shared by the
// sampler kernel (gbs_sampler.hip) and the persistent request loop
// (tor_pserver.hip).  A chain measures the modes in ascending order; at mode j
// with clicked set C and no-click set N among the earlier modes the no-click
// probability is p(C, N + j) / p(C, N), evaluated as the ratio X0 / X1 of the
// split subset tree over G = K_j[C + j] (K_j = sigma_Q[0..j]^-1, a Jacobi
// complementary-minor identity), and the coin is Philox4x32-10 keyed by
// (seed, chain, mode).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor_kernels.h"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// multiply-xor round with multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key
// increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const unsigned lo0 = c.x * 0xD2511F53u, hi0 = __umulhi(c.x, 0xD2511F53u);
        const unsigned lo1 = c.z * 0xCD9E8D57u, hi1 = __umulhi(c.z, 0xCD9E8D57u);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// uniform in [0, 1) with 53 random bits from the first two output words
__device__ __forceinline__ double philox_uniform(unsigned long long seed, long long chain, int step) {
    uint4 x = philox4x32_10(make_uint4((unsigned)chain, (unsigned)((unsigned long long)chain >> 32),
                                       (unsigned)step, 0u),
                            make_uint2((unsigned)seed, (unsigned)(seed >> 32)));
    unsigned long long b = ((unsigned long long)x.x << 21) | (unsigned long long)(x.y >> 11);
    return (double)b * 0x1.0p-53;
}

// Root split of a TL-mode tree for J <= 3 (one leaf): X0 = T(exclude last),
// X1s = -q T(include last), and the sums of the terms' magnitudes A0, A1 of
// the two halves.
template <class S, int R, int D>
__device__ __forceinline__ void leaf_split(const S *M, dd &X0, dd &X1s, double &A0, double &A1) {
    if constexpr (R == 1) {
        S q;
        if constexpr (D == 0) q = rsqrt_s(det2(M[0], M[1], M[2]));
        else q = make_pivot_m<S, D>(M, 1, 2).q;
        X0 = dd_from(1.0);
        X1s = dd_neg(to_dd(q));
        A0 = 1.0;
        A1 = hi_of(q);
    } else {
        constexpr int p0 = 2 * R - 2 + MR(D), p1 = 2 * R - 1 + MR(D), RC = 2 * R - 2 + MR(D);
        Leaf<S, R - 1, D>::run(M, X0, A0);
        Pivot<S> pv = make_pivot_m<S, D>(M, p0, p1);
        S v1[RC], v2[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            S m0 = M[pidx(p0, c)];
            v1[c] = mul_s(m0, pv.s1);
            v2[c] = mul_s(sub_mul(M[pidx(p1, c)], pv.l, m0), pv.s2);
        }
        S Cm[EN(R - 1, MR(D))];
#pragma unroll
        for (int a = 0; a < RC; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) Cm[pidx(a, b)] = sub_dot2(M[pidx(a, b)], v1[a], v1[b], v2[a], v2[b]);
        dd T1;
        double Ac;
        Leaf<S, R - 1, D>::run(Cm, T1, Ac);
        X1s = dd_neg(coef_mul(T1, pv.q));
        A1 = hi_of(pv.q) * Ac;
    }
}

// Include-child of an r-mode node in LDS (cooperative rank-2 Schur update of
// the last mode); returns q.  in and out must not overlap.
template <class S, int D>
__device__ __forceinline__ S wave_schur_last(const S *in, int r, S *out, S *vt, int lane) {
    const int R = 2 * r + MR(D), RC = R - 2, EC = EN(r - 1, MR(D));
    Pivot<S> pv = make_pivot_m<S, D>(in, R - 2, R - 1);
    for (int c = lane; c < RC; c += 64) {
        S m0 = in[pidx(R - 2, c)];
        vt[c] = mul_s(m0, pv.s1);
        vt[RC + c] = mul_s(sub_mul(in[pidx(R - 1, c)], pv.l, m0), pv.s2);
    }
    wave_sync();
    for (int e = lane; e < EC; e += 64) {
        int a, b;
        unpack(e, a, b);
        out[e] = sub_dot2(in[e], vt[a], vt[b], vt[RC + a], vt[RC + b]);
    }
    wave_sync();
    return pv.q;
}

template <class S, int J, int D> struct ChainStep {
    // tree of the k = J modes already gathered into the wave LDS (k <= 9);
    // this lane's shares of the two halves' sums and magnitude sums
    static __device__ __forceinline__ void run(unsigned char *raw, int lane, dd &X0, dd &X1s, double &A0,
                                               double &A1) {
        using C = WaveCfg<S, J, D>;
        WaveSmem<S, J, D> &sm = *reinterpret_cast<WaveSmem<S, J, D> *>(raw);
        if constexpr (C::TW == 0) {
            X0 = dd_from(0.0);
            X1s = dd_from(0.0);
            A0 = A1 = 0.0;
            if (lane == 0) {
                S M[EN(J, MR(D))];
#pragma unroll
                for (int e = 0; e < EN(J, MR(D)); ++e) M[e] = sm.mat[e];
                leaf_split<S, J, D>(M, X0, X1s, A0, A1);
            }
            wave_sync();
        } else {
            dd T;
            double A;
            wave_tree<S, J, D>(sm, dd_from(1.0), 1.0, lane, T, A);
            X0 = (lane & 1) ? dd_from(0.0) : T;
            X1s = (lane & 1) ? T : dd_from(0.0);
            A0 = (lane & 1) ? 0.0 : A;
            A1 = (lane & 1) ? A : 0.0;
            wave_sync();
        }
    }
};

template <class S, int D> struct ChainLds {
    static constexpr size_t wave_bytes = sizeof(WaveSmem<S, 9, D>);
};

// Run chain P.chain_begin + ci to its end and write its outcomes (and the
// optional trace) at row ci of P's outputs.  raw: LDS of
// ChainLds<S, D>::wave_bytes; g0 (the step's matrix G) and g12 (two buffers
// one after the other for its Schur complements, ping-pong), vt, Cl: LDS for
// the top decisions of trees with more than nine modes (EN(KMAX) scalars per
// buffer, KMAX modes at most; g12 may lie in raw's slot area past the
// nine-mode matrix, which the nine-mode tree overwrites only after they are
// read).  All 64 lanes call it.
template <class S, int KMAX, int D>
__device__ __forceinline__ void run_chain(const ChainParams &P, int ci, unsigned char *raw, S *g0, S *g12,
                                          S *vt, int *Cl, int lane) {
    constexpr int O = MR(D);  // mean rows
    // ab[] then mat[] sit at the same offsets in WaveSmem<S, J, D> for every J
    S *wmat = reinterpret_cast<WaveSmem<S, 9, D> *>(raw)->mat;
    const long long chain = P.chain_begin + ci;
    int nc = 0;
    signed char st = 1;
    double nsub = 0.0;
    int j = 0;
    for (; j < P.m; ++j) {
        if (P.n_post >= 0 && (nc > P.n_post || nc + (P.m - j) < P.n_post)) {
            st = 0;
            break;
        }
        if (nc + 1 > KMAX || nc > P.cap) {
            st = 2;
            break;
        }
        const int k = nc + 1;
        const int ld = 2 * j + 2;
        const double *Kj = P.K + P.koff[j];
        const double *Klj = P.Klo ? P.Klo + P.koff[j] : nullptr;
        S *G = k <= 9 ? wmat : g0;
        for (int e = lane; e < EN(k, O); e += 64) {
            int a, b;
            unpack(e, a, b);
            if (O && b == 0) {  // the mean column: h_j of the row's quadrature (0 at the corner)
                const int aa = a - 1;
                const int ma = (aa >> 1) < nc ? Cl[aa >> 1] : j;
                const size_t he = P.hoff[j] + 2 * ma + (aa & 1);
                G[e] = a == 0 ? from_pair<S>(0.0, 0.0) : from_pair<S>(P.H[he], P.Hlo ? P.Hlo[he] : 0.0);
                continue;
            }
            a -= O;
            b -= O;
            const int ma = (a >> 1) < nc ? Cl[a >> 1] : j;
            const int mb = (b >> 1) < nc ? Cl[b >> 1] : j;
            const size_t ke = (size_t)(2 * ma + (a & 1)) * ld + 2 * mb + (b & 1);
            G[e] = (S)from_pair<S>(Kj[ke], Klj ? Klj[ke] : 0.0);
        }
        wave_sync();
        dd X0 = dd_from(0.0), X1s = dd_from(0.0);
        double A0 = 0.0, A1 = 0.0;
        if (k <= 9) {
            switch (k) {
            case 1: ChainStep<S, 1, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 2: ChainStep<S, 2, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 3: ChainStep<S, 3, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 4: ChainStep<S, 4, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 5: ChainStep<S, 5, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 6: ChainStep<S, 6, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 7: ChainStep<S, 7, D>::run(raw, lane, X0, X1s, A0, A1); break;
            case 8: ChainStep<S, 8, D>::run(raw, lane, X0, X1s, A0, A1); break;
            default: ChainStep<S, 9, D>::run(raw, lane, X0, X1s, A0, A1); break;
            }
        } else {
            // decisions on the top u = k - 9 modes (bit b: mode k-1-b; bit 0 is mode j)
            const int u = k - 9;
            WaveSmem<S, 9, D> &sm = *reinterpret_cast<WaveSmem<S, 9, D> *>(raw);
            for (int p = 0; p < (1 << u); ++p) {
                const S *cur = g0;
                int r = k, nb = 1;
                dd c = dd_from(1.0);
                double a = 1.0;
                for (int b = 0; b < u; ++b, --r) {
                    if ((p >> b) & 1) {
                        S *o = g12 + (nb == 1 ? 0 : EN(KMAX, MR(D)));
                        S q = wave_schur_last<S, D>(cur, r, o, vt, lane);
                        c = dd_neg(coef_mul(c, q));
                        a *= hi_of(q);
                        cur = o;
                        nb = 3 - nb;
                    }
                }
                for (int e = lane; e < EN(9, O); e += 64) sm.mat[e] = cur[e];
                wave_sync();
                dd T;
                double A;
                wave_tree<S, 9, D>(sm, c, a, lane, T, A);
                if (p & 1) {
                    X1s = dd_add(X1s, T);
                    A1 += A;
                } else {
                    X0 = dd_add(X0, T);
                    A0 += A;
                }
                wave_sync();
            }
        }
        wave_reduce(X0, A0);
        wave_reduce(X1s, A1);
        nsub += (double)(1 << k);
        // P(no click) = X0 / X1 with X1 = -X1s; all lanes hold the same sums.
        // Double-double terms: P(click) = (X1s + X0) / X1s, the difference
        // taken before the rounding to binary64.
        const double x0 = X0.hi + X0.lo, x1 = -(X1s.hi + X1s.lo);
        double pclick;
        if constexpr (sizeof(S) > sizeof(double)) {
            const dd num = dd_add(X1s, X0);
            pclick = (num.hi + num.lo) / (X1s.hi + X1s.lo);
        } else {
            pclick = 1.0 - x0 / x1;
        }
        const double uni = philox_uniform(P.seed, chain, j);
        const bool click = uni < pclick;
        if (lane == 0) {
            const size_t o = (size_t)ci * (size_t)P.m + (size_t)j;
            P.outcome[o] = click ? 1 : 0;
            if (P.trace_p) P.trace_p[o] = pclick;
            if (P.trace_u) P.trace_u[o] = uni;
            if (P.trace_r || P.trace_b) {
                // each half's relative error is at most 16 (k + 1) u R_i (k
                // Schur levels, the rounding of G's entries, R_i its
                // cancellation ratio; binary64 G for binary64 terms, G to
                // ~2m u_dd for double-double terms), so the ratio's is their
                // sum; then the final quotient and difference in binary64
                const double r0 = A0 / fabs(x0), r1 = A1 / fabs(x1), ratio = fabs(x0 / x1);
                const double u = sizeof(S) > sizeof(double) ? 0x1.0p-104 : 0x1.0p-53;
                const double uk = sizeof(S) > sizeof(double) ? 2.0 * P.m * 0x1.0p-104 : 0.0;
                if (P.trace_r) P.trace_r[o] = r0 > r1 ? r0 : r1;
                if (P.trace_b)
                    P.trace_b[o] = 16.0 * ((k + 1) * u + uk) * (r0 + r1) * ratio + 0x1.0p-52 * (ratio + fabs(pclick));
            }
            if (click) Cl[nc] = j;
        }
        wave_sync();
        if (click) nc++;
    }
    if (st == 1 && P.n_post >= 0 && nc != P.n_post) st = 0;
    for (int jj = j + lane; jj < P.m; jj += 64) {
        const size_t o = (size_t)ci * (size_t)P.m + (size_t)jj;
        P.outcome[o] = 0;
        if (P.trace_p) P.trace_p[o] = __builtin_nan("");
        if (P.trace_u) P.trace_u[o] = __builtin_nan("");
        if (P.trace_r) P.trace_r[o] = __builtin_nan("");
        if (P.trace_b) P.trace_b[o] = __builtin_nan("");
    }
    if (lane == 0) {
        P.status[ci] = st;
        if (P.subsets) P.subsets[ci] = nsub;
    }
}

}  // namespace tor
