// Device building blocks of the subset tree, shared by the probability
// kernels (tor_kernels.hip) and the chain-rule sampler (gbs_sampler.hip).
//
// A node holds the symmetric matrix M of its r undecided modes in packed
// row-major lower storage (E(r) = r(2r+1) scalars; mode k is rows 2k, 2k+1).
// Deciding the node's last mode: the exclude child is the leading block of M
// (a prefix of the same array); the include child is the Schur complement of
// the last mode's 2x2 pivot block, the vacuum-conditioning update Eq.
// MatrixUpdate of arXiv:1810.00900, with factor q = det(pivot)^-1/2 (the q_k of
// Eq. (prob) at zero mean), and T(M) = T(exclude) - q T(include).
#pragma once
#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "qd.hpp"
#include "tor_kernels.h"

#pragma clang fp contract(off)

namespace tor {

__host__ __device__ constexpr int E(int r) { return r * (2 * r + 1); }
// Entries of an r-mode node: displaced states (D = 1) carry the mean vector as
// an extra leading row [c, mu^T] of the packed matrix (rows 1 + 2k, 2 + 2k for
// mode k); the Schur update of the pivot block then moves the mean exactly as
// the no-click update of Sec. II does.  D = 0: the plain 2r x 2r matrix.
__host__ __device__ constexpr int EN(int r, int D) { return (2 * r + D) * (2 * r + D + 1) / 2; }
// Mean-row mode of the tree templates: D = 0 no mean row; D = 1 a mean row
// whose pivots carry exp(-|w|^2 / 2) (vacuum overlap of a displaced mode);
// D = -1 a mean row whose pivots carry exp(+|w|^2 / 2) (the information-form
// trees of the sampler, where the row holds K mu instead of mu).  MR(D) is
// the number of mean rows.
__host__ __device__ constexpr int MR(int D) { return D != 0 ? 1 : 0; }
__host__ __device__ constexpr int pidx(int a, int b) { return a * (a + 1) / 2 + b; }

// packed lower-triangle index -> (row, column)
__device__ __forceinline__ void unpack(int e, int &a, int &b) {
    int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    if ((r + 1) * (r + 2) / 2 <= e) r++;
    if (r * (r + 1) / 2 > e) r--;
    a = r;
    b = e - r * (r + 1) / 2;
}

// Ordering of LDS accesses among the lanes of a one-wave workgroup (every
// kernel that runs the subset tree launches 64 threads).  LDS operations of a
// wave execute in issue order, so a wavefront-scope fence, which only keeps
// the compiler from moving LDS accesses across it, orders a lane's writes
// before other lanes' later reads; unlike a workgroup barrier it does not
// wait for outstanding stores or global loads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class S> __device__ __forceinline__ S szero();
template <> __device__ __forceinline__ double szero<double>() { return 0.0; }
template <> __device__ __forceinline__ dd szero<dd>() { return dd_make(0.0, 0.0); }

__device__ __forceinline__ double sub_mul(double x, double a, double b) { return fma(-a, b, x); }
__device__ __forceinline__ dd sub_mul(dd x, dd a, dd b) { return dd_sub_mul1(x, a, b); }

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
    // q = det^-1/2 and s1 = alpha^-1/2 are independent (shorter dependency
    // chain); s2 = (gamma - beta^2/alpha)^-1/2 = q alpha^{1/2} = q alpha s1.
    Pivot<S> p;
    const S det = det2(al, be, ga);
    p.s1 = rsqrt_s(al);
    p.q = rsqrt_s(det);
    const S s1sq = mul_s(p.s1, p.s1);
    p.l = mul_s(be, s1sq);
    p.s2 = mul_s(p.q, mul_s(al, p.s1));
    return p;
}

// Pivot of the mode in rows p0, p1 of the packed matrix M.  With D = 1 the
// vacuum probability of the mode gains the overlap factor exp(-|w|^2 / 2) of
// its (conditioned) mean, w = L^-1 mu_B = (v1(0), v2(0)): row 0 holds the
// means, so w is the mean row's entry of the two scaled pivot columns.
// The same from the entries themselves: al, be, ga of the pivot block and,
// with a mean row, the block's mean entries m0, m1 (ignored without one).
template <class S, int D>
__device__ __forceinline__ Pivot<S> make_pivot_v(S al, S be, S ga, S m0, S m1) {
    Pivot<S> pv = make_pivot(al, be, ga);
    if constexpr (D != 0) {
        const S w1 = mul_s(m0, pv.s1);
        const S w2 = mul_s(sub_mul(m1, pv.l, m0), pv.s2);
        pv.q = mul_s(pv.q, exp_s(scale_s(add_s(mul_s(w1, w1), mul_s(w2, w2)), D > 0 ? -0.5 : 0.5)));
    }
    return pv;
}

template <class S, int D>
__device__ __forceinline__ Pivot<S> make_pivot_m(const S *M, int p0, int p1) {
    if constexpr (D != 0)
        return make_pivot_v<S, D>(M[pidx(p0, p0)], M[pidx(p1, p0)], M[pidx(p1, p1)], M[pidx(p0, 0)], M[pidx(p1, 0)]);
    else
        return make_pivot_v<S, D>(M[pidx(p0, p0)], M[pidx(p1, p0)], M[pidx(p1, p1)], M[0], M[0]);
}

// Signed sums and path coefficients: double-double for the binary64 and
// double-double term tiers, quad-double for the quad-double tier.  The
// acc_* overloads give the tree code one spelling for both.
template <class S> struct AccOf { using type = dd; };
template <> struct AccOf<qd> { using type = qd; };

__device__ __forceinline__ dd coef_mul(dd c, double q) { return dd_mul_d(c, q); }
__device__ __forceinline__ dd coef_mul(dd c, dd q) { return dd_mul(c, q); }
__device__ __forceinline__ qd coef_mul(qd c, qd q) { return qd_mul(c, q); }

template <class A> __device__ __forceinline__ A acc_const(double x);
template <> __device__ __forceinline__ dd acc_const<dd>(double x) { return dd_from(x); }
template <> __device__ __forceinline__ qd acc_const<qd>(double x) { return qd_from(x); }
__device__ __forceinline__ dd acc_neg(dd a) { return dd_neg(a); }
__device__ __forceinline__ qd acc_neg(qd a) { return qd_neg(a); }
__device__ __forceinline__ dd acc_mul(dd a, dd b) { return dd_mul(a, b); }
__device__ __forceinline__ qd acc_mul(qd a, qd b) { return qd_mul(a, b); }
__device__ __forceinline__ dd acc_add(dd a, dd b) { return dd_add(a, b); }
__device__ __forceinline__ qd acc_add(qd a, qd b) { return qd_add(a, b); }
// T0 - q T1
__device__ __forceinline__ dd acc_sub_mul(dd t0, double q, dd t1) { return dd_sub_mul(t0, q, t1); }
__device__ __forceinline__ dd acc_sub_mul(dd t0, dd q, dd t1) { return dd_sub_mul(t0, q, t1); }
__device__ __forceinline__ qd acc_sub_mul(qd t0, qd q, qd t1) { return qd_sub(t0, qd_mul(q, t1)); }
// 1 - q
__device__ __forceinline__ dd acc_one_minus(double q) { return dd_sub(dd_from(1.0), to_dd(q)); }
__device__ __forceinline__ dd acc_one_minus(dd q) { return dd_sub(dd_from(1.0), to_dd(q)); }
__device__ __forceinline__ qd acc_one_minus(qd q) { return qd_sub(qd_from(1.0), q); }

// ---------------------------------------------------------------- leaf tier

template <class S, int R, int D = 0> struct Leaf {
    using Acc = typename AccOf<S>::type;
    static __device__ __forceinline__ void run(const S *M, Acc &T, double &A) {
        constexpr int p0 = 2 * R - 2 + MR(D), p1 = 2 * R - 1 + MR(D), RC = 2 * R - 2 + MR(D);
        Acc T0;
        double A0;
        Leaf<S, R - 1, D>::run(M, T0, A0);  // exclude: the prefix of M
        Pivot<S> pv = make_pivot_m<S, D>(M, p0, p1);
        S v1[RC], v2[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            S m0 = M[pidx(p0, c)];
            v1[c] = mul_s(m0, pv.s1);
            v2[c] = mul_s(sub_mul(M[pidx(p1, c)], pv.l, m0), pv.s2);
        }
        S C[EN(R - 1, MR(D))];
#pragma unroll
        for (int a = 0; a < RC; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b)
                C[pidx(a, b)] = sub_dot2(M[pidx(a, b)], v1[a], v1[b], v2[a], v2[b]);
        Acc T1;
        double A1;
        Leaf<S, R - 1, D>::run(C, T1, A1);
        T = acc_sub_mul(T0, pv.q, T1);
        A = A0 + hi_of(pv.q) * A1;
    }
};

template <class S, int D> struct Leaf<S, 1, D> {
    using Acc = typename AccOf<S>::type;
    static __device__ __forceinline__ void run(const S *M, Acc &T, double &A) {
        S q;
        if constexpr (D == 0) q = rsqrt_s(det2(M[0], M[1], M[2]));
        else q = make_pivot_m<S, D>(M, 1, 2).q;
        T = acc_one_minus(q);
        A = 1.0 + hi_of(q);
    }
};

template <class S, int D> struct Leaf<S, 0, D> {
    using Acc = typename AccOf<S>::type;
    static __device__ __forceinline__ void run(const S *, Acc &T, double &A) {
        T = acc_const<Acc>(1.0);
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

__device__ __forceinline__ void wave_reduce(qd &T, double &A) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        qd o = qd_make(shfl_xor_d(T.x0, m), shfl_xor_d(T.x1, m), shfl_xor_d(T.x2, m), shfl_xor_d(T.x3, m));
        double oa = shfl_xor_d(A, m);
        bool low = (threadIdx.x & m) == 0;
        T = low ? qd_add(T, o) : qd_add(o, T);
        A = low ? A + oa : oa + A;
    }
}

// ---------------------------------------------------------------- wave tier

// Modes of the per-lane register leaf: three (binary64, double-double), two
// for quad-double terms (a three-mode leaf does not fit the register file).
template <class S> struct LeafModes { static constexpr int value = 3; };
template <> struct LeafModes<qd> { static constexpr int value = 2; };

template <class S, int J, int D = 0> struct WaveCfg {
    static constexpr int TL = J < LeafModes<S>::value ? J : LeafModes<S>::value;  // leaf modes (registers)
    static constexpr int TW = J - TL;           // levels above the leaves
    static constexpr int TWC = TW > 0 ? TW - 1 : 0;  // levels expanded cooperatively in LDS
    static constexpr int NN = 1 << TWC;         // nodes after the cooperative levels
    static constexpr int NL = 1 << TW;          // leaves (<= 64), one per lane
    // LDS slot offsets: slot base for include children created at level k
    static constexpr int soff(int k) {
        int o = EN(J, MR(D));
        for (int kk = 0; kk < k; ++kk) o += (1 << kk) * EN(J - kk - 1, MR(D));
        return o;
    }
    static constexpr int MAT = soff(TWC);
    // Scaled pivot columns of node 0 at any level (the other nodes keep theirs
    // in their own dead pivot rows)
    static constexpr int VMAX = 2 * (2 * J - 2 + MR(D));
};

// (row, column) of packed index e, for every e < EN(8, D) (the largest child
// of a 9-mode node); identical for every node size since packed storage of a
// smaller matrix is a prefix.
__host__ __device__ constexpr int ab_n(int D) { return EN(8, D); }

// Rank-2 updates a lane keeps in flight per chunk of a cooperative level:
// double-double updates, whose dependency chains are the longest, take up to
// 12 (a nine-mode tree's largest level, 9 per lane, in one chunk); binary64
// trees take 8 (12 measured no faster); quad-double terms 4.
template <class S> struct ChunkW { static constexpr int value = 4; };
template <> struct ChunkW<dd> { static constexpr int value = 12; };
template <> struct ChunkW<double> { static constexpr int value = 8; };

// LDS offset of node i of a J-mode tree after K cooperative levels: node 0 at
// 0, node i >= 1 the include child formed at level k = floor(log2 i) from node
// i - 2^k, in that level's slots.
template <class S, int J, int D, int K>
__device__ __forceinline__ int node_loc(int i) {
    using C = WaveCfg<S, J, D>;
    int o = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (i >= (1 << k)) o = C::soff(k) + (i - (1 << k)) * EN(J - k - 1, MR(D));
    return o;
}

template <class S, int J, int K, int D = 0> struct WaveLevel {
    using C = WaveCfg<S, J, D>;
    using Acc = typename AccOf<S>::type;
    static __device__ __forceinline__ void run(const unsigned short *ab, S *mat, S *vbuf, Acc *coef, double *acoef,
                                               int lane) {
        if constexpr (K < C::TWC) {
            constexpr int r = J - K, R = 2 * r + MR(D), NK = 1 << K, RC = R - 2, EC = EN(r - 1, MR(D));
            // phases 0 and 1: the 64 / NK lanes of each node form its pivot
            // themselves (the same value in each) and then its two scaled
            // columns, a few columns per lane, into the node's own pivot rows,
            // dead once read (node 0's rows, the caller's matrix, are kept: its
            // columns go to vbuf); the node's first lane stores the include
            // child's path coefficients.  Phase 2 updates, in each
            // lane, entries of the lane's own node, so their packed indices and
            // values are loaded here, while the pivot is formed.
            static_assert(64 % NK == 0, "at most 64 nodes per level");
            constexpr int LPN = 64 / NK, NCOL = (RC + LPN - 1) / LPN, NE = (EC + LPN - 1) / LPN;
            const int i = lane / LPN, c0 = lane - i * LPN;
            unsigned short w[NE];
#pragma unroll
            for (int u = 0; u < NE; ++u) w[u] = ab[c0 + LPN * u < EC ? c0 + LPN * u : EC - 1];
            const int nl = node_loc<S, J, D, K>(i);
            S *base = mat + nl;
            // 2 RC <= 2 R - 1 entries: the two pivot rows hold both columns
            S *vcol = mat + (i == 0 ? (int)(vbuf - mat) : nl + pidx(R - 2, 0));
            const Pivot<S> pv = make_pivot_m<S, D>(base, R - 2, R - 1);
            S m0[NCOL], m1[NCOL], x[NE];
#pragma unroll
            for (int j = 0; j < NCOL; ++j) {
                const int c = c0 + LPN * j < RC ? c0 + LPN * j : RC - 1;
                m0[j] = base[pidx(R - 2, c)];
                m1[j] = base[pidx(R - 1, c)];
            }
#pragma unroll
            for (int u = 0; u < NE; ++u) x[u] = base[c0 + LPN * u < EC ? c0 + LPN * u : EC - 1];
#pragma unroll
            for (int j = 0; j < NCOL; ++j) {
                const int c = c0 + LPN * j;
                const S x1 = mul_s(m0[j], pv.s1);
                const S x2 = mul_s(sub_mul(m1[j], pv.l, m0[j]), pv.s2);
                if (c < RC) {
                    vcol[c] = x1;
                    vcol[RC + c] = x2;
                }
            }
            if (c0 == 0) {
                coef[NK + i] = acc_neg(coef_mul(coef[i], pv.q));
                acoef[NK + i] = acoef[i] * hi_of(pv.q);
            }
            wave_sync();
            // phase 2: rank-2 updates of the lane's entries into the include
            // child's slot, in chunks: the chunk's column values first, then
            // the independent updates (so that their dependency chains
            // interleave), then the stores.
            {
                const S *v = vcol;
                S *dst = mat + C::soff(K) + i * EC;
                constexpr int NCH = (NE + ChunkW<S>::value - 1) / ChunkW<S>::value, CH = (NE + NCH - 1) / NCH;
#pragma unroll
                for (int j0 = 0; j0 < NE; j0 += CH) {
                    S p1[CH], q1[CH], p2[CH], q2[CH], r[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int uu = j0 + u < NE ? j0 + u : NE - 1;
                        const int a = w[uu] & 0xff, b = w[uu] >> 8;
                        p1[u] = v[a];
                        q1[u] = v[b];
                        p2[u] = v[RC + a];
                        q2[u] = v[RC + b];
                    }
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int uu = j0 + u < NE ? j0 + u : NE - 1;
                        r[u] = sub_dot2(x[uu], p1[u], q1[u], p2[u], q2[u]);
                    }
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int e = c0 + LPN * (j0 + u);
                        if (j0 + u < NE && e < EC) dst[e] = r[u];
                    }
                }
            }
            wave_sync();
            WaveLevel<S, J, K + 1, D>::run(ab, mat, vbuf, coef, acoef, lane);
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

// LDS working set of the wave tier for a J-mode node.  The index table comes
// first and mat second, at the same offsets for every J.
template <class S, int J, int D = 0> struct WaveSmem {
    using C = WaveCfg<S, J, D>;
    unsigned short ab[ab_n(MR(D))];
    S mat[C::MAT];
    S vbuf[C::VMAX];
    typename AccOf<S>::type coef[C::NN];
    double acoef[C::NN];
};

// Fill the packed-index table (once per workgroup, before the first tree).
template <int D = 0>
__device__ __forceinline__ void wave_tree_init(unsigned short *ab, int lane) {
    for (int e = lane; e < ab_n(MR(D)); e += 64) {
        int a, b;
        unpack(e, a, b);
        ab[e] = (unsigned short)(a | (b << 8));
    }
    wave_sync();
}

// Subset tree of the J-mode node stored in sm.mat[0 .. EN(J, MR(D))) with path
// coefficient (c, a).  The wave expands all but the last of the J - TL levels
// above the leaves breadth-first in LDS; lane l < NL then takes node
// l mod NN, decides its last mode itself (l >= NN: include, a rank-2 Schur
// update in registers; else exclude, the same code with zero update vectors)
// and finishes the TL-mode leaf in registers.  Returns this lane's share
// (T, A) (zero for lanes >= NL).  Lane bit 0 is the decision on the node's last
// mode (1 = included) when J > TL.  The node's matrix is left as it was (the
// levels write only the slot area beyond it, vbuf and the dead pivot rows of
// the nodes in slots).  Must be called by all 64 lanes.
template <class S, int J, int D = 0>
__device__ __forceinline__ void wave_tree(WaveSmem<S, J, D> &sm, typename AccOf<S>::type c, double a, int lane,
                                          typename AccOf<S>::type &T, double &A) {
    using C = WaveCfg<S, J, D>;
    using Acc = typename AccOf<S>::type;
    if (lane == 0) {
        sm.coef[0] = c;
        sm.acoef[0] = a;
    }
    wave_sync();
    WaveLevel<S, J, 0, D>::run(sm.ab, sm.mat, sm.vbuf, sm.coef, sm.acoef, lane);
    T = acc_const<Acc>(0.0);
    A = 0.0;
    if constexpr (C::TW == 0) {
        if (lane == 0) {
            S M[EN(C::TL, MR(D))];
#pragma unroll
            for (int e = 0; e < EN(C::TL, MR(D)); ++e) M[e] = sm.mat[e];
            Acc Tl;
            double Al;
            Leaf<S, C::TL, D>::run(M, Tl, Al);
            T = acc_mul(c, Tl);
            A = a * Al;
        }
    } else {
        if (lane < C::NL) {
            constexpr int R1 = C::TL + 1, p0 = 2 * R1 - 2 + MR(D), p1 = 2 * R1 - 1 + MR(D), RC = 2 * R1 - 2 + MR(D);
            const int i = lane & (C::NN - 1);
            const bool inc = lane >= C::NN;
            const S *base = sm.mat + node_loc<S, J, D, C::TWC>(i);
            S M[EN(R1, MR(D))];
#pragma unroll
            for (int e = 0; e < EN(R1, MR(D)); ++e) M[e] = base[e];
            Pivot<S> pv = make_pivot_m<S, D>(M, p0, p1);
            const S zero = from_pair<S>(0.0, 0.0);
            S v1[RC], v2[RC];
#pragma unroll
            for (int cc = 0; cc < RC; ++cc) {
                S m0 = M[pidx(p0, cc)];
                S x1 = mul_s(m0, pv.s1);
                S x2 = mul_s(sub_mul(M[pidx(p1, cc)], pv.l, m0), pv.s2);
                v1[cc] = inc ? x1 : zero;
                v2[cc] = inc ? x2 : zero;
            }
            S Ml[EN(C::TL, MR(D))];
#pragma unroll
            for (int x = 0; x < RC; ++x)
#pragma unroll
                for (int y = 0; y <= x; ++y) Ml[pidx(x, y)] = sub_dot2(M[pidx(x, y)], v1[x], v1[y], v2[x], v2[y]);
            Acc cl = sm.coef[i];
            double al = sm.acoef[i];
            if (inc) {
                cl = acc_neg(coef_mul(cl, pv.q));
                al *= hi_of(pv.q);
            }
            Acc Tl;
            double Al;
            Leaf<S, C::TL, D>::run(Ml, Tl, Al);
            T = acc_mul(cl, Tl);
            A = al * Al;
        }
    }
}

}  // namespace tor
