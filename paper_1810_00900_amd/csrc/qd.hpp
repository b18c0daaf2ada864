// Quad-double ("qd") arithmetic on IEEE binary64, host and device.
//
// A qd value is an unevaluated sum x0 + x1 + x2 + x3 of binary64 words with
// |x_{i+1}| <= ulp(x_i) (about 212 significant bits).  Sums and products are
// formed level by level: level k collects the exact error terms and partial
// products of order u^k (u = 2^-53) relative to the operands, using the
// error-free transformations TwoSum and TwoProd (dd.hpp) down to level 2 and
// plain binary64 sums at levels 3 and 4; a renormalisation then turns the
// five levels into a non-overlapping expansion.  The design follows the
// level-accumulation scheme of Hida, Li and Bailey (ARITH 2001) and the
// expansion renormalisation of Priest (1991), written here from those
// descriptions.  Error model (checked against mpmath in the CPU tests):
//   add: |err| <= c u^4 (|a| + |b|),  mul: |err| <= c u^4 |a b|,  c ~ 16;
//   rsqrt: relative error about 1.5 e^2 <= ~100 u^4 for a double-double seed
//   with relative error e ~ 2^-103 (one Newton step).
// Weak (operand-relative) accuracy is what the subset tree needs: its error
// bound is relative to the sum of the magnitudes of the terms.
//
// Compile with -ffp-contract=off like dd.hpp.
#pragma once

#include "dd.hpp"

#pragma clang fp contract(off)

struct __align__(16) qd {
    double x0, x1, x2, x3;
};

DD_FN qd qd_make(double a, double b, double c, double d) {
    qd r;
    r.x0 = a;
    r.x1 = b;
    r.x2 = c;
    r.x3 = d;
    return r;
}
DD_FN qd qd_from(double a) { return qd_make(a, 0.0, 0.0, 0.0); }
DD_FN qd qd_from_dd(dd a) { return qd_make(a.hi, a.lo, 0.0, 0.0); }
DD_FN dd qd_to_dd(qd a) {
    // round the leading two levels together with the rest
    double s, e;
    two_sum(a.x0, a.x1 + (a.x2 + a.x3), s, e);
    return dd_make(s, e);
}
DD_FN qd qd_neg(qd a) { return qd_make(-a.x0, -a.x1, -a.x2, -a.x3); }

// Five level sums (|x_k| roughly u^k relative to the leading level, the
// leading levels possibly cancelled) -> non-overlapping four-word expansion.
// Two exact bottom-up TwoSum sweeps (each moves the rounded partial sums up
// and leaves exact errors below) followed by a top-down FastTwoSum sweep that
// compresses the expansion into four words; only the last word is rounded.
DD_FN qd qd_renorm5(double x0, double x1, double x2, double x3, double x4) {
    double s, e1, e2, e3, e4;
    two_sum(x3, x4, s, e4);
    two_sum(x2, s, s, e3);
    two_sum(x1, s, s, e2);
    two_sum(x0, s, s, e1);
    // second sweep over (s, e1, e2, e3, e4)
    double t, f1, f2, f3, f4;
    two_sum(e3, e4, t, f4);
    two_sum(e2, t, t, f3);
    two_sum(e1, t, t, f2);
    two_sum(s, t, t, f1);
    // top-down compression of t + f1 + f2 + f3 + f4
    double r0, r1, r2, r3, c;
    fast_two_sum(t, f1, r0, c);
    two_sum(c, f2, r1, c);
    two_sum(c, f3, r2, c);
    r3 = c + f4;
    // make the words non-overlapping after the compression
    fast_two_sum(r2, r3, r2, r3);
    fast_two_sum(r1, r2, r1, r2);
    fast_two_sum(r0, r1, r0, r1);
    fast_two_sum(r1, r2, r1, r2);
    fast_two_sum(r2, r3, r2, r3);
    return qd_make(r0, r1, r2, r3);
}

// a + b
DD_FN qd qd_add(qd a, qd b) {
    double s0, e0, s1, e1, s2, e2, s3, e3;
    two_sum(a.x0, b.x0, s0, e0);  // level 0 (+ error at level 1)
    two_sum(a.x1, b.x1, s1, e1);  // level 1 (+ level 2)
    two_sum(a.x2, b.x2, s2, e2);  // level 2 (+ level 3)
    two_sum(a.x3, b.x3, s3, e3);  // level 3 (+ level 4)
    double l1, c1, l2, c2, c3;
    two_sum(s1, e0, l1, c1);      // level 1, carry to level 2
    two_sum(s2, e1, l2, c2);      // level 2, carry to level 3
    two_sum(l2, c1, l2, c3);
    const double l3 = s3 + e2 + (c2 + c3);
    return qd_renorm5(s0, l1, l2, l3, e3);
}
DD_FN qd qd_sub(qd a, qd b) { return qd_add(a, qd_neg(b)); }

// Level sums of a * b before renormalisation: a*b = L0 + L1 + L2 + L3 + L4
// up to order-5 terms, with L0..L2 single words (the exact errors of their
// TwoSums pushed to the next level) and L3, L4 plain binary64 sums.
struct QdLevels {
    double l0, l1, l2, l3, l4;
};
DD_FN QdLevels qd_mul_levels(qd a, qd b) {
    QdLevels o;
    double q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
    two_prod(a.x0, b.x0, o.l0, q00);
    two_prod(a.x0, b.x1, p01, q01);
    two_prod(a.x1, b.x0, p10, q10);
    two_prod(a.x0, b.x2, p02, q02);
    two_prod(a.x1, b.x1, p11, q11);
    two_prod(a.x2, b.x0, p20, q20);
    double c1, c2;
    two_sum(p01, p10, o.l1, c1);
    two_sum(o.l1, q00, o.l1, c2);
    double d1, d2, d3, d4, d5, d6;
    two_sum(p02, p11, o.l2, d1);
    two_sum(o.l2, p20, o.l2, d2);
    two_sum(o.l2, q01, o.l2, d3);
    two_sum(o.l2, q10, o.l2, d4);
    two_sum(o.l2, c1, o.l2, d5);
    two_sum(o.l2, c2, o.l2, d6);
    const double o3 = fma(a.x0, b.x3, fma(a.x1, b.x2, fma(a.x2, b.x1, a.x3 * b.x0)));
    o.l3 = o3 + ((q02 + q11) + q20) + (((d1 + d2) + (d3 + d4)) + (d5 + d6));
    o.l4 = fma(a.x1, b.x3, fma(a.x2, b.x2, a.x3 * b.x1));
    return o;
}

// a * b: partial products a_i b_j of order i + j <= 2 exact (TwoProd), order 3
// with their rounding, order 4 in binary64; orders >= 5 dropped.
DD_FN qd qd_mul(qd a, qd b) {
    const QdLevels p = qd_mul_levels(a, b);
    return qd_renorm5(p.l0, p.l1, p.l2, p.l3, p.l4);
}

// a * b for a binary64 b
DD_FN qd qd_mul_d(qd a, double b) {
    double p0, q0, p1, q1, p2, q2;
    two_prod(a.x0, b, p0, q0);
    two_prod(a.x1, b, p1, q1);
    two_prod(a.x2, b, p2, q2);
    double l1, c1, l2, c2, c3;
    two_sum(p1, q0, l1, c1);
    two_sum(p2, q1, l2, c2);
    two_sum(l2, c1, l2, c3);
    const double l3 = fma(a.x3, b, q2 + (c2 + c3));
    return qd_renorm5(p0, l1, l2, l3, 0.0);
}

// x - a1 b1 - a2 b2 (the rank-2 Schur update of one entry), fused: the two
// products stay level sums, the three operands are combined level by level
// (exact TwoSums at levels 0-2, their errors carried down; plain sums at
// levels 3-4) and the result is renormalised once.  Error within c u^4
// (|x| + |a1 b1| + |a2 b2|), as for the unfused form.
DD_FN qd qd_sub_dot2(qd x, qd a1, qd b1, qd a2, qd b2) {
    const QdLevels p = qd_mul_levels(a1, b1), r = qd_mul_levels(a2, b2);
    double s0, s1, s2, e0, e1, f0, f1, f2, f3, g0, g1, g2, g3, g4, g5;
    two_sum(x.x0, -p.l0, s0, e0);  // level 0
    two_sum(s0, -r.l0, s0, e1);
    two_sum(x.x1, -p.l1, s1, f0);  // level 1
    two_sum(s1, -r.l1, s1, f1);
    two_sum(s1, e0, s1, f2);
    two_sum(s1, e1, s1, f3);
    two_sum(x.x2, -p.l2, s2, g0);  // level 2
    two_sum(s2, -r.l2, s2, g1);
    two_sum(s2, f0, s2, g2);
    two_sum(s2, f1, s2, g3);
    two_sum(s2, f2, s2, g4);
    two_sum(s2, f3, s2, g5);
    const double s3 = ((x.x3 - p.l3) - r.l3) + (((g0 + g1) + (g2 + g3)) + (g4 + g5));
    const double s4 = -(p.l4 + r.l4);
    return qd_renorm5(s0, s1, s2, s3, s4);
}
// x - a b
DD_FN qd qd_sub_mul(qd x, qd a, qd b) {
    const QdLevels p = qd_mul_levels(a, b);
    double s0, s1, s2, e0, f0, f1, g0, g1, g2;
    two_sum(x.x0, -p.l0, s0, e0);
    two_sum(x.x1, -p.l1, s1, f0);
    two_sum(s1, e0, s1, f1);
    two_sum(x.x2, -p.l2, s2, g0);
    two_sum(s2, f0, s2, g1);
    two_sum(s2, f1, s2, g2);
    const double s3 = (x.x3 - p.l3) + ((g0 + g1) + g2);
    return qd_renorm5(s0, s1, s2, s3, -p.l4);
}
// a c - b^2 (2x2 determinant), fused like qd_sub_dot2
DD_FN qd qd_det2(qd a, qd b, qd c) {
    const QdLevels p = qd_mul_levels(a, c), r = qd_mul_levels(b, b);
    double s0, s1, s2, e0, f0, f1, g0, g1, g2;
    two_sum(p.l0, -r.l0, s0, e0);
    two_sum(p.l1, -r.l1, s1, f0);
    two_sum(s1, e0, s1, f1);
    two_sum(p.l2, -r.l2, s2, g0);
    two_sum(s2, f0, s2, g1);
    two_sum(s2, f1, s2, g2);
    const double s3 = (p.l3 - r.l3) + ((g0 + g1) + g2);
    return qd_renorm5(s0, s1, s2, s3, p.l4 - r.l4);
}

// x^-1/2: the double-double estimate, then one Newton step in qd,
// y <- y + y (1 - x y^2) / 2 (quadratic convergence: 2^-104 -> 2^-207).
DD_FN qd qd_rsqrt(qd x) {
    const dd y0 = dd_rsqrt(qd_to_dd(x));
    const qd y = qd_from_dd(y0);
    const qd r = qd_sub(qd_from(1.0), qd_mul(x, qd_mul(y, y)));
    return qd_add(y, qd_mul_d(qd_mul(y, r), 0.5));
}

// exp(x) of a quad-double x (finite, x.x0 < 709).  Reduction x = k ln2 + r
// with a four-word ln2 (|r| <= ln2 / 2), t = r / 1024.  expm1(t) = t P(t),
// P(t) = sum_{j=0}^{16} t^j / (j+1)!, by Horner: the coefficients 1/13!..1/17!
// in binary64 and 1/9!..1/12! in double-word (their terms sit below 2^-51 and
// 2^-110 of the result, so those precisions suffice), 1/1!..1/8! in
// quad-double; the next term, t^17/18!, is below 2^-220.  Ten doublings
// e^{2t} - 1 = a (2 + a) keep a's relative precision; exp(x) = 2^k (1 + a).
// The constants are the round-to-nearest four-word splits of ln2 and 1/j!.
// Relative error within a few max(1, |x|) 2^-208 (the conditioning of exp on
// a four-word argument) for results above 1e-290; 0 below exp(-745).
DD_FN qd qd_exp(qd x) {
    if (x.x0 < -745.0) return qd_from(0.0);
    const qd ln2 = qd_make(0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56, 0x1.7b57a079a1934p-111,
                           -0x1.ace93a4ebe5d1p-165);
    const double k = rint(x.x0 / ln2.x0);
    qd t = qd_sub(x, qd_mul_d(ln2, k));
    t = qd_make(ldexp(t.x0, -10), ldexp(t.x1, -10), ldexp(t.x2, -10), ldexp(t.x3, -10));
    double p = 0x1.952c77030ad4ap-49;         // 1/17!
    p = fma(p, t.x0, 0x1.ae7f3e733b81fp-45);  // 1/16!
    p = fma(p, t.x0, 0x1.ae7f3e733b81fp-41);  // 1/15!
    p = fma(p, t.x0, 0x1.93974a8c07c9dp-37);  // 1/14!
    p = fma(p, t.x0, 0x1.6124613a86d09p-33);  // 1/13!
    const dd td = dd_make(t.x0, t.x1);
    const double dh[4] = {0x1.1eed8eff8d898p-29, 0x1.ae64567f544e4p-26, 0x1.27e4fb7789f5cp-22,
                          0x1.71de3a556c734p-19};  // 1/12!, 1/11!, 1/10!, 1/9!
    const double dl[4] = {-0x1.2aec959e14c06p-83, -0x1.c062e06d1f209p-80, 0x1.cbbc05b4fa99ap-76,
                          -0x1.c154f8ddc6c00p-73};
    dd sd = dd_from(p);
    for (int j = 0; j < 4; ++j) sd = dd_add_small(dd_make(dh[j], dl[j]), dd_mul(td, sd));
    const double c[8][4] = {  // 1/8!, 1/7!, ..., 1/1!
        {0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76, 0x1.a01a01a01a01ap-136, 0x1.a01a01a01a01ap-196},
        {0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-73, 0x1.a01a01a01a01ap-133, 0x1.a01a01a01a01ap-193},
        {0x1.6c16c16c16c17p-10, -0x1.f49f49f49f49fp-65, -0x1.27d27d27d27d2p-119, -0x1.f49f49f49f49fp-173},
        {0x1.1111111111111p-7, 0x1.1111111111111p-63, 0x1.1111111111111p-119, 0x1.1111111111111p-175},
        {0x1.5555555555555p-5, 0x1.5555555555555p-59, 0x1.5555555555555p-113, 0x1.5555555555555p-167},
        {0x1.5555555555555p-3, 0x1.5555555555555p-57, 0x1.5555555555555p-111, 0x1.5555555555555p-165},
        {0x1.0000000000000p-1, 0.0, 0.0, 0.0},
        {1.0, 0.0, 0.0, 0.0}};
    qd s = qd_from_dd(sd);
    for (int j = 0; j < 8; ++j) s = qd_add(qd_make(c[j][0], c[j][1], c[j][2], c[j][3]), qd_mul(t, s));
    qd a = qd_mul(t, s);
    for (int i = 0; i < 10; ++i) a = qd_mul(a, qd_add(qd_from(2.0), a));
    a = qd_add(qd_from(1.0), a);
    const int ik = (int)k;
    return qd_make(ldexp(a.x0, ik), ldexp(a.x1, ik), ldexp(a.x2, ik), ldexp(a.x3, ik));
}

// helpers with the call shape of the other scalar tiers
DD_FN qd sub_dot2(qd x, qd a1, qd b1, qd a2, qd b2) { return qd_sub_dot2(x, a1, b1, a2, b2); }
DD_FN qd sub_mul(qd x, qd a, qd b) { return qd_sub_mul(x, a, b); }
DD_FN qd det2(qd a, qd b, qd c) { return qd_det2(a, b, c); }
DD_FN qd rsqrt_s(qd x) { return qd_rsqrt(x); }
DD_FN qd mul_s(qd a, qd b) { return qd_mul(a, b); }
DD_FN double hi_of(qd a) { return a.x0; }
DD_FN qd exp_s(qd x) { return qd_exp(x); }
DD_FN qd add_s(qd a, qd b) { return qd_add(a, b); }
DD_FN qd scale_s(qd a, double f) { return qd_mul_d(a, f); }

template <> DD_FN qd from_pair<qd>(double h, double l) {
    double s, e;
    two_sum(h, l, s, e);
    return qd_make(s, e, 0.0, 0.0);
}
