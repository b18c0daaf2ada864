// Double-double ("dd") arithmetic on IEEE binary64, host and device.
//
// A dd value is an unevaluated sum hi + lo with |lo| <= ulp(hi)/2, giving about
// 106 significant bits.  The error-free transformations are Knuth's TwoSum,
// Dekker's FastTwoSum and the FMA-based TwoProd; addition follows the
// "accurate" double-word sum and multiplication the double-word product analysed
// by Joldes, Muller and Popescu (ACM TOMS 44(4), 2017), relative error <= 3u^2
// and <= 5u^2 (u = 2^-53).  Every routine here is written from those
// published algorithms.
//
// This file MUST be compiled with floating-point contraction disabled
// (-ffp-contract=off): TwoSum and FastTwoSum are exact only if each operation
// rounds on its own.  FMAs are written explicitly where an algorithm needs one.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
#define DD_FN __host__ __device__ __forceinline__
#else
#define DD_FN inline
#endif

#pragma clang fp contract(off)

struct __align__(16) dd {
    double hi, lo;
};

DD_FN dd dd_make(double h, double l) { dd r; r.hi = h; r.lo = l; return r; }
DD_FN dd dd_from(double x) { return dd_make(x, 0.0); }

// s + e == a + b exactly (any a, b).
DD_FN void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// s + e == a + b exactly, requires exponent(a) >= exponent(b) (e.g. |a| >= |b|).
DD_FN void fast_two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    e = b - (s - a);
}

// p + e == a * b exactly (barring underflow), using one FMA.
DD_FN void two_prod(double a, double b, double &p, double &e) {
    p = a * b;
    e = fma(a, b, -p);
}

DD_FN dd dd_neg(dd a) { return dd_make(-a.hi, -a.lo); }

// Accurate double-word + double-word.
DD_FN dd dd_add(dd x, dd y) {
    double sh, sl, th, tl;
    two_sum(x.hi, y.hi, sh, sl);
    two_sum(x.lo, y.lo, th, tl);
    sl += th;
    double vh, vl;
    fast_two_sum(sh, sl, vh, vl);
    vl += tl;
    dd r;
    fast_two_sum(vh, vl, r.hi, r.lo);
    return r;
}

DD_FN dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

// double-word * double
DD_FN dd dd_mul_d(dd x, double y) {
    double p, e;
    two_prod(x.hi, y, p, e);
    e = fma(x.lo, y, e);
    dd r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
}

// double-word * double-word
DD_FN dd dd_mul(dd x, dd y) {
    double p, e;
    two_prod(x.hi, y.hi, p, e);
    double t = x.lo * y.hi;
    t = fma(x.hi, y.lo, t);
    e += t;
    dd r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
}

// x - a1*b1 - a2*b2 in one pass.  The leading products are split exactly
// (p + e == a.hi*b.hi via FMA), the cross terms a.hi*b.lo + a.lo*b.hi are
// folded into e with two more FMAs, the leading sum x.hi - p1 - p2 is formed
// error-free with two TwoSums, and every second-order term is gathered in one
// binary64 sum.  The absolute error is a small multiple of
// u^2 (|x| + |a1 b1| + |a2 b2|): the backward error of a double-double rank-2
// update, which is what the Schur-complement analysis needs (the final
// FastTwoSum may round once more when the leading sum cancels completely, an
// error of the same order).
DD_FN dd dd_sub_dot2(dd x, dd a1, dd b1, dd a2, dd b2) {
    const double p1 = a1.hi * b1.hi;
    double c1 = fma(a1.hi, b1.hi, -p1);
    c1 = fma(a1.hi, b1.lo, c1);
    c1 = fma(a1.lo, b1.hi, c1);
    const double p2 = a2.hi * b2.hi;
    double c2 = fma(a2.hi, b2.hi, -p2);
    c2 = fma(a2.hi, b2.lo, c2);
    c2 = fma(a2.lo, b2.hi, c2);
    double s, t1, t2;
    two_sum(x.hi, -p1, s, t1);
    two_sum(s, -p2, s, t2);
    const double low = ((x.lo + t1) + t2) - (c1 + c2);
    dd r;
    fast_two_sum(s, low, r.hi, r.lo);
    return r;
}

// x - a*b, the one-term form of dd_sub_dot2 (same error behaviour).
DD_FN dd dd_sub_mul1(dd x, dd a, dd b) {
    const double p = a.hi * b.hi;
    double c = fma(a.hi, b.hi, -p);
    c = fma(a.hi, b.lo, c);
    c = fma(a.lo, b.hi, c);
    double s, t;
    two_sum(x.hi, -p, s, t);
    const double low = (x.lo + t) - c;
    dd r;
    fast_two_sum(s, low, r.hi, r.lo);
    return r;
}

// a*c - b*b (determinant of a symmetric 2x2 block [[a, b], [b, c]]).
DD_FN dd dd_det2(dd a, dd b, dd c) {
    double p1, e1, p2, e2;
    two_prod(a.hi, c.hi, p1, e1);
    two_prod(b.hi, b.hi, p2, e2);
    double c1 = fma(a.hi, c.lo, a.lo * c.hi);
    double c2 = 2.0 * (b.hi * b.lo);
    double s, t;
    two_sum(p1, -p2, s, t);
    double low = (t + e1 + c1) - (e2 + c2);
    dd r;
    two_sum(s, low, r.hi, r.lo);
    return r;
}

// Binary64 reciprocal square root accurate to about one ulp for positive
// normal x: the hardware estimate (v_rsq_f64 on the device) refined by two
// Newton steps y <- y + y (1 - x y^2) / 2, each of which squares the relative
// error until binary64 rounding dominates.  On the host the estimate is
// 1/sqrt(x).
DD_FN double rsqrt_f64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
    r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
    return y;
#else
    return 1.0 / sqrt(x);
#endif
}

// 1/sqrt(x) for x > 0: a binary64 seed refined by one Newton step
// y = y0 + y0 (1 - x y0^2) / 2 whose residual is formed in double-word
// precision; the seed's relative error e becomes ~1.5 e^2 + O(u^2).
// Non-positive or non-finite x propagates NaN/inf.
DD_FN dd dd_rsqrt(dd x) {
    double y0 = rsqrt_f64(x.hi);
    double p, e;
    two_prod(y0, y0, p, e);           // y0^2 = p + e exactly
    double h, l;
    two_prod(x.hi, p, h, l);
    l = fma(x.hi, e, l);
    l = fma(x.lo, p, l);              // x*y0^2 = h + l (to ~u^2)
    double r = (1.0 - h) - l;         // 1 - h is exact since h ~ 1
    double corr = 0.5 * (y0 * r);
    dd out;
    fast_two_sum(y0, corr, out.hi, out.lo);
    return out;
}

// double-word / double: q1 = a.hi / b, the remainder a - q1 b formed exactly
// with one TwoProd, then one correction (relative error a few u^2).
DD_FN dd dd_div_d(dd a, double b) {
    const double q1 = a.hi / b;
    double p, e;
    two_prod(q1, b, p, e);
    const double r = ((a.hi - p) - e + a.lo) / b;
    dd o;
    fast_two_sum(q1, r, o.hi, o.lo);
    return o;
}

// a + b where |b| is far below |a| (no cancellation possible): one TwoSum of
// the leading words, the trailing words added in binary64 (Dekker's sum).
DD_FN dd dd_add_small(dd a, dd b) {
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    dd r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}

// exp(x) of a double-word x (finite, x.hi < 709).  Reduction x = k ln2 + r,
// |r| <= ln2 / 2, t = r / 32.  The expm1 series a = e^t - 1 = sum_{j>=1} t^j/j!
// is evaluated by Horner: the terms j >= 8 (below 5e-19 relative) in
// binary64, j <= 7 in double-word with |t s| far below each 1/j! (so the
// cheaper sum suffices); truncation after j = 12 is below 1e-33 relative.
// Five doublings e^{2t} - 1 = a (2 + a) keep a's relative precision, then
// exp(x) = 2^k (1 + a).  Relative error within 4 max(1, |x|) 2^-106 (about
// the conditioning of exp on a double-word argument) for results above 1e-290;
// below that the trailing word is subnormal.  Returns 0 below exp(-745).
DD_FN dd dd_exp(dd x) {
    if (x.hi < -745.0) return dd_from(0.0);
    const dd ln2 = dd_make(6.93147180559945286227e-01, 2.31904681384629955842e-17);
    const double k = rint(x.hi / ln2.hi);
    dd t = dd_add(x, dd_neg(dd_mul_d(ln2, k)));
    t = dd_make(t.hi * 0.03125, t.lo * 0.03125);
    // 1/j! for j = 2..7 as double-words
    const double ch[6] = {0.5, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
                          0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13};
    const double cl[6] = {0.0, 0x1.5555555555555p-57, 0x1.5555555555555p-59, 0x1.1111111111111p-63,
                          -0x1.f49f49f49f49fp-65, 0x1.a01a01a01a01ap-73};
    double p = 0x1.1eed8eff8d898p-29;       // 1/12!
    p = fma(p, t.hi, 0x1.ae64567f544e4p-26);  // 1/11!
    p = fma(p, t.hi, 0x1.27e4fb7789f5cp-22);  // 1/10!
    p = fma(p, t.hi, 0x1.71de3a556c734p-19);  // 1/9!
    p = fma(p, t.hi, 0x1.a01a01a01a01ap-16);  // 1/8!
    dd s = dd_from(p);
    for (int j = 5; j >= 0; --j) s = dd_add_small(dd_make(ch[j], cl[j]), dd_mul(t, s));
    s = dd_add_small(dd_from(1.0), dd_mul(t, s));
    dd a = dd_mul(t, s);
    for (int i = 0; i < 5; ++i) a = dd_mul(a, dd_add_small(dd_from(2.0), a));
    a = dd_add_small(dd_from(1.0), a);
    const int ik = (int)k;
    return dd_make(ldexp(a.hi, ik), ldexp(a.lo, ik));
}

// binary64 helpers with the same call shape, for the binary64-term tier
DD_FN double sub_dot2(double x, double a1, double b1, double a2, double b2) {
    return fma(-a2, b2, fma(-a1, b1, x));
}
DD_FN dd sub_dot2(dd x, dd a1, dd b1, dd a2, dd b2) { return dd_sub_dot2(x, a1, b1, a2, b2); }
DD_FN double det2(double a, double b, double c) { return fma(a, c, -b * b); }
DD_FN dd det2(dd a, dd b, dd c) { return dd_det2(a, b, c); }
DD_FN double rsqrt_s(double x) { return rsqrt_f64(x); }
DD_FN dd rsqrt_s(dd x) { return dd_rsqrt(x); }
DD_FN double mul_s(double a, double b) { return a * b; }
DD_FN dd mul_s(dd a, dd b) { return dd_mul(a, b); }
DD_FN dd to_dd(double a) { return dd_from(a); }
DD_FN dd to_dd(dd a) { return a; }
// scalar from a dd (hi, lo) pair: binary64 tier rounds to hi + lo
template <class S> DD_FN S from_pair(double h, double l);
template <> DD_FN double from_pair<double>(double h, double l) { return h + l; }
template <> DD_FN dd from_pair<dd>(double h, double l) {
    dd r;
    two_sum(h, l, r.hi, r.lo);
    return r;
}
// T-recursion step: t0 - q * t1 with dd accumulation
DD_FN dd dd_sub_mul(dd t0, double q, dd t1) { return dd_sub_mul1(t0, t1, dd_from(q)); }
DD_FN dd dd_sub_mul(dd t0, dd q, dd t1) { return dd_sub_mul1(t0, t1, q); }
DD_FN double hi_of(double a) { return a; }
DD_FN double hi_of(dd a) { return a.hi; }
DD_FN double exp_s(double x) { return exp(x); }
DD_FN dd exp_s(dd x) { return dd_exp(x); }
DD_FN double add_s(double a, double b) { return a + b; }
DD_FN dd add_s(dd a, dd b) { return dd_add(a, b); }
DD_FN double scale_s(double a, double f) { return a * f; }
DD_FN dd scale_s(dd a, double f) { return dd_make(a.hi * f, a.lo * f); }
