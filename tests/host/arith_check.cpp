// Host build of the double-double and quad-double exp and the quad-double arithmetic used by
// the GPU kernels (the same headers), driven by tests/test_arith_host.py:
// prints operands and results as hex floats for an mpmath comparison.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "qd.hpp"

static uint64_t g_state = 0x9e3779b97f4a7c15ULL;
static double urand() {
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}
static qd rand_qd(double scale) {
    const double s = (urand() < 0.5 ? -1.0 : 1.0) * scale * (0.5 + urand());
    double w = s, parts[3];
    for (int i = 0; i < 3; i++) {
        w *= 1.1102230246251565e-16 * (urand() - 0.5);
        parts[i] = w;
    }
    return qd_renorm5(s, parts[0], parts[1], parts[2], 0.0);
}
static void put(qd a) { printf(" %a %a %a %a", a.x0, a.x1, a.x2, a.x3); }

int main(int argc, char **argv) {
    const int n = argc > 1 ? atoi(argv[1]) : 3000;
    for (int i = 0; i < n; i++) {
        const int kind = i % 10;
        qd a = rand_qd(ldexp(1.0, (int)(urand() * 40) - 20)), b = rand_qd(ldexp(1.0, (int)(urand() * 40) - 20));
        if (kind == 1) {  // b = -a perturbed at one level: heavy cancellation
            b = qd_neg(a);
            double *w = &b.x0;
            w[(int)(urand() * 4)] *= 1.0 + 1e-3 * (urand() - 0.5);
            b = qd_renorm5(b.x0, b.x1, b.x2, b.x3, 0.0);
        }
        printf("%d", kind);
        switch (kind) {
        case 0: case 1: put(a); put(b); put(qd_add(a, b)); break;
        case 2: put(a); put(b); put(qd_mul(a, b)); break;
        case 3: {
            const qd x = qd_add(qd_mul(a, a), qd_from(1e-3));
            put(x); put(qd_rsqrt(x));
            break;
        }
        case 4: { const qd c = rand_qd(1.0); put(c); put(a); put(b); put(qd_sub_dot2(c, a, b, b, a)); break; }
        case 5: {
            double x = i == 5 ? 0.0 : -urand() * (i % 3 == 0 ? 0.5 : 60.0);
            double lo = (urand() - 0.5) * 1e-16 * fabs(x), s, e;
            two_sum(x, lo, s, e);
            const dd r = dd_exp(dd_make(s, e));
            printf(" %a %a %a %a", s, e, r.hi, r.lo);
            break;
        }
        case 6: { const dd r = qd_to_dd(a); put(a); printf(" %a %a", r.hi, r.lo); break; }
        case 7: { const qd c = rand_qd(1.0); put(a); put(b); put(c); put(qd_det2(a, b, c)); break; }
        case 8: { const qd c = rand_qd(1.0); put(c); put(a); put(b); put(qd_sub_mul(c, a, b)); break; }
        case 9: {  // quad-double exp on [-60, 5] (both signs of the tree's exponents), and exp(0)
            const double x0 = i == 9 ? 0.0 : (i % 4 == 0 ? urand() * 5.0 : -urand() * (i % 3 == 0 ? 0.5 : 60.0));
            const qd x = x0 == 0.0 ? qd_from(0.0) : rand_qd(1.0).x0 > 0 ? qd_renorm5(x0, x0 * 1e-17 * urand(),
                                                                                    x0 * 1e-34 * urand(), 0.0, 0.0)
                                                                        : qd_from(x0);
            put(x);
            put(qd_exp(x));
            break;
        }
        }
        printf("\n");
    }
    return 0;
}
