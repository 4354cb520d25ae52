// Double-double arithmetic (a value is hi + lo with |lo| <= ulp(hi)/2, about
// 106 significant bits), host and device.
//
// Built from the error-free transformations of Knuth (TwoSum) and Dekker
// (FastTwoSum; TwoProduct, here with a fused multiply-add).  The elementary
// functions use standard published reductions:
//   sqrt  one Newton step from the double square root (Karp & Markstein);
//   exp   exp(r) = 2^k (1 + s)^(2^m) with s = expm1(r / 2^m) from its Taylor
//         series, squared in the expm1 form s <- 2s + s^2;
//   log   one Newton step y <- y + a exp(-y) - 1 from the double logarithm;
//   atan  argument halving atan(a) = 2 atan(a / (1 + sqrt(1 + a^2))), then
//         the Taylor series; atan(a) = pi/2 - atan(1/a) for a > 1.
// Accuracy is about 1e-30 relative, which the Newell second difference needs:
// it cancels O(r^6) relative at an offset of r cells.
//
// Floating-point contraction is switched off inside every function here
// (TOF_NOCONTRACT opens each body): a product fused into a later sum (the
// device compiler contracts across statements after inlining by default)
// breaks the error-free transformations.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

#define TOF_HD __host__ __device__ inline
#define TOF_NOCONTRACT _Pragma("clang fp contract(off)")

struct dd {
    double hi, lo;
};

TOF_HD dd dd_make(double a) { return dd{a, 0.0}; }

TOF_HD dd two_sum(double a, double b)
{
    TOF_NOCONTRACT
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd{s, e};
}

TOF_HD dd fast_two_sum(double a, double b)   // requires |a| >= |b| or a == 0
{
    TOF_NOCONTRACT
    double s = a + b;
    return dd{s, b - (s - a)};
}

TOF_HD dd two_prod(double a, double b)
{
    TOF_NOCONTRACT
    double p = a * b;
    return dd{p, fma(a, b, -p)};
}

TOF_HD dd dd_add(dd a, dd b)
{
    TOF_NOCONTRACT
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

TOF_HD dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
TOF_HD dd dd_sub(dd a, dd b) { TOF_NOCONTRACT return dd_add(a, dd_neg(b)); }

TOF_HD dd dd_mul(dd a, dd b)
{
    TOF_NOCONTRACT
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

TOF_HD dd dd_mul_d(dd a, double b)
{
    TOF_NOCONTRACT
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}

// exact scaling by a power of two
TOF_HD dd dd_ldexp(dd a, int e) { return dd{ldexp(a.hi, e), ldexp(a.lo, e)}; }

TOF_HD dd dd_div(dd a, dd b)
{
    TOF_NOCONTRACT
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd_make(q3));
}

TOF_HD dd dd_div_d(dd a, double b) { return dd_div(a, dd_make(b)); }

TOF_HD bool dd_is_zero(dd a) { return a.hi == 0.0; }

TOF_HD dd dd_sqrt(dd a)
{
    TOF_NOCONTRACT
    if (a.hi <= 0.0) return dd_make(0.0);
    double s = sqrt(a.hi);
    dd r = dd_sub(a, two_prod(s, s));
    return fast_two_sum(s, r.hi / (2.0 * s));
}

// ln 2, pi/2 as double-double (hi, lo)
#define TOF_DD_LN2 dd{0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56}
#define TOF_DD_PI_2 dd{0x1.921fb54442d18p+0, 0x1.1a62633145c07p-54}
#define TOF_DD_PI dd{0x1.921fb54442d18p+1, 0x1.1a62633145c07p-53}

TOF_HD dd dd_exp(dd a)
{
    TOF_NOCONTRACT
    const int m = 6;                       // r / 2^6 keeps |r'| <= 0.0055
    double k = rint(a.hi / TOF_DD_LN2.hi);
    dd r = dd_sub(a, dd_mul_d(TOF_DD_LN2, k));
    r = dd_ldexp(r, -m);
    // s = expm1(r) = r + r^2/2! + ... ; 14 terms reach 1e-40 relative
    dd term = r;
    dd s = r;
    for (int i = 2; i <= 14; ++i) {
        term = dd_div_d(dd_mul(term, r), (double)i);
        s = dd_add(s, term);
    }
    for (int i = 0; i < m; ++i) s = dd_add(dd_mul_d(s, 2.0), dd_mul(s, s));
    dd e = dd_add(dd_make(1.0), s);
    return dd_ldexp(e, (int)k);
}

TOF_HD dd dd_log(dd a)   // a > 0
{
    TOF_NOCONTRACT
    dd y = dd_make(log(a.hi));
    // y <- y + a exp(-y) - 1
    dd t = dd_mul(a, dd_exp(dd_neg(y)));
    return dd_add(y, dd_sub(t, dd_make(1.0)));
}

// asinh(t) for t >= 0
TOF_HD dd dd_asinh(dd t)
{
    TOF_NOCONTRACT
    if (dd_is_zero(t)) return dd_make(0.0);
    dd r = dd_sqrt(dd_add(dd_mul(t, t), dd_make(1.0)));
    return dd_log(dd_add(t, r));
}

// atan(a) for a >= 0
TOF_HD dd dd_atan(dd a)
{
    TOF_NOCONTRACT
    if (dd_is_zero(a)) return dd_make(0.0);
    bool inv = a.hi > 1.0;
    if (inv) a = dd_div(dd_make(1.0), a);
    // three halvings: a <= tan(pi/32) ~ 0.0985
    for (int i = 0; i < 3; ++i) {
        dd den = dd_add(dd_make(1.0), dd_sqrt(dd_add(dd_make(1.0), dd_mul(a, a))));
        a = dd_div(a, den);
    }
    dd a2 = dd_mul(a, a);
    dd term = a;
    dd s = a;
    for (int k = 1; k <= 17; ++k) {
        term = dd_neg(dd_mul(term, a2));
        s = dd_add(s, dd_div_d(term, (double)(2 * k + 1)));
    }
    s = dd_ldexp(s, 3);
    if (inv) s = dd_sub(TOF_DD_PI_2, s);
    return s;
}

// ---------------------------------------------------------------------------
// Newell, Williams & Dunlop (1993) auxiliary functions for the cell-averaged
// field of a uniformly magnetized cuboid (the closed form of the sixfold
// integral of eq. (demag_tensor)).  f is even in each argument; g is odd in
// its first two arguments and even in the third.  A term whose polynomial
// prefactor vanishes is dropped (its limit is zero).

TOF_HD dd dd_abs(dd a) { return a.hi < 0.0 ? dd_neg(a) : a; }

TOF_HD dd newell_f_dd(dd x, dd y, dd z)
{
    TOF_NOCONTRACT
    x = dd_abs(x);
    y = dd_abs(y);
    z = dd_abs(z);
    dd x2 = dd_mul(x, x), y2 = dd_mul(y, y), z2 = dd_mul(z, z);
    dd R = dd_sqrt(dd_add(dd_add(x2, y2), z2));
    dd r = dd_make(0.0);
    dd c = dd_mul(dd_ldexp(y, -1), dd_sub(z2, x2));
    if (!dd_is_zero(c)) r = dd_add(r, dd_mul(c, dd_asinh(dd_div(y, dd_sqrt(dd_add(x2, z2))))));
    c = dd_mul(dd_ldexp(z, -1), dd_sub(y2, x2));
    if (!dd_is_zero(c)) r = dd_add(r, dd_mul(c, dd_asinh(dd_div(z, dd_sqrt(dd_add(x2, y2))))));
    c = dd_mul(dd_mul(x, y), z);
    if (!dd_is_zero(c)) r = dd_sub(r, dd_mul(c, dd_atan(dd_div(dd_mul(y, z), dd_mul(x, R)))));
    dd poly = dd_sub(dd_sub(dd_mul_d(x2, 2.0), y2), z2);
    r = dd_add(r, dd_div_d(dd_mul(poly, R), 6.0));
    return r;
}

TOF_HD dd newell_g_dd(dd x, dd y, dd z)
{
    TOF_NOCONTRACT
    bool neg = false;
    if (x.hi < 0.0) { x = dd_neg(x); neg = !neg; }
    if (y.hi < 0.0) { y = dd_neg(y); neg = !neg; }
    z = dd_abs(z);
    dd x2 = dd_mul(x, x), y2 = dd_mul(y, y), z2 = dd_mul(z, z);
    dd R = dd_sqrt(dd_add(dd_add(x2, y2), z2));
    dd r = dd_make(0.0);
    dd c = dd_mul(dd_mul(x, y), z);
    if (!dd_is_zero(c)) r = dd_add(r, dd_mul(c, dd_asinh(dd_div(z, dd_sqrt(dd_add(x2, y2))))));
    c = dd_div_d(dd_mul(y, dd_sub(dd_mul_d(z2, 3.0), y2)), 6.0);
    if (!dd_is_zero(c)) r = dd_add(r, dd_mul(c, dd_asinh(dd_div(x, dd_sqrt(dd_add(y2, z2))))));
    c = dd_div_d(dd_mul(x, dd_sub(dd_mul_d(z2, 3.0), x2)), 6.0);
    if (!dd_is_zero(c)) r = dd_add(r, dd_mul(c, dd_asinh(dd_div(y, dd_sqrt(dd_add(x2, z2))))));
    c = dd_div_d(dd_mul(z, z2), 6.0);
    if (!dd_is_zero(c)) r = dd_sub(r, dd_mul(c, dd_atan(dd_div(dd_mul(x, y), dd_mul(z, R)))));
    c = dd_ldexp(dd_mul(z, y2), -1);
    if (!dd_is_zero(c)) r = dd_sub(r, dd_mul(c, dd_atan(dd_div(dd_mul(x, z), dd_mul(y, R)))));
    c = dd_ldexp(dd_mul(z, x2), -1);
    if (!dd_is_zero(c)) r = dd_sub(r, dd_mul(c, dd_atan(dd_div(dd_mul(y, z), dd_mul(x, R)))));
    r = dd_sub(r, dd_div_d(dd_mul(dd_mul(x, y), R), 3.0));
    return neg ? dd_neg(r) : r;
}

// Auxiliary function of tensor component c (xx, yy, zz, xy, xz, yz) at the
// lattice point (X, Y, Z): the diagonal permutes f's arguments, the
// off-diagonal g's.
TOF_HD dd newell_component_dd(int c, dd X, dd Y, dd Z)
{
    TOF_NOCONTRACT
    switch (c) {
    case 0: return newell_f_dd(X, Y, Z);
    case 1: return newell_f_dd(Y, X, Z);
    case 2: return newell_f_dd(Z, Y, X);
    case 3: return newell_g_dd(X, Y, Z);
    case 4: return newell_g_dd(X, Z, Y);
    default: return newell_g_dd(Y, Z, X);
    }
}

// Parity of component c along each axis (true = odd).
TOF_HD bool comp_odd_x(int c) { return c == 3 || c == 4; }
TOF_HD bool comp_odd_y(int c) { return c == 3 || c == 5; }
TOF_HD bool comp_odd_z(int c) { return c == 4 || c == 5; }

// 1 / (4 pi V) in double-double, V = dx dy dz
TOF_HD dd inv_4pi_volume(double dx, double dy, double dz)
{
    TOF_NOCONTRACT
    dd V = dd_mul_d(two_prod(dx, dy), dz);
    dd den = dd_mul(dd_ldexp(TOF_DD_PI, 2), V);
    return dd_div(dd_make(1.0), den);
}
