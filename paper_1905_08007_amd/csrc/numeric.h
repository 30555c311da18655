// Number types of the integrand evaluator: plain double, double with a
// running magnitude (for the error bound), and double-double.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define QA_HD __host__ __device__ __forceinline__

// ---- value + magnitude: every operation also propagates |.| so that the
// final magnitude bounds the rounding error of the value (a priori bound).
struct EB {
    double v, a;
};
QA_HD EB eb(double x) { return EB{x, fabs(x)}; }
QA_HD EB operator+(EB x, EB y) { return EB{x.v + y.v, x.a + y.a}; }
QA_HD EB operator-(EB x, EB y) { return EB{x.v - y.v, x.a + y.a}; }
QA_HD EB operator*(EB x, EB y) { return EB{x.v * y.v, x.a * y.a}; }
QA_HD EB operator*(EB x, double c) { return EB{x.v * c, x.a * fabs(c)}; }
QA_HD EB& operator+=(EB& x, EB y) { x = x + y; return x; }
QA_HD EB& operator*=(EB& x, EB y) { x = x * y; return x; }
QA_HD EB operator/(EB x, EB y) { return EB{x.v / y.v, x.a / fabs(y.v)}; }
QA_HD EB operator-(EB x) { return EB{-x.v, x.a}; }
QA_HD EB fma_(EB a, EB b, EB c) { return EB{fma(a.v, b.v, c.v), a.a * b.a + c.a}; }
QA_HD double val(EB x) { return x.v; }
QA_HD double mag(EB x) { return x.a; }

// ---- value + rounding-error variance estimate.  q estimates the variance of
// the accumulated rounding error in units of u^2 under the probabilistic
// model of rounding (each operation's relative error an independent,
// zero-mean variable bounded by u; Higham and Mary, SIAM J. Sci. Comput. 41
// (2019) A2815), propagated to first order: each operation adds the square
// of its own result (its rounding) to the propagated terms.
struct ER {
    double v, q;
};
QA_HD ER operator+(ER x, ER y) {
    const double v = x.v + y.v;
    return ER{v, x.q + y.q + v * v};
}
QA_HD ER operator-(ER x, ER y) {
    const double v = x.v - y.v;
    return ER{v, x.q + y.q + v * v};
}
QA_HD ER operator*(ER x, ER y) {
    const double v = x.v * y.v;
    return ER{v, x.q * (y.v * y.v) + y.q * (x.v * x.v) + v * v};
}
QA_HD ER operator*(ER x, double c) {
    const double v = x.v * c;
    return ER{v, x.q * (c * c) + v * v};
}
QA_HD ER operator/(ER x, ER y) {
    const double v = x.v / y.v;
    return ER{v, (x.q + y.q * (v * v)) / (y.v * y.v) + v * v};
}
QA_HD ER operator-(ER x) { return ER{-x.v, x.q}; }
QA_HD double val(ER x) { return x.v; }

QA_HD double fma_(double a, double b, double c) { return fma(a, b, c); }
QA_HD double val(double x) { return x; }
QA_HD double mag(double x) { return fabs(x); }

// ---- double-double (Dekker / Knuth error-free transformations).  Floating
// point contraction is switched off inside these primitives: fusing the
// product of two_prod into the next addition would break the error-free
// transformations.
struct DD {
    double hi, lo;
};
QA_HD DD two_sum(double a, double b) {
#pragma clang fp contract(off)

    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return DD{s, e};
}
QA_HD DD quick_two_sum(double a, double b) {
#pragma clang fp contract(off)

    double s = a + b;
    double e = b - (s - a);
    return DD{s, e};
}
QA_HD DD two_prod(double a, double b) {
#pragma clang fp contract(off)

    double p = a * b;
    double e = fma(a, b, -p);
    return DD{p, e};
}
// double-double plus double (accurate: two_sum of the high parts)
QA_HD DD add_d(DD a, double b) {
#pragma clang fp contract(off)

    DD s = two_sum(a.hi, b);
    s.lo += a.lo;
    return quick_two_sum(s.hi, s.lo);
}
QA_HD DD dd(double x) {
#pragma clang fp contract(off)
 return DD{x, 0.0}; }
QA_HD DD operator+(DD a, DD b) {
#pragma clang fp contract(off)

    DD s = two_sum(a.hi, b.hi);
    DD t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
QA_HD DD operator-(DD a) {
#pragma clang fp contract(off)
 return DD{-a.hi, -a.lo}; }
QA_HD DD operator-(DD a, DD b) {
#pragma clang fp contract(off)
 return a + (-b); }
QA_HD DD operator*(DD a, DD b) {
#pragma clang fp contract(off)

    DD p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
QA_HD DD operator*(DD a, double c) {
#pragma clang fp contract(off)

    DD p = two_prod(a.hi, c);
    p.lo += a.lo * c;
    return quick_two_sum(p.hi, p.lo);
}
QA_HD DD operator/(DD a, DD b) {
#pragma clang fp contract(off)

    double q1 = a.hi / b.hi;
    DD r = a - b * q1;
    double q2 = r.hi / b.hi;
    r = r - b * q2;
    double q3 = r.hi / b.hi;
    DD q = quick_two_sum(q1, q2);
    return q + dd(q3);
}
QA_HD DD& operator+=(DD& x, DD y) {
#pragma clang fp contract(off)
 x = x + y; return x; }
QA_HD DD& operator*=(DD& x, DD y) {
#pragma clang fp contract(off)
 x = x * y; return x; }
QA_HD DD fma_(DD a, DD b, DD c) {
#pragma clang fp contract(off)
 return a * b + c; }
QA_HD double val(DD x) {
#pragma clang fp contract(off)
 return x.hi + x.lo; }
QA_HD double mag(DD x) {
#pragma clang fp contract(off)
 return fabs(x.hi); }
QA_HD DD sqrt_(DD a) {
#pragma clang fp contract(off)

    double x = sqrt(a.hi);
    DD r = a - two_prod(x, x);
    return quick_two_sum(x, r.hi / (2.0 * x));
}
QA_HD double sqrt_(double a) {
#pragma clang fp contract(off)
 return sqrt(a); }
QA_HD DD operator/(DD a, double b) {
#pragma clang fp contract(off)
 return a / dd(b); }

QA_HD DD operator/(DD a, int b) {
#pragma clang fp contract(off)
 return a / dd((double)b); }
QA_HD double to_d(DD x) {
#pragma clang fp contract(off)
 return x.hi + x.lo; }

template <class T> QA_HD T from_d(double x);
// storage type of the geometry variables for an evaluation type (the
// geometry itself is always computed in double-double), and the lift
template <class T> struct GeoOf { using type = double; };
template <> struct GeoOf<DD> { using type = DD; };
QA_HD void store_geo(double& dst, DD x) { dst = x.hi + x.lo; }
QA_HD void store_geo(DD& dst, DD x) { dst = x; }

// block accumulators: plain, value in double-double with magnitude, double-double
template <class T> struct Acc { using type = T; };
struct EBAcc {
    DD v;
    double a;
};
template <> struct Acc<EB> { using type = EBAcc; };
// ER tables accumulate EQ blocks: the value in double-double, and
// nb * q_block, nb the number of roundings on any path through the block, each
// contributing at most u times a monomial
struct ERAcc {
    DD v;
    double q;
};
template <> struct Acc<ER> { using type = ERAcc; };
// A block of an ER evaluation: its value v and q >= the sum of the squares of
// its monomials (coefficient times the product of its geometry values).
struct EQ {
    double v, q;
};
template <class T> struct BlockOf { using type = T; };
template <> struct BlockOf<ER> { using type = EQ; };
QA_HD double acc_zero(double*) { return 0.0; }
QA_HD EBAcc acc_zero(EBAcc*) { return EBAcc{DD{0.0, 0.0}, 0.0}; }
QA_HD DD acc_zero(DD*) { return DD{0.0, 0.0}; }
QA_HD ERAcc acc_zero(ERAcc*) { return ERAcc{DD{0.0, 0.0}, 0.0}; }
QA_HD void acc_add(double& s, double x) { s += x; }
QA_HD void acc_add(EBAcc& s, EB x) {
#pragma clang fp contract(off)
    s.v = add_d(s.v, x.v);
    s.a += x.a;
}
QA_HD void acc_add(DD& s, DD x) { s = s + x; }
QA_HD void acc_add(double& s, double x, int) { s += x; }
QA_HD void acc_add(DD& s, DD x, int) { s = s + x; }
QA_HD void acc_add(EBAcc& s, EB x, int) { acc_add(s, x); }
QA_HD void acc_add(ERAcc& s, EQ x, int nb) {
#pragma clang fp contract(off)
    s.v = add_d(s.v, x.v);
    s.q += (double)nb * x.q;
}
QA_HD double acc_get(double s) { return s; }
QA_HD EB acc_get(EBAcc s) { return EB{s.v.hi + s.v.lo, s.a}; }
QA_HD DD acc_get(DD s) { return s; }
QA_HD ER acc_get(ERAcc s) {
    const double v = s.v.hi + s.v.lo;
    return ER{v, s.q + v * v};
}
// division by the exact integer denominator of a table
QA_HD double div_den(double x, double d) { return x / d; }
QA_HD EB div_den(EB x, double d) { return EB{x.v / d, x.a / d}; }
QA_HD DD div_den(DD x, double d) { return x / dd(d); }
QA_HD ER div_den(ER x, double d) {
    const double v = x.v / d;
    return ER{v, x.q / (d * d) + v * v};
}
QA_HD double lift(double x, double*) { return x; }
QA_HD EB lift(double x, EB*) { return EB{x, fabs(x)}; }
QA_HD DD lift(DD x, DD*) { return x; }
// a geometry value rounded from double-double to double: one rounding
QA_HD ER lift(double x, ER*) { return ER{x, x * x}; }
template <class T, class S> QA_HD T lift_to(S x) { return lift(x, (T*)nullptr); }
template <> QA_HD double from_d<double>(double x) { return x; }
template <> QA_HD EB from_d<EB>(double x) { return eb(x); }
template <> QA_HD DD from_d<DD>(double x) { return dd(x); }
template <> QA_HD ER from_d<ER>(double x) { return ER{x, 0.0}; }
