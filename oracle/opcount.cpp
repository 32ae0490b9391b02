// opcount.cpp -- operation-counting build of the oracle.  TEST INFRASTRUCTURE ONLY.
//
// The oracle's source (gks_oracle.c) is compiled here unchanged, with its FP64 scalar type
// replaced by a number type that counts every floating-point operation by kind: additions
// and subtractions, multiplications, divisions, square roots, exponentials and erfc calls
// (negation, absolute value, min/max and comparisons are not counted).  The type holds one
// double and performs the same IEEE operation in the same order, so the counting build
// computes the oracle's values bitwise (with contraction off in both builds).  It gives the
// oracle's own operation count of a face flux, beside the HIP library's count of its
// closed-form evaluation.
#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

namespace opc {
enum { ADD, MUL, DIV, SQRT, EXP, ERFC, NKIND };
static unsigned long long counts[NKIND];

struct D {
    double v;
    D() = default;
    D(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
    explicit operator long() const { return (long)v; }
    D& operator+=(D b) { ++counts[ADD]; v += b.v; return *this; }
    D& operator-=(D b) { ++counts[ADD]; v -= b.v; return *this; }
    D& operator*=(D b) { ++counts[MUL]; v *= b.v; return *this; }
    D& operator/=(D b) { ++counts[DIV]; v /= b.v; return *this; }
};
inline D operator+(D a, D b) { ++counts[ADD]; return D(a.v + b.v); }
inline D operator-(D a, D b) { ++counts[ADD]; return D(a.v - b.v); }
inline D operator*(D a, D b) { ++counts[MUL]; return D(a.v * b.v); }
inline D operator/(D a, D b) { ++counts[DIV]; return D(a.v / b.v); }
inline D operator-(D a) { return D(-a.v); }
inline D operator+(D a) { return a; }
inline bool operator<(D a, D b) { return a.v < b.v; }
inline bool operator>(D a, D b) { return a.v > b.v; }
inline bool operator<=(D a, D b) { return a.v <= b.v; }
inline bool operator>=(D a, D b) { return a.v >= b.v; }
inline bool operator==(D a, D b) { return a.v == b.v; }
inline bool operator!=(D a, D b) { return a.v != b.v; }
inline D sqrt(D a) { ++counts[SQRT]; return D(::sqrt(a.v)); }
inline D exp(D a) { ++counts[EXP]; return D(::exp(a.v)); }
inline D erfc(D a) { ++counts[ERFC]; return D(::erfc(a.v)); }
inline D fabs(D a) { return D(::fabs(a.v)); }
inline D fmax(D a, D b) { return D(::fmax(a.v, b.v)); }
inline D fmin(D a, D b) { return D(::fmin(a.v, b.v)); }
inline bool isfinite(D a) { return ::isfinite(a.v); }
}  // namespace opc

static_assert(sizeof(opc::D) == sizeof(double), "the counting type has the layout of a double");

// the oracle's OpenMP reductions over its scalar type (the counting build runs one thread)
#pragma omp declare reduction(max : opc::D : omp_out = (omp_in > omp_out ? omp_in : omp_out)) initializer(omp_priv = omp_orig)
#pragma omp declare reduction(+ : opc::D : omp_out += omp_in) initializer(omp_priv = opc::D(0.0))

#define double opc::D
extern "C" {   // the oracle's entry points keep their C names
#include "gks_oracle.c"
}
#undef double

extern "C" {
// counts since the last reset: [add/sub, mul, div, sqrt, exp, erfc]
void og_ops_reset(void) { memset(opc::counts, 0, sizeof(opc::counts)); }
void og_ops_get(unsigned long long* out)
{
    for (int k = 0; k < opc::NKIND; ++k) out[k] = opc::counts[k];
}
}
