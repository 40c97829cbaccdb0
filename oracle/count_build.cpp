// count_build.cpp -- TEST INFRASTRUCTURE ONLY: the oracle (hydro_ref.c,
// included unchanged) compiled as C++ with every floating-point value of
// the method replaced by a type that counts the operations done on it.
// Only the tests and the benchmark's report of the definition's operation
// count load this build.
//
// What counts as one operation (the rule the package's cost model states):
// each +, -, *, /, sqrt, pow, min, max and comparison of two values; the
// absolute value, copysign and negation count 0, and so does the finiteness
// test of the status word (not part of the method's arithmetic).  Constants
// the source spells as an expression of literals (1.0 / 6.0) are folded
// before they become counted values.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace refcount {

unsigned long long g_ops = 0;   // the counting build runs single-threaded

struct cd {
    double v;
    cd() = default;
    cd(double x) : v(x) {}
    explicit operator double() const { return v; }
};

inline cd operator+(cd a, cd b) { ++g_ops; return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { ++g_ops; return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { ++g_ops; return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { ++g_ops; return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }
inline bool operator<(cd a, cd b) { ++g_ops; return a.v < b.v; }
inline bool operator<=(cd a, cd b) { ++g_ops; return a.v <= b.v; }
inline bool operator>(cd a, cd b) { ++g_ops; return a.v > b.v; }
inline bool operator>=(cd a, cd b) { ++g_ops; return a.v >= b.v; }
inline bool operator==(cd a, cd b) { ++g_ops; return a.v == b.v; }
inline bool operator!=(cd a, cd b) { ++g_ops; return a.v != b.v; }

}  // namespace refcount

using refcount::cd;

inline cd fabs(cd a) { return cd(std::fabs(a.v)); }
inline cd copysign(cd a, cd b) { return cd(std::copysign(a.v, b.v)); }
inline cd fmin(cd a, cd b) { ++refcount::g_ops; return cd(std::fmin(a.v, b.v)); }
inline cd fmax(cd a, cd b) { ++refcount::g_ops; return cd(std::fmax(a.v, b.v)); }
inline cd sqrt(cd a) { ++refcount::g_ops; return cd(std::sqrt(a.v)); }
inline cd pow(cd a, cd b) { ++refcount::g_ops; return cd(std::pow(a.v, b.v)); }
#ifdef isfinite
#undef isfinite
#endif
inline bool isfinite(cd a) { return std::isfinite(a.v); }

static_assert(sizeof(cd) == sizeof(double), "the counted value keeps the layout of a double");

extern "C" {
#define double cd
#include "hydro_ref.c"
#undef double

unsigned long long hydro_ref_flops(void) { return refcount::g_ops; }
void hydro_ref_flops_reset(void) { refcount::g_ops = 0; }
}
