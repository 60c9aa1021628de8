// Test infrastructure, not product code.
//
// The oracle (nmc_oracle.c) compiled as C++ with every `double` replaced by a
// counting wrapper, so that the arithmetic the reference algorithm performs
// is tallied operation by operation: additions and subtractions, products,
// quotients, square roots and the transcendental calls (exp, log, pow, cbrt).
// Negation, absolute values, minima, maxima and comparisons are not counted.
// The wrapper has the size, alignment and calling convention of a double, so
// liboracle_tally.so keeps the oracle's C ABI; it adds ora_tally_read and
// ora_tally_reset.  The counters are plain globals: call it from one thread
// (nthreads = 1).  Only tests and the benchmark's CPU-baseline leg load it.
// Built with -fpermissive: the oracle's C allocations return void *.
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace tally {

struct Counts {
  uint64_t add, mul, div, sqrt, trans;
};
Counts g = {0, 0, 0, 0, 0};

struct f64 {
  double v;
  f64() = default;
  constexpr f64(double x) : v(x) {}
  explicit operator double() const { return v; }
  explicit operator int() const { return (int)v; }
  explicit operator long() const { return (long)v; }
  f64& operator+=(f64 o) { ++g.add; v += o.v; return *this; }
  f64& operator-=(f64 o) { ++g.add; v -= o.v; return *this; }
  f64& operator*=(f64 o) { ++g.mul; v *= o.v; return *this; }
  f64& operator/=(f64 o) { ++g.div; v /= o.v; return *this; }
};
static_assert(sizeof(f64) == sizeof(double) && alignof(f64) == alignof(double), "layout of a double");

inline f64 operator+(f64 a, f64 b) { ++g.add; return f64(a.v + b.v); }
inline f64 operator-(f64 a, f64 b) { ++g.add; return f64(a.v - b.v); }
inline f64 operator*(f64 a, f64 b) { ++g.mul; return f64(a.v * b.v); }
inline f64 operator/(f64 a, f64 b) { ++g.div; return f64(a.v / b.v); }
inline f64 operator-(f64 a) { return f64(-a.v); }
inline f64 operator+(f64 a) { return a; }
inline bool operator<(f64 a, f64 b) { return a.v < b.v; }
inline bool operator>(f64 a, f64 b) { return a.v > b.v; }
inline bool operator<=(f64 a, f64 b) { return a.v <= b.v; }
inline bool operator>=(f64 a, f64 b) { return a.v >= b.v; }
inline bool operator==(f64 a, f64 b) { return a.v == b.v; }
inline bool operator!=(f64 a, f64 b) { return a.v != b.v; }

inline f64 sqrt(f64 a) { ++g.sqrt; return f64(std::sqrt(a.v)); }
inline f64 exp(f64 a) { ++g.trans; return f64(std::exp(a.v)); }
inline f64 log(f64 a) { ++g.trans; return f64(std::log(a.v)); }
inline f64 cbrt(f64 a) { ++g.trans; return f64(std::cbrt(a.v)); }
inline f64 pow(f64 a, f64 b) { ++g.trans; return f64(std::pow(a.v, b.v)); }
inline f64 cos(f64 a) { ++g.trans; return f64(std::cos(a.v)); }
inline f64 fabs(f64 a) { return f64(std::fabs(a.v)); }
inline f64 fmin(f64 a, f64 b) { return f64(std::fmin(a.v, b.v)); }
inline f64 fmax(f64 a, f64 b) { return f64(std::fmax(a.v, b.v)); }
inline f64 floor(f64 a) { return f64(std::floor(a.v)); }
inline f64 ceil(f64 a) { return f64(std::ceil(a.v)); }
inline f64 ldexp(f64 a, int e) { return f64(std::ldexp(a.v, e)); }
inline f64 frexp(f64 a, int* e) { return f64(std::frexp(a.v, e)); }
inline bool isfinite(f64 a) { return std::isfinite(a.v); }
inline bool isnan(f64 a) { return std::isnan(a.v); }

}  // namespace tally

using tally::f64;
using tally::sqrt;
using tally::exp;
using tally::log;
using tally::cbrt;
using tally::pow;
using tally::cos;
using tally::frexp;
using tally::fabs;
using tally::fmin;
using tally::fmax;
using tally::floor;
using tally::ceil;
using tally::ldexp;
using tally::isfinite;
using tally::isnan;

#define double f64
#include "nmc_oracle.c"
#undef double

extern "C" {
// counts since the last reset: additions and subtractions, products,
// quotients, square roots, transcendental calls
void ora_tally_read(uint64_t* out) {
  out[0] = tally::g.add;
  out[1] = tally::g.mul;
  out[2] = tally::g.div;
  out[3] = tally::g.sqrt;
  out[4] = tally::g.trans;
}
void ora_tally_reset(void) { tally::g = tally::Counts{0, 0, 0, 0, 0}; }
}
