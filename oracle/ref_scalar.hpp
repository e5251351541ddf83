// Oracle scalar types. TEST INFRASTRUCTURE ONLY: nothing in the product path
// may include, link or execute anything under oracle/.
//
// The simulator templates are instantiated with `double` (the FP64 reference)
// and with `Cnt`, a double that tallies every arithmetic operation it performs.
// Running one rollout with `Cnt` gives the algorithmic operation count of the
// method per environment step: +, -, * count 1, fma 2, / and sqrt 1, and the
// transcendental calls are tallied on their own.  Compares and selects are free.
#pragma once
#include <cmath>
#include <cstdint>

namespace ref {

struct Tally {
  uint64_t add = 0, mul = 0, fma = 0, div = 0, sqrt = 0, trans = 0;
  uint64_t flops() const { return add + mul + 2 * fma + div + sqrt; }
};
extern thread_local Tally g_tally;

struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}  // NOLINT: implicit by design, literals promote
  explicit operator double() const { return v; }
  Cnt &operator+=(Cnt o) { ++g_tally.add; v += o.v; return *this; }
  Cnt &operator-=(Cnt o) { ++g_tally.add; v -= o.v; return *this; }
  Cnt &operator*=(Cnt o) { ++g_tally.mul; v *= o.v; return *this; }
  Cnt &operator/=(Cnt o) { ++g_tally.div; v /= o.v; return *this; }
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_tally.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_tally.add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_tally.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_tally.div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator==(Cnt a, Cnt b) { return a.v == b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }

// Math entry points used by the templates; overloads for double and Cnt.
inline double r_sqrt(double x) { return std::sqrt(x); }
inline double r_sin(double x) { return std::sin(x); }
inline double r_cos(double x) { return std::cos(x); }
inline double r_atan2(double y, double x) { return std::atan2(y, x); }
inline double r_abs(double x) { return std::fabs(x); }
inline double r_max(double a, double b) { return a > b ? a : b; }
inline double r_min(double a, double b) { return a < b ? a : b; }
inline bool r_finite(double x) { return std::isfinite(x); }
inline double r_val(double x) { return x; }

inline Cnt r_sqrt(Cnt x) { ++g_tally.sqrt; return Cnt(std::sqrt(x.v)); }
inline Cnt r_sin(Cnt x) { ++g_tally.trans; return Cnt(std::sin(x.v)); }
inline Cnt r_cos(Cnt x) { ++g_tally.trans; return Cnt(std::cos(x.v)); }
inline Cnt r_atan2(Cnt y, Cnt x) { ++g_tally.trans; return Cnt(std::atan2(y.v, x.v)); }
inline Cnt r_abs(Cnt x) { return Cnt(std::fabs(x.v)); }
inline Cnt r_max(Cnt a, Cnt b) { return a.v > b.v ? a : b; }
inline Cnt r_min(Cnt a, Cnt b) { return a.v < b.v ? a : b; }
inline bool r_finite(Cnt x) { return std::isfinite(x.v); }
inline double r_val(Cnt x) { return x.v; }

}  // namespace ref
