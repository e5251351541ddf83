// Oracle scalar types. TEST INFRASTRUCTURE ONLY: nothing in the product path
// may include, link or execute anything under oracle/.
//
// The simulator templates are instantiated with `double` (the FP64 reference)
// and with `Cnt`, a double that tallies the arithmetic operations it performs.
// Running one rollout with `Cnt` gives the algorithmic operation count of the
// method per environment step: +, -, * count 1, fma 2, / and sqrt 1, and the
// transcendental calls are tallied on their own.  Compares and selects are
// free, and so are operations fixed by the problem's structure (see Cnt).
#pragma once
#include <cmath>
#include <cstdint>

namespace ref {

struct Tally {
  uint64_t add = 0, mul = 0, fma = 0, div = 0, sqrt = 0, trans = 0;
  uint64_t flops() const { return add + mul + 2 * fma + div + sqrt; }
};
extern thread_local Tally g_tally;

// `s` marks a structural constant: a value that is exactly 0, 1 or -1 where it
// enters (literals, zero geometry, zero initial rates), or the result of an
// operation on structural constants only.  An operation whose result is fixed
// by structure (on structural operands only, x*0, x*(+-1), x+0, x-0, 0/x,
// x/(+-1)) is not counted: code specialised to the problem's structure
// (axis-aligned joints, zero offsets, the sparsity of the spatial transforms)
// does not perform it.  The value is always computed exactly as with double,
// so a counted rollout follows the FP64 rollout's trajectory.
struct Cnt {
  double v;
  bool s;
  Cnt() : v(0.0), s(true) {}
  Cnt(double x) : v(x), s(x == 0.0 || x == 1.0 || x == -1.0) {}  // NOLINT: implicit by design, literals promote
  explicit operator double() const { return v; }
};
inline Cnt cnt_make(double v, bool s) {
  Cnt c;
  c.v = v;
  c.s = s;
  return c;
}
inline bool cnt_zero(Cnt a) { return a.s && a.v == 0.0; }
inline bool cnt_unit(Cnt a) { return a.s && (a.v == 1.0 || a.v == -1.0); }
inline Cnt operator+(Cnt a, Cnt b) {
  if (a.s && b.s) return cnt_make(a.v + b.v, true);
  if (cnt_zero(a)) return cnt_make(a.v + b.v, b.s);
  if (cnt_zero(b)) return cnt_make(a.v + b.v, a.s);
  ++g_tally.add;
  return cnt_make(a.v + b.v, false);
}
inline Cnt operator-(Cnt a, Cnt b) {
  if (a.s && b.s) return cnt_make(a.v - b.v, true);
  if (cnt_zero(a)) return cnt_make(a.v - b.v, b.s);
  if (cnt_zero(b)) return cnt_make(a.v - b.v, a.s);
  ++g_tally.add;
  return cnt_make(a.v - b.v, false);
}
inline Cnt operator*(Cnt a, Cnt b) {
  if ((a.s && b.s) || cnt_zero(a) || cnt_zero(b)) return cnt_make(a.v * b.v, true);
  if (cnt_unit(a)) return cnt_make(a.v * b.v, b.s);
  if (cnt_unit(b)) return cnt_make(a.v * b.v, a.s);
  ++g_tally.mul;
  return cnt_make(a.v * b.v, false);
}
inline Cnt operator/(Cnt a, Cnt b) {
  if ((a.s && b.s) || cnt_zero(a)) return cnt_make(a.v / b.v, true);
  if (cnt_unit(b)) return cnt_make(a.v / b.v, a.s);
  ++g_tally.div;
  return cnt_make(a.v / b.v, false);
}
inline Cnt operator-(Cnt a) { return cnt_make(-a.v, a.s); }
inline Cnt &operator+=(Cnt &a, Cnt b) { return a = a + b; }
inline Cnt &operator-=(Cnt &a, Cnt b) { return a = a - b; }
inline Cnt &operator*=(Cnt &a, Cnt b) { return a = a * b; }
inline Cnt &operator/=(Cnt &a, Cnt b) { return a = a / b; }
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

inline Cnt r_sqrt(Cnt x) {
  if (!x.s) ++g_tally.sqrt;
  return cnt_make(std::sqrt(x.v), x.s);
}
inline Cnt r_sin(Cnt x) {
  if (!x.s) ++g_tally.trans;
  return cnt_make(std::sin(x.v), x.s);
}
inline Cnt r_cos(Cnt x) {
  if (!x.s) ++g_tally.trans;
  return cnt_make(std::cos(x.v), x.s);
}
inline Cnt r_atan2(Cnt y, Cnt x) {
  if (!(x.s && y.s)) ++g_tally.trans;
  return cnt_make(std::atan2(y.v, x.v), x.s && y.s);
}
inline Cnt r_abs(Cnt x) { return cnt_make(std::fabs(x.v), x.s); }
inline Cnt r_max(Cnt a, Cnt b) { return a.v > b.v ? a : b; }
inline Cnt r_min(Cnt a, Cnt b) { return a.v < b.v ? a : b; }
inline bool r_finite(Cnt x) { return std::isfinite(x.v); }
inline double r_val(Cnt x) { return x.v; }

}  // namespace ref
