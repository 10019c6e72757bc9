// Forward-mode dual numbers v + d*eps (eps^2 = 0) for the serial oracle --
// TEST INFRASTRUCTURE ONLY.
//
// Running the templated oracle on this scalar carries, next to every FP64
// value v, its exact derivative d along one chosen input direction (the chain
// rule applied operation by operation).  The value part is computed with the
// very same double operations as the plain FP64 oracle, so the branches taken
// (clamps, fallbacks, comparisons) are those of the FP64 run; comparisons look
// at the value part only.
#pragma once

#include <cmath>

namespace fsref {

struct Dual {
  double v = 0.0;  // value
  double d = 0.0;  // directional derivative
  Dual() = default;
  Dual(double value) : v(value), d(0.0) {}  // constants carry no derivative
  Dual(double value, double deriv) : v(value), d(deriv) {}
};

inline Dual operator+(const Dual& a, const Dual& b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(const Dual& a, const Dual& b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(const Dual& a) { return {-a.v, -a.d}; }
// (a b)' = a' b + a b'
inline Dual operator*(const Dual& a, const Dual& b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
// (a / b)' = (a' - (a/b) b') / b
inline Dual operator/(const Dual& a, const Dual& b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
// sqrt(a)' = a' / (2 sqrt(a))
inline Dual sqrt(const Dual& a) {
  const double r = std::sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}

inline bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
inline bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
inline bool operator<=(const Dual& a, const Dual& b) { return a.v <= b.v; }
inline bool operator>=(const Dual& a, const Dual& b) { return a.v >= b.v; }
inline bool operator==(const Dual& a, const Dual& b) { return a.v == b.v; }
inline bool operator!=(const Dual& a, const Dual& b) { return a.v != b.v; }

}  // namespace fsref
