/*
 * or_dual.h -- first-order dual numbers for the tangent build of the CPU
 * oracle (TEST INFRASTRUCTURE ONLY).
 *
 * A dual number carries a value v and a derivative d along one direction.
 * Each operation computes its value with the very same IEEE double operation
 * the plain oracle performs (so the value parts, and every comparison made on
 * them, are bit-for-bit those of the plain oracle) and its derivative by the
 * chain rule of that operation.  Comparisons look at values only, so the
 * derivative is the one of the branch actually taken.  |x| uses sign +1 at
 * x = 0.
 */
#pragma once
#include <math.h>

struct or_dual {
  double v, d;
  or_dual() = default;
  or_dual(double x) : v(x), d(0.0) {}
  or_dual(double x, double y) : v(x), d(y) {}
};

static inline or_dual operator+(or_dual a, or_dual b) { return or_dual(a.v + b.v, a.d + b.d); }
static inline or_dual operator-(or_dual a, or_dual b) { return or_dual(a.v - b.v, a.d - b.d); }
static inline or_dual operator-(or_dual a) { return or_dual(-a.v, -a.d); }
static inline or_dual operator*(or_dual a, or_dual b) {
  return or_dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
static inline or_dual operator/(or_dual a, or_dual b) {
  double q = a.v / b.v;
  return or_dual(q, (a.d - q * b.d) / b.v);
}
static inline or_dual &operator+=(or_dual &a, or_dual b) { return a = a + b; }
static inline or_dual &operator-=(or_dual &a, or_dual b) { return a = a - b; }
static inline or_dual &operator*=(or_dual &a, or_dual b) { return a = a * b; }
static inline or_dual &operator/=(or_dual &a, or_dual b) { return a = a / b; }

static inline bool operator<(or_dual a, or_dual b) { return a.v < b.v; }
static inline bool operator>(or_dual a, or_dual b) { return a.v > b.v; }
static inline bool operator<=(or_dual a, or_dual b) { return a.v <= b.v; }
static inline bool operator>=(or_dual a, or_dual b) { return a.v >= b.v; }
static inline bool operator==(or_dual a, or_dual b) { return a.v == b.v; }
static inline bool operator!=(or_dual a, or_dual b) { return a.v != b.v; }
static inline bool operator!(or_dual a) { return !a.v; }

static inline or_dual sqrt(or_dual a) {
  double r = sqrt(a.v);
  return or_dual(r, a.d / (2.0 * r));
}
static inline or_dual fabs(or_dual a) { return a.v < 0.0 ? -a : a; }
static inline bool isfinite(or_dual a) { return isfinite(a.v); }
