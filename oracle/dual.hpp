// Oracle (test infrastructure only): forward-mode dual numbers.
//
// A dual number carries a value and one directional derivative; every
// arithmetic operation applies the ordinary differentiation rules, so running
// a function on duals seeded with a direction w gives f(x) and J(x) w exactly
// (up to rounding).  Used for the Jacobian-vector product of the right-hand
// side, from which the oracle's reference gradients are assembled.
#pragma once
#include <cmath>

struct dual {
  double v, d;
  dual() : v(0), d(0) {}
  dual(double x) : v(x), d(0) {}
  dual(double x, double dx) : v(x), d(dx) {}
};

inline dual operator+(dual a, dual b) { return dual(a.v + b.v, a.d + b.d); }
inline dual operator-(dual a, dual b) { return dual(a.v - b.v, a.d - b.d); }
inline dual operator-(dual a) { return dual(-a.v, -a.d); }
inline dual operator*(dual a, dual b) { return dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline dual operator/(dual a, dual b) {
  double q = a.v / b.v;
  return dual(q, (a.d - q * b.d) / b.v);
}
inline dual operator+(dual a, double b) { return dual(a.v + b, a.d); }
inline dual operator+(double a, dual b) { return dual(a + b.v, b.d); }
inline dual operator-(dual a, double b) { return dual(a.v - b, a.d); }
inline dual operator-(double a, dual b) { return dual(a - b.v, -b.d); }
inline dual operator*(dual a, double b) { return dual(a.v * b, a.d * b); }
inline dual operator*(double a, dual b) { return dual(a * b.v, a * b.d); }
inline dual operator/(dual a, double b) { return dual(a.v / b, a.d / b); }
inline dual operator/(double a, dual b) {
  double q = a / b.v;
  return dual(q, -q * b.d / b.v);
}
inline dual& operator+=(dual& a, dual b) { a = a + b; return a; }
inline dual& operator-=(dual& a, dual b) { a = a - b; return a; }
inline dual& operator*=(dual& a, dual b) { a = a * b; return a; }
inline dual exp(dual a) { double e = std::exp(a.v); return dual(e, e * a.d); }
inline dual log(dual a) { return dual(std::log(a.v), a.d / a.v); }
inline dual pow(dual a, double c) {
  double p = std::pow(a.v, c);
  return dual(p, c * p / a.v * a.d);
}
inline double val(dual a) { return a.v; }
inline double val(double a) { return a; }
