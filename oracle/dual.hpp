// Forward-mode dual numbers for the CPU oracle (test infrastructure only).
//
// A Dual carries a value v and one directional derivative d, so evaluating the
// oracle's templated operator on Dual inputs (U, V) yields (F(U), F'(U) V): the
// Jacobian-vector product used to check the GPU adjoint by the dot-product
// identity <w, J v> = <J^T w, v>.
//
// Conventions at non-differentiable points (used identically by the GPU adjoint):
//   |x|  at x == 0   -> derivative 0
//   max(a, b) at a == b -> derivative (a.d + b.d) / 2   (matches central differences)
#pragma once
#include <cmath>

namespace oracle {

struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double y) : v(x), d(y) {}
  Dual& operator+=(const Dual& o) { v += o.v; d += o.d; return *this; }
  Dual& operator-=(const Dual& o) { v -= o.v; d -= o.d; return *this; }
  Dual& operator*=(const Dual& o) { d = d * o.v + v * o.d; v *= o.v; return *this; }
};

inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) {
  const double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}

inline double value(double x) { return x; }
inline double value(const Dual& x) { return x.v; }

inline double sqrt_(double x) { return std::sqrt(x); }
inline Dual sqrt_(Dual x) {
  const double s = std::sqrt(x.v);
  return Dual(s, x.d / (2.0 * s));
}
inline double exp_(double x) { return std::exp(x); }
inline Dual exp_(Dual x) {
  const double e = std::exp(x.v);
  return Dual(e, e * x.d);
}
inline double log_(double x) { return std::log(x); }
inline Dual log_(Dual x) { return Dual(std::log(x.v), x.d / x.v); }

inline double asin_(double x) { return std::asin(x); }
inline Dual asin_(Dual x) { return Dual(std::asin(x.v), x.d / std::sqrt(1.0 - x.v * x.v)); }

inline double abs_(double x) { return std::fabs(x); }
inline Dual abs_(Dual x) {
  if (x.v > 0.0) return x;
  if (x.v < 0.0) return -x;
  return Dual(0.0, 0.0);
}
inline double max_(double a, double b) { return a > b ? a : b; }
inline Dual max_(Dual a, Dual b) {
  if (a.v > b.v) return a;
  if (b.v > a.v) return b;
  return Dual(a.v, 0.5 * (a.d + b.d));
}
inline double min_(double a, double b) { return a < b ? a : b; }
inline Dual min_(Dual a, Dual b) {
  if (a.v < b.v) return a;
  if (b.v < a.v) return b;
  return Dual(a.v, 0.5 * (a.d + b.d));
}

}  // namespace oracle
