// Forward-mode dual numbers for the oracle (test infrastructure only).
//
// Dual<N> carries a value and N tangent components.  Every operator applies
// the textbook chain rule; comparisons and min/max act on the value only, so
// a branch is always taken from the primal value, exactly as in the
// double-precision oracle.  Instantiating the templated solver with Dual<N>
// yields the exact derivative of the discrete map with respect to any N
// seeded inputs (state components, gamma, Mach number).
#pragma once
#include <cmath>

namespace orc {

template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0.0; }  // NOLINT
};

template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v + b.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v - b.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r(-a.v); for (int k = 0; k < N; ++k) r.d[k] = -a.d[k]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v * b.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v / b.v);
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

template <int N> inline bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N> inline bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N> inline bool operator<=(const Dual<N>& a, const Dual<N>& b) { return a.v <= b.v; }
template <int N> inline bool operator>=(const Dual<N>& a, const Dual<N>& b) { return a.v >= b.v; }
template <int N> inline bool operator<(const Dual<N>& a, double b) { return a.v < b; }
template <int N> inline bool operator>(const Dual<N>& a, double b) { return a.v > b; }
template <int N> inline bool operator<=(const Dual<N>& a, double b) { return a.v <= b; }
template <int N> inline bool operator>=(const Dual<N>& a, double b) { return a.v >= b; }

template <int N> inline Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r(std::sqrt(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r; }
template <int N> inline Dual<N> fabs(const Dual<N>& a) { return a.v < 0.0 ? -a : a; }
template <int N> inline Dual<N> tanh(const Dual<N>& a) {
  double t = std::tanh(a.v); Dual<N> r(t);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * (1.0 - t * t);
  return r; }

// value() gives the primal part of a scalar of either kind.
inline double value(double x) { return x; }
template <int N> inline double value(const Dual<N>& x) { return x.v; }

}  // namespace orc
