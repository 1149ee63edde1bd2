// TEST INFRASTRUCTURE ONLY: a double that counts the floating-point
// operations applied to it, for the oracle's counting build.  Every +, -, *, /
// and sqrt is one flop; fabs, comparisons and min/max cost nothing; sin, cos
// and exp are tallied apart (they appear only in the one-time geometry).
#pragma once

#include <cmath>

struct FlopTally {
  long long add = 0, mul = 0, div = 0, sqrt = 0, trans = 0;
};
extern FlopTally g_flops;

struct CountedReal {
  double v;
  CountedReal() : v(0.0) {}
  CountedReal(double x) : v(x) {}
  explicit operator double() const { return v; }
  CountedReal& operator+=(const CountedReal& o) { g_flops.add++; v += o.v; return *this; }
  CountedReal& operator-=(const CountedReal& o) { g_flops.add++; v -= o.v; return *this; }
  CountedReal& operator*=(const CountedReal& o) { g_flops.mul++; v *= o.v; return *this; }
  CountedReal& operator/=(const CountedReal& o) { g_flops.div++; v /= o.v; return *this; }
};

inline CountedReal operator+(CountedReal a, CountedReal b) { g_flops.add++; return a.v + b.v; }
inline CountedReal operator-(CountedReal a, CountedReal b) { g_flops.add++; return a.v - b.v; }
inline CountedReal operator*(CountedReal a, CountedReal b) { g_flops.mul++; return a.v * b.v; }
inline CountedReal operator/(CountedReal a, CountedReal b) { g_flops.div++; return a.v / b.v; }
inline CountedReal operator-(CountedReal a) { return -a.v; }
inline bool operator<(CountedReal a, CountedReal b) { return a.v < b.v; }
inline bool operator>(CountedReal a, CountedReal b) { return a.v > b.v; }
inline bool operator<=(CountedReal a, CountedReal b) { return a.v <= b.v; }
inline bool operator>=(CountedReal a, CountedReal b) { return a.v >= b.v; }
inline bool operator==(CountedReal a, CountedReal b) { return a.v == b.v; }
inline bool operator!=(CountedReal a, CountedReal b) { return a.v != b.v; }
inline CountedReal sqrt(CountedReal a) { g_flops.sqrt++; return std::sqrt(a.v); }
inline CountedReal fabs(CountedReal a) { return std::fabs(a.v); }
inline CountedReal sin(CountedReal a) { g_flops.trans++; return std::sin(a.v); }
inline CountedReal cos(CountedReal a) { g_flops.trans++; return std::cos(a.v); }
inline CountedReal exp(CountedReal a) { g_flops.trans++; return std::exp(a.v); }
inline bool isfinite(CountedReal a) { return std::isfinite(a.v); }
