// opcount.hpp -- an operation-counting scalar for the oracle (test
// infrastructure: it measures the arithmetic the oracle's templates perform,
// e.g. per rollout step, to price the device path's work).
//
// Flop holds a double and tallies every arithmetic operation applied to it.
// Besides the raw tally it counts "non-trivial" operations: an addition or
// subtraction whose operands are both nonzero, a multiplication whose operands
// are both outside {0, 1, -1}, a division whose numerator is nonzero and whose
// denominator is outside {1, -1}.  Products with exact zeros and ones come from
// the dense 3x3 and 6x6 forms (identity joint frames, structural zeros of
// spatial transforms and inertias) that a structured implementation does not
// evaluate; the non-trivial tally is the work that remains.
#pragma once
#include <cmath>
#include <cstdint>
#include <limits>

namespace orc {

struct OpTally {
  uint64_t add = 0, mul = 0, div = 0, sqrt = 0, trans = 0, cmp = 0;  // raw
  uint64_t nt_add = 0, nt_mul = 0, nt_div = 0;                       // non-trivial
};
inline OpTally g_tally;

struct Flop {
  double v;
  Flop() : v(0) {}
  Flop(double x) : v(x) {}
  explicit operator double() const { return v; }
  Flop& operator+=(Flop b);
  Flop& operator-=(Flop b);
  Flop& operator*=(Flop b);
  Flop& operator/=(Flop b);
};

inline bool unit_or_zero(double x) { return x == 0.0 || x == 1.0 || x == -1.0; }

inline Flop operator+(Flop a, Flop b) {
  ++g_tally.add;
  if (a.v != 0.0 && b.v != 0.0) ++g_tally.nt_add;
  return Flop(a.v + b.v);
}
inline Flop operator-(Flop a, Flop b) {
  ++g_tally.add;
  if (a.v != 0.0 && b.v != 0.0) ++g_tally.nt_add;
  return Flop(a.v - b.v);
}
inline Flop operator*(Flop a, Flop b) {
  ++g_tally.mul;
  if (!unit_or_zero(a.v) && !unit_or_zero(b.v)) ++g_tally.nt_mul;
  return Flop(a.v * b.v);
}
inline Flop operator/(Flop a, Flop b) {
  ++g_tally.div;
  if (a.v != 0.0 && b.v != 1.0 && b.v != -1.0) ++g_tally.nt_div;
  return Flop(a.v / b.v);
}
inline Flop operator-(Flop a) { return Flop(-a.v); }  // a sign flip, not an operation
inline Flop& Flop::operator+=(Flop b) { return *this = *this + b; }
inline Flop& Flop::operator-=(Flop b) { return *this = *this - b; }
inline Flop& Flop::operator*=(Flop b) { return *this = *this * b; }
inline Flop& Flop::operator/=(Flop b) { return *this = *this / b; }

#define ORC_FLOP_CMP(op)                        \
  inline bool operator op(Flop a, Flop b) {     \
    ++g_tally.cmp;                              \
    return a.v op b.v;                          \
  }
ORC_FLOP_CMP(<)
ORC_FLOP_CMP(>)
ORC_FLOP_CMP(<=)
ORC_FLOP_CMP(>=)
ORC_FLOP_CMP(==)
ORC_FLOP_CMP(!=)
#undef ORC_FLOP_CMP

}  // namespace orc

// The math functions the oracle calls through std::, for the counting scalar.
namespace std {
inline orc::Flop sqrt(orc::Flop x) { ++orc::g_tally.sqrt; return orc::Flop(std::sqrt(x.v)); }
inline orc::Flop sin(orc::Flop x) { ++orc::g_tally.trans; return orc::Flop(std::sin(x.v)); }
inline orc::Flop cos(orc::Flop x) { ++orc::g_tally.trans; return orc::Flop(std::cos(x.v)); }
inline orc::Flop exp(orc::Flop x) { ++orc::g_tally.trans; return orc::Flop(std::exp(x.v)); }
inline orc::Flop log(orc::Flop x) { ++orc::g_tally.trans; return orc::Flop(std::log(x.v)); }
inline orc::Flop atan2(orc::Flop y, orc::Flop x) { ++orc::g_tally.trans; return orc::Flop(std::atan2(y.v, x.v)); }
inline orc::Flop fabs(orc::Flop x) { ++orc::g_tally.cmp; return orc::Flop(std::fabs(x.v)); }
inline orc::Flop floor(orc::Flop x) { ++orc::g_tally.cmp; return orc::Flop(std::floor(x.v)); }
inline bool isfinite(orc::Flop x) { return std::isfinite(x.v); }
template <> class numeric_limits<orc::Flop> {
 public:
  static orc::Flop infinity() { return orc::Flop(std::numeric_limits<double>::infinity()); }
};
}  // namespace std
