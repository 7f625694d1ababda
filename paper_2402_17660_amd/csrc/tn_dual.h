// Dual numbers v + d*eps (eps^2 = 0) for forward-mode differentiation on the device.
//
// The training step needs the parameter gradient of a loss on the forces, which are
// themselves a position gradient of the energy (Sec. 2.5: force training differentiates
// through the force computation a second time).  Running the hand-written reverse sweep
// (energy -> parameters) on dual numbers whose positions carry a tangent w gives, in the
// eps parts, the directional derivative of that parameter gradient along w: a mixed
// second derivative d2E / (d theta d r) . w, exactly (forward-over-reverse), without a
// second reverse pass.  The node kernels are templated on their arithmetic type and reach
// exp, sqrt, cos and sin through the dexp/dsqrt/dcos/dsin overloads, so they compile for
// Dual<S> unchanged; comparisons look at the value part only.
#pragma once

#include "tn_device.h"

#include <type_traits>

namespace tn {

template <class S>
struct Dual {
  using scalar = S;
  S v, d;
  Dual() = default;   // trivial, so arrays of Dual may live in LDS
  template <class U, class = typename std::enable_if<std::is_arithmetic<U>::value>::type>
  __host__ __device__ constexpr Dual(U x) : v(static_cast<S>(x)), d(S(0)) {}
  __host__ __device__ constexpr Dual(S x, S y) : v(x), d(y) {}

  friend __host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
  friend __host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
  friend __host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.v * b.d + a.d * b.v); }
  friend __host__ __device__ inline Dual operator/(Dual a, Dual b) {
    const S r = S(1) / b.v;
    const S q = a.v * r;
    return Dual(q, (a.d - q * b.d) * r);
  }
  friend __host__ __device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
  __host__ __device__ inline Dual &operator+=(Dual b) { v += b.v; d += b.d; return *this; }
  __host__ __device__ inline Dual &operator-=(Dual b) { v -= b.v; d -= b.d; return *this; }
  __host__ __device__ inline Dual &operator*=(Dual b) { *this = *this * b; return *this; }
  __host__ __device__ inline Dual &operator/=(Dual b) { *this = *this / b; return *this; }
  friend __host__ __device__ inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __host__ __device__ inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
  friend __host__ __device__ inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
  friend __host__ __device__ inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
};
// Lane shuffles of dual numbers, component by component (used by the wave reductions).
template <class S>
__device__ __forceinline__ Dual<S> lane_shfl_down(Dual<S> x, int off) {
  return Dual<S>(__shfl_down(x.v, off, 64), __shfl_down(x.d, off, 64));
}
template <class S>
__device__ __forceinline__ Dual<S> lane_shfl(Dual<S> x, int src) {
  return Dual<S>(__shfl(x.v, src, 64), __shfl(x.d, src, 64));
}


template <class S> __device__ inline Dual<S> dexp(Dual<S> x) {
  const S e = dexp(x.v);
  return Dual<S>(e, e * x.d);
}
template <class S> __device__ inline Dual<S> dsqrt(Dual<S> x) {
  const S r = dsqrt(x.v);
  return Dual<S>(r, x.d / (S(2) * r));
}
template <class S> __device__ inline Dual<S> dcos(Dual<S> x) { return Dual<S>(dcos(x.v), -dsin(x.v) * x.d); }
template <class S> __device__ inline Dual<S> dsin(Dual<S> x) { return Dual<S>(dsin(x.v), dcos(x.v) * x.d); }

template <class T> struct is_dual : std::false_type {};
template <class S> struct is_dual<Dual<S>> : std::true_type {};

}  // namespace tn
