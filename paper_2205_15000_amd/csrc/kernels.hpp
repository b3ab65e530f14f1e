// Device-side building blocks: complex arithmetic and the Riccati step.
//
// Everything here runs in either FP64 or FP32 (the mixed path).  The FP32
// versions use the hardware square root and reciprocal (1 ulp); the FP64
// versions use correctly rounded library sqrt and division.
#pragma once

#include <hip/hip_runtime.h>

namespace qc {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return mk(s * a.x, s * a.y); }
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return mk(-a.y, a.x); }  // i * a

__device__ __forceinline__ double dsqrt(double v) { return __builtin_sqrt(v); }
__device__ __forceinline__ float dsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double drcp(double v) { return 1.0 / v; }
__device__ __forceinline__ double dabs(double v) { return __builtin_fabs(v); }
__device__ __forceinline__ float dabs(float v) { return __builtin_fabsf(v); }
__device__ __forceinline__ double dsign(double m, double s) { return __builtin_copysign(m, s); }
__device__ __forceinline__ float dsign(float m, float s) { return __builtin_copysignf(m, s); }
__device__ __forceinline__ float drcp(float v) { return __builtin_amdgcn_rcpf(v); }

// a / b as a * conj(b) / |b|^2 (operands here are O(1): no scaling needed)
template <typename T>
__device__ __forceinline__ cpx<T> cdiv(cpx<T> a, cpx<T> b) {
  const T r = drcp(b.x * b.x + b.y * b.y);
  return mk((a.x * b.x + a.y * b.y) * r, (a.y * b.x - a.x * b.y) * r);
}

// Principal square root (branch cut on the negative real axis, the sign of
// a zero imaginary part picks the side): sqrt((|w|+|x|)/2) formula.
template <typename T>
__device__ __forceinline__ cpx<T> csqrt(cpx<T> w) {
  const T r = dsqrt(w.x * w.x + w.y * w.y);
  if (r == T(0)) return mk(T(0), T(0));
  const T t = dsqrt(T(0.5) * (r + dabs(w.x)));
  const T q = T(0.5) * drcp(t);
  if (w.x >= T(0)) return mk(t, w.y * q);
  return mk(dabs(w.y) * q, dsign(t, w.y));
}

// One implicit-midpoint step of d gamma/ds = i[D* g^2 + 2 z g + D]
// (App. C, v_F = 1) in the closed form g' = 2 c0 / (-c1 + sqrt(c1^2 - 4 c2 c0));
// the root is flipped if it points away from -c1, so g' -> g as h -> 0.
template <typename T>
__device__ __forceinline__ cpx<T> riccati_step(cpx<T> g, cpx<T> dm, cpx<T> zm, T hstep) {
  const T hq = T(0.25) * hstep;
  const cpx<T> c2 = mk(hq * dm.y, hq * dm.x);  // (i h/4) conj(dm)
  const cpx<T> c2g = c2 * g;
  const cpx<T> ihz = mk(-hstep * zm.y, hstep * zm.x);
  const cpx<T> c1 = mk(T(2) * c2g.x + ihz.x - T(1), T(2) * c2g.y + ihz.y);
  const cpx<T> c0 = mk(c1.x - c2g.x + T(2), c1.y - c2g.y) * g - mk(T(4) * c2.x, T(-4) * c2.y);
  const cpx<T> c1s = c1 * c1;
  const cpx<T> c20 = c2 * c0;
  cpx<T> rt = csqrt(mk(c1s.x - T(4) * c20.x, c1s.y - T(4) * c20.y));
  if (rt.x * c1.x + rt.y * c1.y > T(0)) rt = mk(-rt.x, -rt.y);  // Re(rt conj(-c1)) < 0
  return cdiv(mk(T(2) * c0.x, T(2) * c0.y), rt - c1);
}

// Stable homogeneous root of D* g^2 + 2 z g + D = 0: -D / (z + s) with
// s = sqrt(z^2 - |D|^2), Im s > 0.
template <typename T>
__device__ __forceinline__ cpx<T> bulk_root(cpx<T> z, cpx<T> d) {
  const cpx<T> z2 = z * z;
  cpx<T> s = csqrt(mk(z2.x - (d.x * d.x + d.y * d.y), z2.y));
  if (s.y < T(0)) s = mk(-s.x, -s.y);
  const cpx<T> num = mk(-d.x, -d.y);
  return cdiv(num, z + s);
}

}  // namespace qc
