// Forward-mode dual numbers for the adjoint: running the Jacobians' own
// formulas on them yields dF/dp next to F itself.  DualN<N> carries N
// directions: the plane Jacobian depends on (z, kappa, phi, theta) -- D4 --,
// the cylinder Jacobian on (x, y, kappa, phi, theta) -- D5.
#pragma once

#include "kf_device.h"

namespace kf {

template <int N>
struct DualN {
  float v;
  float d[N];
  __device__ __forceinline__ DualN() : v(0.0f) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0f;
  }
  __device__ __forceinline__ explicit DualN(float c) : v(c) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0f;
  }
};
using D4 = DualN<4>;
using D5 = DualN<5>;

template <int N>
__device__ __forceinline__ DualN<N> operator-(const DualN<N>& a) {
  DualN<N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ DualN<N> operator+(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ DualN<N> operator-(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ DualN<N> operator*(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ DualN<N> operator*(float a, const DualN<N>& b) {
  DualN<N> r;
  r.v = a * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a * b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ DualN<N> operator*(const DualN<N>& a, float b) { return b * a; }
template <int N>
__device__ __forceinline__ DualN<N> operator+(const DualN<N>& a, float b) {
  DualN<N> r = a;
  r.v = a.v + b;
  return r;
}
template <int N>
__device__ __forceinline__ DualN<N> operator+(float a, const DualN<N>& b) { return b + a; }
template <int N>
__device__ __forceinline__ DualN<N> operator-(const DualN<N>& a, float b) { return a + (-b); }
template <int N>
__device__ __forceinline__ DualN<N> operator-(float a, const DualN<N>& b) { return (-b) + a; }

template <int N>
__device__ __forceinline__ DualN<N> chain(const DualN<N>& a, float fv, float dfv) {
  DualN<N> r;
  r.v = fv;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = dfv * a.d[i];
  return r;
}

template <int N>
__device__ __forceinline__ float val(const DualN<N>& x) { return x.v; }

template <int N>
__device__ __forceinline__ void sincos_t(const DualN<N>& x, DualN<N>* s, DualN<N>* c) {
  float sv, cv;
  sincos_r(x.v, &sv, &cv);
  *s = chain(x, sv, cv);
  *c = chain(x, cv, -sv);
}

template <int N>
__device__ __forceinline__ DualN<N> rcp_t(const DualN<N>& x) {
  const float r = rcp(x.v);
  return chain(x, r, -r * r);
}

// d sinc/du = -G(u);  dG/du = sinc(u) - 2 G(u)/u, or for |u| < 1/2 its Taylor
// series 1/3 - u^2/10 + u^4/168 - u^6/6480 + u^8/443520.
template <int N>
__device__ __forceinline__ void sinc_g_t(const DualN<N>& u, const DualN<N>& su, const DualN<N>& cu, DualN<N>& sinc,
                                         DualN<N>& g) {
  float s0, g0;
  sinc_g(u.v, su.v, cu.v, s0, g0);
  const float u2 = u.v * u.v;
  const float gs = 1.0f / 3.0f - u2 * (0.1f - u2 * (1.0f / 168.0f - u2 * (1.0f / 6480.0f - u2 * (1.0f / 443520.0f))));
  const float gd = s0 - 2.0f * g0 * rcp(u.v);
  const float dg = fabsf(u.v) < 0.5f ? gs : gd;
  sinc = chain(u, s0, -g0);
  g = chain(u, g0, dg);
}

template <int N>
__device__ __forceinline__ void helix_trig_t(const DualN<N>& u, DualN<N>& su, DualN<N>& cu, DualN<N>& sinc,
                                             DualN<N>& g) {
  sincos_t(u, &su, &cu);
  sinc_g_t(u, su, cu, sinc, g);
}

}  // namespace kf
