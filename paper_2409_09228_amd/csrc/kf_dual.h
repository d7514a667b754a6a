// Forward-mode dual numbers with four directions, for the adjoint: running the
// plane Jacobian's own formulas on them yields dF/dp along (z, kappa, phi,
// theta) -- the only parameters F depends on -- next to F itself.
#pragma once

#include "kf_device.h"

namespace kf {

struct D4 {
  float v;
  float d[4];
  __device__ __forceinline__ D4() : v(0.0f), d{0.0f, 0.0f, 0.0f, 0.0f} {}
  __device__ __forceinline__ explicit D4(float c) : v(c), d{0.0f, 0.0f, 0.0f, 0.0f} {}
};

__device__ __forceinline__ D4 operator-(const D4& a) {
  D4 r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.d[i] = -a.d[i];
  return r;
}
__device__ __forceinline__ D4 operator+(const D4& a, const D4& b) {
  D4 r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
__device__ __forceinline__ D4 operator-(const D4& a, const D4& b) {
  D4 r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
__device__ __forceinline__ D4 operator*(const D4& a, const D4& b) {
  D4 r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
__device__ __forceinline__ D4 operator*(float a, const D4& b) {
  D4 r;
  r.v = a * b.v;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.d[i] = a * b.d[i];
  return r;
}
__device__ __forceinline__ D4 operator*(const D4& a, float b) { return b * a; }
__device__ __forceinline__ D4 operator+(const D4& a, float b) {
  D4 r = a;
  r.v = a.v + b;
  return r;
}
__device__ __forceinline__ D4 operator+(float a, const D4& b) { return b + a; }
__device__ __forceinline__ D4 operator-(const D4& a, float b) { return a + (-b); }
__device__ __forceinline__ D4 operator-(float a, const D4& b) { return (-b) + a; }

__device__ __forceinline__ D4 chain(const D4& a, float fv, float dfv) {
  D4 r;
  r.v = fv;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.d[i] = dfv * a.d[i];
  return r;
}

__device__ __forceinline__ void sincos_t(const D4& x, D4* s, D4* c) {
  float sv, cv;
  sincos_r(x.v, &sv, &cv);
  *s = chain(x, sv, cv);
  *c = chain(x, cv, -sv);
}

__device__ __forceinline__ D4 rcp_t(const D4& x) {
  const float r = rcp(x.v);
  return chain(x, r, -r * r);
}

// d sinc/du = -G(u);  dG/du = sinc(u) - 2 G(u)/u, or for |u| < 1/2 its Taylor
// series 1/3 - u^2/10 + u^4/168 - u^6/6480 + u^8/443520.
__device__ __forceinline__ void sinc_g_t(const D4& u, const D4& su, const D4& cu, D4& sinc, D4& g) {
  float s0, g0;
  sinc_g(u.v, su.v, cu.v, s0, g0);
  const float u2 = u.v * u.v;
  const float gs = 1.0f / 3.0f - u2 * (0.1f - u2 * (1.0f / 168.0f - u2 * (1.0f / 6480.0f - u2 * (1.0f / 443520.0f))));
  const float gd = s0 - 2.0f * g0 * rcp(u.v);
  const float dg = fabsf(u.v) < 0.5f ? gs : gd;
  sinc = chain(u, s0, -g0);
  g = chain(u, g0, dg);
}

__device__ __forceinline__ void helix_trig_t(const D4& u, D4& su, D4& cu, D4& sinc, D4& g) {
  sincos_t(u, &su, &cu);
  sinc_g_t(u, su, cu, sinc, g);
}

}  // namespace kf
