// Device-side building blocks of the Kalman-filter step for gfx950.
//
// One lane carries one track.  Its state -- 6 parameters and the 21 packed
// covariance numbers -- lives in VGPRs for the whole layer loop; every index
// below is a compile-time constant after unrolling, so no array is ever
// spilled to scratch.  The 6x6 and 3x3 products are far too small for MFMA
// tiles, so everything is per-lane VALU arithmetic, written against the
// sparsity of the propagation Jacobian.
//
// Parameter order p = (x, y, z, kappa = q/pT, phi, theta); transverse
// curvature omega = -b kappa with b = 0.00299792458 * Bz.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace kf {

enum : uint32_t { S_NONFINITE = 1u, S_NOT_PD = 2u, S_NO_CROSSING = 4u, S_NEWTON = 8u };

// packed lower-triangle index of symmetric element (i, j)
__host__ __device__ constexpr int ix(int i, int j) {
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

// 1-ulp hardware reciprocal.  Every quantity inverted with it is well away
// from zero and overflow in the domains checked by the callers, and its
// error is far below the FP32 tolerance of the step.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Marks the rare side of a per-lane branch: the empty volatile statement
// keeps the compiler from evaluating that side unconditionally (as a select),
// so a wave whose lanes all take the common side skips it.
__device__ __forceinline__ void rare_path() { __asm__ volatile(""); }

__device__ __forceinline__ bool fin(float x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool fin(double x) { return __builtin_isfinite(x); }

// sin and cos of x.  For |x| <= 8192: x = k pi/2 + r with |r| <= pi/4 by
// Cody-Waite reduction (pi/2 split into two floats, fused multiply-adds;
// the split's residual 1.7e-15 times |k| <= 5216 stays below 1e-11), then the
// Taylor polynomials of sin through r^9 and of cos through r^10 (truncation
// below 3e-9 relative on |r| <= pi/4), and the quarter-turn rotation by k mod 4.
// Larger or non-finite x go to the library sincosf.
__device__ __forceinline__ void sincos_r(float x, float* s, float* c) {
  if (!(fabsf(x) <= 8192.0f)) {
    sincosf(x, s, c);
    return;
  }
  const float kf = __builtin_rintf(x * 0x1.45f306p-1f);  // x * 2/pi
  float r = __builtin_fmaf(kf, -0x1.921fb6p+0f, x);       // - k * (pi/2 high part)
  r = __builtin_fmaf(kf, 0x1.777a5cp-25f, r);             // - k * (pi/2 low part), low part < 0
  const float r2 = r * r;
  const float sp = __builtin_fmaf(
      r * r2, -1.0f / 6.0f + r2 * (1.0f / 120.0f + r2 * (-1.0f / 5040.0f + r2 * (1.0f / 362880.0f))), r);
  const float cp =
      1.0f + r2 * (-0.5f + r2 * (1.0f / 24.0f + r2 * (-1.0f / 720.0f + r2 * (1.0f / 40320.0f + r2 * (-1.0f / 3628800.0f)))));
  const int k = int(kf);
  const bool swap = (k & 1) != 0;
  const float sv = swap ? cp : sp;
  const float cv = swap ? sp : cp;
  *s = __int_as_float(__float_as_int(sv) ^ ((k & 2) << 30));
  *c = __int_as_float(__float_as_int(cv) ^ (((k + 1) & 2) << 30));
}

// sinc(u) = sin(u)/u and G(u) = (sin u - u cos u)/u^2 = -d sinc/du.
// |u| < 1/2: their Taylor series (relative truncation error < 1e-10, and no
// cancellation); otherwise the closed forms.  su, cu = sin u, cos u.
__device__ __forceinline__ void sinc_g(float u, float su, float cu, float& sinc, float& g) {
  const float u2 = u * u;
  const float ss = 1.0f - u2 * (1.0f / 6.0f) * (1.0f - u2 * (1.0f / 20.0f) * (1.0f - u2 * (1.0f / 42.0f) * (1.0f - u2 * (1.0f / 72.0f))));
  const float gs = u * (1.0f / 3.0f - u2 * (1.0f / 30.0f - u2 * (1.0f / 840.0f - u2 * (1.0f / 45360.0f - u2 * (1.0f / 3991680.0f)))));
  const float ru = rcp(u);
  const bool small = fabsf(u) < 0.5f;
  sinc = small ? ss : su * ru;
  g = small ? gs : (su - u * cu) * ru * ru;
}

// Horner forms in u^2 of the series used on |u| < 1/2 (truncation after the
// last term shown, relative to the function's value):
//   sinc u   = 1 - u^2/6 + u^4/120 - u^6/5040 + u^8/362880          (< 3e-11)
//   cos u    = 1 - u^2/2 + u^4/24 - u^6/720 + u^8/40320             (< 4e-10)
//   G(u)/u   = 1/3 - u^2/30 + u^4/840 - u^6/45360                   (< 3e-9)
__device__ __forceinline__ float sinc_series(float u2) {
  return __builtin_fmaf(u2, __builtin_fmaf(u2, __builtin_fmaf(u2, __builtin_fmaf(u2, 1.0f / 362880.0f, -1.0f / 5040.0f),
                                                                1.0f / 120.0f), -1.0f / 6.0f), 1.0f);
}
__device__ __forceinline__ float cos_series(float u2) {
  return __builtin_fmaf(u2, __builtin_fmaf(u2, __builtin_fmaf(u2, __builtin_fmaf(u2, 1.0f / 40320.0f, -1.0f / 720.0f),
                                                                1.0f / 24.0f), -0.5f), 1.0f);
}
__device__ __forceinline__ float g_over_u_series(float u2) {
  return __builtin_fmaf(u2, __builtin_fmaf(u2, __builtin_fmaf(u2, -1.0f / 45360.0f, 1.0f / 840.0f), -1.0f / 30.0f),
                        1.0f / 3.0f);
}

// sin u, cos u, sinc u and (WANT_G) G(u) for the helix's half turning angle
// u.  Each lane takes one of two branches by its own |u|, so a track's result
// never depends on the other tracks of its wave: the series above for
// |u| < 1/2 (the usual case: a few degrees between layers), else the reduced
// sin/cos and the closed forms.
template <bool WANT_G>
__device__ __forceinline__ void helix_trig(float u, float& su, float& cu, float& sinc, float& g) {
  if (fabsf(u) < 0.5f) {
    const float u2 = u * u;
    sinc = sinc_series(u2);
    su = u * sinc;
    cu = cos_series(u2);
    if (WANT_G) g = u * g_over_u_series(u2);
  } else {
    rare_path();
    sincos_r(u, &su, &cu);
    const float ru = rcp(u);
    sinc = su * ru;
    if (WANT_G) g = (su - u * cu) * ru * ru;
  }
}

// sin and cos of the two direction angles (phi, theta), carried from layer to
// layer instead of being re-evaluated: propagation hands over the direction
// at the surface, and an update that moves an angle by d rotates the pair by
// d.  For |d| <= 1/8 the rotation uses sin d = d - d^3/6 + d^5/120 (error
// < 1e-10) and cos d = 1 - d^2/2 + d^4/24 - d^6/720 (< 2e-12); a larger step
// (a poor seed) re-evaluates sin and cos of the updated angle itself.  The
// rounding of the carried pair drifts by about one ulp per layer.
template <class T>
struct DirT {
  T sp, cp, st, ct;  // sin phi, cos phi, sin theta, cos theta
};
using Dir = DirT<float>;

__device__ __forceinline__ void dir_init(const float p[6], Dir& d) {
  sincos_r(p[4], &d.sp, &d.cp);
  sincos_r(p[5], &d.st, &d.ct);
}

__device__ __forceinline__ void rotate_by(float& s, float& c, float d, float angle) {
  if (fabsf(d) <= 0.125f) {
    const float d2 = d * d;
    const float sd = __builtin_fmaf(d * d2, __builtin_fmaf(d2, 1.0f / 120.0f, -1.0f / 6.0f), d);
    const float cd = __builtin_fmaf(d2, __builtin_fmaf(d2, __builtin_fmaf(d2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f), 1.0f);
    const float sn = s * cd + c * sd;
    c = c * cd - s * sd;
    s = sn;
  } else {
    rare_path();
    sincos_r(angle, &s, &c);
  }
}

// ----------------------------------------------------------------------------
// Scalar-generic helpers: the same formulas run on float and, for the adjoint,
// on dual numbers (kf_dual.h) to differentiate the Jacobian itself.
__device__ __forceinline__ void sincos_t(float x, float* s, float* c) { sincos_r(x, s, c); }
__device__ __forceinline__ float rcp_t(float x) { return rcp(x); }
__device__ __forceinline__ void sinc_g_t(float u, float su, float cu, float& sinc, float& g) { sinc_g(u, su, cu, sinc, g); }
__device__ __forceinline__ void helix_trig_t(float u, float& su, float& cu, float& sinc, float& g) {
  helix_trig<true>(u, su, cu, sinc, g);
}
__device__ __forceinline__ void helix_sinc_t(float u, float& su, float& cu, float& sinc) {
  float unused;
  helix_trig<false>(u, su, cu, sinc, unused);
}
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }
__device__ __forceinline__ float fmax_t(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ float fabs_t(float x) { return fabsf(x); }
__device__ __forceinline__ float val(float x) { return x; }
__device__ __forceinline__ double val(double x) { return x; }

// The same helpers in FP64 (the full-FP64 form of the step).  The division is
// exact IEEE division.  For |u| < 1/2, the range the FP32 helpers give to their
// series too (a curved track's half turning angle between layers reaches a
// few tenths), sin u, cos u, sinc u and G(u) come from their Taylor series --
// sinc and cos through u^14, G through u^13: truncation below 5e-20, 1e-18 and
// 1e-17 relative -- and beyond from the library's sin and cos and the closed
// forms, where the cancellation in sin u - u cos u (about u^3/3) costs at most
// 1e-15 relative.  A lane past 1/2 makes its whole wave run both branches, so
// the series' range decides how often the library's sin and cos run at all.
// The direction's sin and cos are carried across layers as in FP32: an update
// that moves an angle by |d| <= 1/8 rotates the pair by d (sin d through d^11,
// cos d through d^10: truncation below 1e-19), a larger one re-evaluates
// them; the carried pair drifts by about one ulp per layer.
__device__ __forceinline__ void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ double fmax_t(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double fabs_t(double x) { return fabs(x); }

// x y + c with c read from a pair of scalar registers.  c must hold the same
// value in every lane -- every caller passes a literal series coefficient --
// since a scalar operand is one value for the whole wave.  A VOP3 FMA takes
// such a 64-bit constant from SGPRs (set by two scalar moves); the compiler's
// own choice is to copy it into two VGPRs first, two more vector instructions
// per coefficient.
__device__ __forceinline__ double fma_sc(double x, double y, double c) {
  double r;
  __asm__("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(y), "s"(c));
  return r;
}
// The series of sinc u, cos u and (WANT_G) G(u)/u in x = u^2 by Horner's
// rule, the chains advanced in lockstep: each FMA waits for its own chain's
// last one only, so the chains' FMAs overlap (one chain alone would wait out
// every FMA's latency).  The innermost term of each chain is a product and a
// sum, in statements of their own (no contraction): an FMA reads at most one
// scalar operand.
template <bool WANT_G>
__device__ __forceinline__ void trig_series64(double x, double& sinc, double& cosu, double& g_over_u) {
  double a = x * (-1.0 / 1307674368000.0);  // sinc: through u^14
  double c = x * (-1.0 / 87178291200.0);    // cos: through u^14
  double g = x * (1.0 / 93405312000.0);     // G/u: through u^12
  a = a + 1.0 / 6227020800.0;
  c = c + 1.0 / 479001600.0;
  if (WANT_G) g = g - 1.0 / 518918400.0;
  a = fma_sc(x, a, -1.0 / 39916800.0);
  c = fma_sc(x, c, -1.0 / 3628800.0);
  if (WANT_G) g = fma_sc(x, g, 1.0 / 3991680.0);
  a = fma_sc(x, a, 1.0 / 362880.0);
  c = fma_sc(x, c, 1.0 / 40320.0);
  if (WANT_G) g = fma_sc(x, g, -1.0 / 45360.0);
  a = fma_sc(x, a, -1.0 / 5040.0);
  c = fma_sc(x, c, -1.0 / 720.0);
  if (WANT_G) g = fma_sc(x, g, 1.0 / 840.0);
  a = fma_sc(x, a, 1.0 / 120.0);
  c = fma_sc(x, c, 1.0 / 24.0);
  if (WANT_G) g = fma_sc(x, g, -1.0 / 30.0);
  a = fma_sc(x, a, -1.0 / 6.0);
  c = fma_sc(x, c, -1.0 / 2.0);
  if (WANT_G) g = fma_sc(x, g, 1.0 / 3.0);
  sinc = __builtin_fma(x, a, 1.0);
  cosu = __builtin_fma(x, c, 1.0);
  if (WANT_G) g_over_u = g;
}

__device__ __forceinline__ void helix_sinc_t(double u, double& su, double& cu, double& sinc) {
  if (fabs(u) < 0.5) {
    double unused;
    trig_series64<false>(u * u, sinc, cu, unused);
    su = u * sinc;
  } else {
    rare_path();
    sincos(u, &su, &cu);
    sinc = su / u;
  }
}
__device__ __forceinline__ void helix_trig_t(double u, double& su, double& cu, double& sinc, double& g) {
  if (fabs(u) < 0.5) {
    double gu;
    trig_series64<true>(u * u, sinc, cu, gu);
    su = u * sinc;
    g = u * gu;
  } else {
    rare_path();
    sincos(u, &su, &cu);
    sinc = su / u;
    g = (su - u * cu) / (u * u);
  }
}
__device__ __forceinline__ void dir_init(const double p[6], DirT<double>& d) {
  sincos(p[4], &d.sp, &d.cp);
  sincos(p[5], &d.st, &d.ct);
}
__device__ __forceinline__ void rotate_by(double& s, double& c, double d, double angle) {
  if (fabs(d) <= 0.125) {
    const double x = d * d;
    double a = x * (-1.0 / 39916800.0);  // sin d / d: through d^10
    double b = x * (-1.0 / 3628800.0);   // cos d: through d^10
    a = a + 1.0 / 362880.0;
    b = b + 1.0 / 40320.0;
    a = fma_sc(x, a, -1.0 / 5040.0);
    b = fma_sc(x, b, -1.0 / 720.0);
    a = fma_sc(x, a, 1.0 / 120.0);
    b = fma_sc(x, b, 1.0 / 24.0);
    a = fma_sc(x, a, -1.0 / 6.0);
    b = fma_sc(x, b, -1.0 / 2.0);
    const double sd = d * __builtin_fma(x, a, 1.0);
    const double cd = __builtin_fma(x, b, 1.0);
    const double sn = s * cd + c * sd;
    c = c * cd - s * sd;
    s = sn;
  } else {
    rare_path();
    sincos(angle, &s, &c);
  }
}

// The non-trivial entries of the plane Jacobian F:
//   row x   = e_x + a0 e_z + a1 e_k + a2 e_phi + a3 e_th
//   row y   = e_y + b0 e_z + b1 e_k + b2 e_phi + b3 e_th
//   row phi = c0 e_z + c1 e_k + e_phi + c3 e_th
// rows kappa and theta are the identity's; row z is zero.
template <class T>
struct PlaneJac {
  T a0, a1, a2, a3, b0, b1, b2, b3, c0, c1, c3;
};

// ----------------------------------------------------------------------------
// Propagation to a plane z = zk.
//
// The transverse path to the plane is s = (zk - z) tan(theta).  With
// u = omega s / 2 and A = phi + u the helix moves by
//   dx = s sinc(u) cos A,  dy = s sinc(u) sin A,  dphi = omega s
// (the cancellation-free chord form), and z lands exactly on zk.
// F = J_s + (dp/ds) (grad s)^T, with J_s the fixed-s partials:
//   d dx/d omega = -(s^2/2)(sin A sinc u + cos A G(u)),
//   d dy/d omega =  (s^2/2)(cos A sinc u - sin A G(u)),
//   d dx/d phi = -dy, d dy/d phi = dx, d phi'/d kappa = -b s,
// dp/ds = (cos phi', sin phi', cot theta, 0, omega, 0) and
// grad s = (0, 0, -tan theta, 0, 0, (zk - z)/cos^2 theta).  The z row of F is
// identically zero, so the z row and column of the transported covariance vanish.
// T: the state's scalar (float, double, or dual numbers); S: the geometry's
// (layer position and field constant: float, or double in the FP64 form).
template <class T, class S>
__device__ __forceinline__ void helix_to_plane_dir(const T p[6], const T& sth, const T& cth, const T& sp, const T& cp,
                                                   S zk, S b, T q[6], PlaneJac<T>& J, T& sP, T& cP) {
  const T rcth = rcp_t(cth);
  const T tanth = sth * rcth;
  const T dz = zk - p[2];
  const T s = dz * tanth;
  const T om = -b * p[3];
  const T u = 0.5f * om * s;
  T su, cu, sinc, g;
  helix_trig_t(u, su, cu, sinc, g);
  const T cA = cp * cu - sp * su;
  const T sA = sp * cu + cp * su;
  const T chord = s * sinc;
  const T dx = chord * cA;
  const T dy = chord * sA;
  cP = cA * cu - sA * su;  // direction at the plane
  sP = sA * cu + cA * su;
  q[0] = p[0] + dx;
  q[1] = p[1] + dy;
  q[2] = T(zk);
  q[3] = p[3];
  q[4] = p[4] + om * s;
  q[5] = p[5];

  const T hs2 = 0.5f * s * s;
  const T dxdom = -hs2 * (sA * sinc + cA * g);
  const T dydom = hs2 * (cA * sinc - sA * g);
  const T dsdth = dz * rcth * rcth;
  J.a0 = -tanth * cP;
  J.a1 = -b * dxdom;
  J.a2 = -dy;
  J.a3 = cP * dsdth;
  J.b0 = -tanth * sP;
  J.b1 = -b * dydom;
  J.b2 = dx;
  J.b3 = sP * dsdth;
  J.c0 = -om * tanth;
  J.c1 = -b * s;
  J.c3 = om * dsdth;
}

// The same, evaluating the direction's sin and cos from p itself.
template <class T, class S>
__device__ __forceinline__ void helix_to_plane(const T p[6], S zk, S b, T q[6], PlaneJac<T>& J) {
  T sth, cth, sp, cp, sP, cP;
  sincos_t(p[5], &sth, &cth);
  sincos_t(p[4], &sp, &cp);
  helix_to_plane_dir<T, S>(p, sth, cth, sp, cp, zk, b, q, J, sP, cP);
}

// Pt = F C F^T for the plane Jacobian, on packed covariances.  ZIN: the z row
// and column of C are known to be zero (C is the result of a plane update),
// which removes the z column from every product.
template <bool ZIN, class T>
__device__ __forceinline__ void transport_plane(const PlaneJac<T>& J, const T C[21], T Pt[21]) {
  const T a0 = J.a0, a1 = J.a1, a2 = J.a2, a3 = J.a3;
  const T b0 = J.b0, b1 = J.b1, b2 = J.b2, b3 = J.b3;
  const T c0 = J.c0, c1 = J.c1, c3 = J.c3;
  // W_r = C F_r^T (column r of C F^T) for the three non-trivial rows
  T Wx[6], Wy[6], Wf[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T c3_ = C[ix(i, 3)], c4 = C[ix(i, 4)], c5 = C[ix(i, 5)];
    if (ZIN) {
      if (i == 2) {
        Wx[i] = Wy[i] = Wf[i] = T(0);
        continue;
      }
      Wx[i] = C[ix(i, 0)] + a1 * c3_ + a2 * c4 + a3 * c5;
      Wy[i] = C[ix(i, 1)] + b1 * c3_ + b2 * c4 + b3 * c5;
      Wf[i] = c1 * c3_ + c4 + c3 * c5;
    } else {
      const T c2 = C[ix(i, 2)];
      Wx[i] = C[ix(i, 0)] + a0 * c2 + a1 * c3_ + a2 * c4 + a3 * c5;
      Wy[i] = C[ix(i, 1)] + b0 * c2 + b1 * c3_ + b2 * c4 + b3 * c5;
      Wf[i] = c0 * c2 + c1 * c3_ + c4 + c3 * c5;
    }
  }
  if (ZIN) {
    Pt[ix(0, 0)] = Wx[0] + a1 * Wx[3] + a2 * Wx[4] + a3 * Wx[5];
    Pt[ix(1, 0)] = Wx[1] + b1 * Wx[3] + b2 * Wx[4] + b3 * Wx[5];
    Pt[ix(1, 1)] = Wy[1] + b1 * Wy[3] + b2 * Wy[4] + b3 * Wy[5];
    Pt[ix(4, 0)] = c1 * Wx[3] + Wx[4] + c3 * Wx[5];
    Pt[ix(4, 1)] = c1 * Wy[3] + Wy[4] + c3 * Wy[5];
    Pt[ix(4, 3)] = c1 * C[ix(3, 3)] + C[ix(4, 3)] + c3 * C[ix(5, 3)];
    Pt[ix(4, 4)] = c1 * Wf[3] + Wf[4] + c3 * Wf[5];
  } else {
    Pt[ix(0, 0)] = Wx[0] + a0 * Wx[2] + a1 * Wx[3] + a2 * Wx[4] + a3 * Wx[5];
    Pt[ix(1, 0)] = Wx[1] + b0 * Wx[2] + b1 * Wx[3] + b2 * Wx[4] + b3 * Wx[5];
    Pt[ix(1, 1)] = Wy[1] + b0 * Wy[2] + b1 * Wy[3] + b2 * Wy[4] + b3 * Wy[5];
    Pt[ix(4, 0)] = c0 * Wx[2] + c1 * Wx[3] + Wx[4] + c3 * Wx[5];
    Pt[ix(4, 1)] = c0 * Wy[2] + c1 * Wy[3] + Wy[4] + c3 * Wy[5];
    Pt[ix(4, 3)] = c0 * C[ix(2, 3)] + c1 * C[ix(3, 3)] + C[ix(4, 3)] + c3 * C[ix(5, 3)];
    Pt[ix(4, 4)] = c0 * Wf[2] + c1 * Wf[3] + Wf[4] + c3 * Wf[5];
  }
  Pt[ix(2, 0)] = T(0);
  Pt[ix(2, 1)] = T(0);
  Pt[ix(2, 2)] = T(0);
  Pt[ix(3, 0)] = Wx[3];
  Pt[ix(3, 1)] = Wy[3];
  Pt[ix(3, 2)] = T(0);
  Pt[ix(3, 3)] = C[ix(3, 3)];
  Pt[ix(4, 2)] = T(0);
  Pt[ix(5, 0)] = Wx[5];
  Pt[ix(5, 1)] = Wy[5];
  Pt[ix(5, 2)] = T(0);
  Pt[ix(5, 3)] = C[ix(5, 3)];
  Pt[ix(5, 4)] = Wf[5];
  Pt[ix(5, 5)] = C[ix(5, 5)];
}

// d: sin and cos of the direction angles of p on entry, of q on return.
template <bool ZIN, class T>
__device__ __forceinline__ void propagate_z(const T p[6], const T C[21], DirT<T>& d, T zk, T b, T q[6], T Pt[21]) {
  PlaneJac<T> J;
  helix_to_plane_dir<T, T>(p, d.st, d.ct, d.sp, d.cp, zk, b, q, J, d.sp, d.cp);
  transport_plane<ZIN>(J, C, Pt);
}

// ----------------------------------------------------------------------------
// Propagation to a cylinder r = rk: first crossing at s > 0.
//
// Reachability in closed form: with rho0^2 = x^2 + y^2 the helix meets the
// cylinder iff |omega (rk^2 - rho0^2)/2 + x sin(phi) - y cos(phi)| <= rk
// (for omega -> 0: the line's distance from the axis is at most rk).  The
// crossing itself: Newton's method on g(s) = x(s)^2 + y(s)^2 - rk^2 from the
// root of g's second-order expansion, at most five steps (cylinder_search).
// The Jacobian adds to the fixed-s partials the path-length term with
// grad s = -(x J_s[x,:] + y J_s[y,:]) / (x cos phi' + y sin phi'),
// which keeps the propagated point on the cylinder to first order.
// Status bits (0 on success): an unreachable cylinder first, then a crossing
// the iteration did not land on.
//
// The non-trivial entries of the cylinder Jacobian F: rows x, y, phi live in
// columns (x, y, kappa, phi), row z in all six; rows kappa and theta are the
// identity's.
template <class T>
struct CylJac {
  T x0, x1, x3, x4, y0, y1, y3, y4, z0, z1, z3, z4, z5, f0, f1, f3, f4;
};

// The search: closed-form reachability, then Newton's method for the path
// length s on g(s) = x(s)^2 + y(s)^2 - rk^2.  With beta = x cos phi + y sin phi
// and gam = y cos phi - x sin phi (the position along and across the
// direction), ch = s sinc(u) the chord and u = omega s / 2 half the turning
// angle, g = g0 + ch (2 (beta cos u + gam sin u) + ch) with g0 = g(0), and
// g'/2 = beta cos 2u + gam sin 2u + ch cos u: the two constants carry the
// start point and direction through every step.
//   Start: the first positive root of g's second-order expansion
// g0 + 2 beta s + a s^2, a = 1 + omega gam (clamped to >= 1/2), in forms with
// no cancellation and no division by a: from inside the cylinder (g0 < 0)
// -g0 / (beta + sqrt(beta^2 - a g0)), from outside moving inward (g0 > 0) the
// near root g0 / (sqrt(beta^2 - a g0) - beta); where that denominator is not
// positive (moving away from the cylinder, or on it moving inward) the
// straight line's crossing -beta + sqrt(beta^2 - g0) instead.
//   Steps: at most five; a lane stops after a step that moved s by no more
// than search_tol |s| and by no more than a tenth of the step before it: the
// quadratic regime, where the next step would move s by about the ratio
// times this step's relative size, 1e-2 search_tol |s| at most, below the
// scalar's rounding.  Next to a double root the error only halves per step,
// the ratio stays near 1/2 and all five steps run.  The stop is each lane's
// own: a track's result never depends on the other tracks of its wave.
// sp, cp: sin and cos of phi.
__device__ __forceinline__ float search_tol(float) { return 1e-5f; }
__device__ __forceinline__ double search_tol(double) { return 1e-9; }
// The start's square root and the steps' reciprocals need not be correctly
// rounded: the iteration corrects both.  In FP32 the hardware's 1-ulp square
// root and reciprocal; in FP64 the hardware's square root (2^-23 relative, a
// start only) and its reciprocal refined by two Newton-Raphson steps (from
// 2^-23 relative to within an ulp or two), in 1 and 5 instructions where the
// IEEE forms take 20 and 11.
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_fast(double x) { return __builtin_amdgcn_sqrt(x); }
__device__ __forceinline__ float rcp_search(float x) { return rcp(x); }
__device__ __forceinline__ double rcp_search(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

template <class T>
__device__ __forceinline__ T cylinder_search(const T p[6], const T& sp, const T& cp, T rk, T b, bool& reachable) {
  const T om = -b * p[3];
  const T x = p[0], y = p[1];
  const T rho2 = x * x + y * y;
  const T rk2 = rk * rk;
  const T reach = 0.5f * om * (rk2 - rho2) + (x * sp - y * cp);
  reachable = fabs_t(reach) <= rk;
  const T beta = x * cp + y * sp;
  const T gam = y * cp - x * sp;
  const T g0 = rho2 - rk2;
  const T a = fmax_t(1.0f + om * gam, T(0.5f));
  const T sq = sqrt_fast(fmax_t(beta * beta - a * g0, T(0)));
  const bool inward = g0 > T(0);
  const T den = inward ? sq - beta : beta + sq;
  T s = (inward ? g0 : -g0) * rcp_search(den);
  if (!(den > T(0))) {
    rare_path();
    s = -beta + sqrt_fast(fmax_t(beta * beta - g0, T(0)));
  }
  const T hom = 0.5f * om;
  const T tol = search_tol(T(0));
  T prev = T(0);  // the step before (none yet: no stop after the first)
  bool run = true;
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    if (run) {
      rare_path();  // a branch, not a select: a wave whose lanes have all stopped skips the step
      const T u = hom * s;
      T su, cu, sinc;
      helix_sinc_t(u, su, cu, sinc);
      const T ch = s * sinc;
      const T t = beta * cu + gam * su;
      const T g = g0 + ch * (2.0f * t + ch);
      const T c2 = cu * cu - su * su;
      const T s2 = 2.0f * su * cu;
      const T gp = 2.0f * (beta * c2 + gam * s2 + ch * cu);
      const T ds = g * rcp_search(gp);
      s = s - ds;
      run = !((fabs_t(ds) <= tol * fabs_t(s)) & (fabs_t(ds) <= T(0.1f) * fabs_t(prev)));
      prev = ds;
    }
  }
  return s;
}

// The state after transverse path s (the search's result) and the Jacobian
// F there, the path length's dependence on p taken from the implicit
// function x(s)^2 + y(s)^2 = rk^2.  sth, cth, sp, cp: sin and cos of theta
// and phi of p; sP, cP: of phi at the crossing.  Returns whether the point
// lies on the cylinder (|x^2 + y^2 - rk^2| <= 1e-4 rk^2: next to tangency, where
// the search stops short, its residual clusters at 2.0e-4 .. 2.3e-4 rk^2).  T: float, or dual
// numbers (then s carries ds/dp); S: the geometry's scalar.
template <class T, class S>
__device__ __forceinline__ bool cylinder_at(const T p[6], const T& sth, const T& cth, const T& sp, const T& cp,
                                            const T& s, S rk, S b, T q[6], CylJac<T>& J, T& sP, T& cP,
                                            T* inc = nullptr) {
  const T om = -b * p[3];
  const T x = p[0], y = p[1];
  const S rk2 = rk * rk;
  const T u = 0.5f * om * s;
  T su, cu, sinc, g;
  helix_trig_t(u, su, cu, sinc, g);
  const T cA = cp * cu - sp * su;
  const T sA = sp * cu + cp * su;
  const T ch = s * sinc;
  const T dx = ch * cA, dy = ch * sA;
  const T X = x + dx, Y = y + dy;
  cP = cA * cu - sA * su;
  sP = sA * cu + cA * su;
  const bool on_surface = fabs_t(val(X * X + Y * Y - rk2)) <= decltype(val(rk2))(1.0e-4f) * val(rk2);
  const T rsth = rcp_t(sth);
  const T cot = cth * rsth;
  q[0] = X;
  q[1] = Y;
  q[2] = p[2] + s * cot;
  q[3] = p[3];
  q[4] = p[4] + om * s;
  q[5] = p[5];
  if (inc) {
    inc[0] = dx;
    inc[1] = dy;
    inc[2] = s * cot;
    inc[4] = om * s;
  }

  const T hs2 = 0.5f * s * s;
  const T Jxk = b * hs2 * (sA * sinc + cA * g);   // -b d dx/d omega
  const T Jyk = -b * hs2 * (cA * sinc - sA * g);  // -b d dy/d omega
  const T Jxf = -dy, Jyf = dx;
  const T Jzt = -s * rsth * rsth;
  const T Jfk = -b * s;
  const T rD = rcp_t(X * cP + Y * sP);
  const T dsx = -X * rD, dsy = -Y * rD;
  const T dsk = -(X * Jxk + Y * Jyk) * rD;
  const T dsf = -(X * Jxf + Y * Jyf) * rD;
  J.x0 = 1.0f + cP * dsx, J.x1 = cP * dsy, J.x3 = Jxk + cP * dsk, J.x4 = Jxf + cP * dsf;
  J.y0 = sP * dsx, J.y1 = 1.0f + sP * dsy, J.y3 = Jyk + sP * dsk, J.y4 = Jyf + sP * dsf;
  J.z0 = cot * dsx, J.z1 = cot * dsy, J.z3 = cot * dsk, J.z4 = cot * dsf, J.z5 = Jzt;
  J.f0 = om * dsx, J.f1 = om * dsy, J.f3 = Jfk + om * dsk, J.f4 = 1.0f + om * dsf;
  return on_surface;
}

// The crossing q and its Jacobian J; returns the status bits.  d: sin and
// cos of the direction angles of p on entry, of q on return.  inc (if not
// NULL): the increments q - p of x, y, z and phi at full precision (entries
// 0, 1, 2, 4).
template <class T>
__device__ __forceinline__ uint32_t helix_to_cylinder(const T p[6], DirT<T>& d, T rk, T b, T q[6], CylJac<T>& J,
                                                      T* inc = nullptr) {
  bool reachable;
  const T s = cylinder_search(p, d.sp, d.cp, rk, b, reachable);
  T sP, cP;
  const bool on_surface = cylinder_at<T, T>(p, d.st, d.ct, d.sp, d.cp, s, rk, b, q, J, sP, cP, inc);
  d.cp = cP;
  d.sp = sP;
  // the first crossing: g' = 2 (x cos phi + y sin phi) there has the opposite
  // sign to g(0) (g rises through zero from inside the cylinder, falls
  // through it from outside), it lies ahead (s > 0) and the helix has not
  // completed a turn (|omega s| < 2 pi); an iterate where any fails is
  // another crossing (a strongly curved track entering a cylinder, whose
  // start lay past the first crossing and whose steps may run on to a
  // crossing behind the track, or one that loops round and enters again),
  // reported like a search that did not land
  const T gs = q[0] * cP + q[1] * sP;
  const bool first = (p[0] * p[0] + p[1] * p[1] > rk * rk ? gs < T(0) : gs > T(0)) & (s > T(0)) &
                     (fabs_t(b * p[3] * s) < T(6.2831853f));
  return !reachable ? S_NO_CROSSING : (!(on_surface & first) ? S_NEWTON : 0u);
}

// Pt = F C F^T for the cylinder Jacobian, on packed covariances.
template <class T>
__device__ __forceinline__ void transport_cylinder(const CylJac<T>& J, const T C[21], T Pt[21]) {
  const T Fx0 = J.x0, Fx1 = J.x1, Fx3 = J.x3, Fx4 = J.x4;
  const T Fy0 = J.y0, Fy1 = J.y1, Fy3 = J.y3, Fy4 = J.y4;
  const T Fz0 = J.z0, Fz1 = J.z1, Fz3 = J.z3, Fz4 = J.z4, Fz5 = J.z5;
  const T Ff0 = J.f0, Ff1 = J.f1, Ff3 = J.f3, Ff4 = J.f4;
  T Wx[6], Wy[6], Wz[6], Wf[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T c0 = C[ix(i, 0)], c1 = C[ix(i, 1)], c2 = C[ix(i, 2)], c3 = C[ix(i, 3)], c4 = C[ix(i, 4)], c5 = C[ix(i, 5)];
    Wx[i] = Fx0 * c0 + Fx1 * c1 + Fx3 * c3 + Fx4 * c4;
    Wy[i] = Fy0 * c0 + Fy1 * c1 + Fy3 * c3 + Fy4 * c4;
    Wz[i] = Fz0 * c0 + Fz1 * c1 + c2 + Fz3 * c3 + Fz4 * c4 + Fz5 * c5;
    Wf[i] = Ff0 * c0 + Ff1 * c1 + Ff3 * c3 + Ff4 * c4;
  }
  Pt[ix(0, 0)] = Fx0 * Wx[0] + Fx1 * Wx[1] + Fx3 * Wx[3] + Fx4 * Wx[4];
  Pt[ix(1, 0)] = Fy0 * Wx[0] + Fy1 * Wx[1] + Fy3 * Wx[3] + Fy4 * Wx[4];
  Pt[ix(1, 1)] = Fy0 * Wy[0] + Fy1 * Wy[1] + Fy3 * Wy[3] + Fy4 * Wy[4];
  Pt[ix(2, 0)] = Fz0 * Wx[0] + Fz1 * Wx[1] + Wx[2] + Fz3 * Wx[3] + Fz4 * Wx[4] + Fz5 * Wx[5];
  Pt[ix(2, 1)] = Fz0 * Wy[0] + Fz1 * Wy[1] + Wy[2] + Fz3 * Wy[3] + Fz4 * Wy[4] + Fz5 * Wy[5];
  Pt[ix(2, 2)] = Fz0 * Wz[0] + Fz1 * Wz[1] + Wz[2] + Fz3 * Wz[3] + Fz4 * Wz[4] + Fz5 * Wz[5];
  Pt[ix(3, 0)] = Wx[3];
  Pt[ix(3, 1)] = Wy[3];
  Pt[ix(3, 2)] = Wz[3];
  Pt[ix(3, 3)] = C[ix(3, 3)];
  Pt[ix(4, 0)] = Ff0 * Wx[0] + Ff1 * Wx[1] + Ff3 * Wx[3] + Ff4 * Wx[4];
  Pt[ix(4, 1)] = Ff0 * Wy[0] + Ff1 * Wy[1] + Ff3 * Wy[3] + Ff4 * Wy[4];
  Pt[ix(4, 2)] = Ff0 * Wz[0] + Ff1 * Wz[1] + Ff3 * Wz[3] + Ff4 * Wz[4];
  Pt[ix(4, 3)] = Ff0 * C[ix(0, 3)] + Ff1 * C[ix(1, 3)] + Ff3 * C[ix(3, 3)] + Ff4 * C[ix(4, 3)];
  Pt[ix(4, 4)] = Ff0 * Wf[0] + Ff1 * Wf[1] + Ff3 * Wf[3] + Ff4 * Wf[4];
  Pt[ix(5, 0)] = Wx[5];
  Pt[ix(5, 1)] = Wy[5];
  Pt[ix(5, 2)] = Wz[5];
  Pt[ix(5, 3)] = C[ix(5, 3)];
  Pt[ix(5, 4)] = Wf[5];
  Pt[ix(5, 5)] = C[ix(5, 5)];
}

// d: sin and cos of the direction angles of p on entry, of q on return.
template <class T>
__device__ __forceinline__ uint32_t propagate_r(const T p[6], const T C[21], DirT<T>& d, T rk, T b, T q[6], T Pt[21]) {
  CylJac<T> J;
  const uint32_t st = helix_to_cylinder(p, d, rk, b, q, J);
  transport_cylinder(J, C, Pt);
  return st;
}



// ----------------------------------------------------------------------------
// The Cholesky factor of a 3x3 residual covariance S = L L^T, kept as L's
// off-diagonal entries and the reciprocals of its diagonal.  Its pivots
// d0 = S00, d1 = S11 - l10^2 and d2 = S22 - l20^2 - l21^2 are the ratios of
// consecutive leading minors of S, so they are all positive exactly when S
// passes Sylvester's criterion (pd).  solve: y = L^-1 x.
template <class T>
struct Chol3 {
  T l10, l20, l21, i0, i1, i2;
  bool pd;
  __device__ __forceinline__ void solve(T x0, T x1, T x2, T& y0, T& y1, T& y2) const {
    y0 = x0 * i0;
    y1 = (x1 - l10 * y0) * i1;
    y2 = (x2 - l20 * y0 - l21 * y1) * i2;
  }
};
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }  // 1 ulp
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }
template <class T>
__device__ __forceinline__ Chol3<T> chol3(T S00, T S10, T S11, T S20, T S21, T S22) {
  Chol3<T> c;
  c.i0 = rsqrt_t(S00);
  c.l10 = S10 * c.i0;
  c.l20 = S20 * c.i0;
  const T d1 = S11 - c.l10 * c.l10;
  c.i1 = rsqrt_t(d1);
  c.l21 = (S21 - c.l20 * c.l10) * c.i1;
  const T d2 = S22 - c.l20 * c.l20 - c.l21 * c.l21;
  c.i2 = rsqrt_t(d2);
  c.pd = (S00 > T(0)) & (d1 > T(0)) & (d2 > T(0));
  return c;
}

// Kalman update with a 3D position hit m, covariance V (packed 6), H = [I3|0]:
//   r = m - q_xyz, S = Pt_xyz + V, K = Pt_{:,xyz} S^-1,
//   q' = q + K r, P' = Pt - K Pt_{xyz,:}, chi2 = r^T S^-1 r.
// ZROW (planes: the z row/column of Pt is known to be zero, which removes
// one column from every product): S^-1 from the symmetric cofactors over
// det S, S passing Sylvester's criterion (S00 > 0, leading 2x2 minor > 0,
// det > 0).  Otherwise (cylinders) through the Cholesky factor S = L L^T:
// with W = Pt_{:,xyz} L^-T (row i: L^-1 times column i of Pt's xyz rows) and
// z = L^-1 r, K r = W z, K Pt_{xyz,:} = W W^T and chi2 = |z|^2 -- no gain
// matrix, and a symmetric correction by construction (about 35 fewer
// instructions than the cofactor form's dense 6x3 gain).
// Branch-free: every lane computes the whole update; q, Pt always receive the
// updated values and the returned status bits (0 on success) say whether they
// may be used.  The checks come in a fixed order: non-finite r or S, then S
// not positive definite, then a non-finite result.
template <bool ZROW, class T>
__device__ __forceinline__ uint32_t update_f32(T q[6], T Pt[21], const T m[3], const T V[6], T& dchi) {
  const T r0 = m[0] - q[0], r1 = m[1] - q[1], r2 = m[2] - q[2];
  const T S00 = Pt[0] + V[0], S10 = Pt[1] + V[1], S11 = Pt[2] + V[2];
  const T S20 = Pt[3] + V[3], S21 = Pt[4] + V[4], S22 = Pt[5] + V[5];
  const bool in_ok = fin(r0) & fin(r1) & fin(r2) & fin(S00) & fin(S10) & fin(S11) & fin(S20) & fin(S21) & fin(S22);
  bool pd;
  // cylinders in FP32 through the Cholesky factor; planes, and the FP64 form
  // (where each of the factor's three pivots would cost an IEEE square root
  // and division against the cofactor form's one division), by cofactors
  if constexpr (ZROW || !std::is_same<T, float>::value) {
    const T c00 = S11 * S22 - S21 * S21;
    const T c10 = S20 * S21 - S10 * S22;
    const T c11 = S00 * S22 - S20 * S20;
    const T c20 = S10 * S21 - S11 * S20;
    const T c21 = S10 * S20 - S00 * S21;
    const T c22 = S00 * S11 - S10 * S10;
    const T det = S00 * c00 + S10 * c10 + S20 * c20;
    pd = (S00 > 0.0f) & (c22 > 0.0f) & (det > 0.0f);
    const T rdet = rcp_t(det);
    const T i00 = c00 * rdet, i10 = c10 * rdet, i11 = c11 * rdet;
    const T i20 = c20 * rdet, i21 = c21 * rdet, i22 = c22 * rdet;
    // t = S^-1 r
    const T t0 = i00 * r0 + i10 * r1 + i20 * r2;
    const T t1 = i10 * r0 + i11 * r1 + i21 * r2;
    const T t2 = i20 * r0 + i21 * r1 + i22 * r2;
    dchi = r0 * t0 + r1 * t1 + r2 * t2;
    if constexpr (ZROW) {
      // row/column 2 of Pt vanish: K_i = Pt_i0 S^-1_0: + Pt_i1 S^-1_1:
      T K0[6], K1[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        if (i == 2) continue;
        const T a = Pt[ix(i, 0)], c = Pt[ix(i, 1)];
        K0[i] = a * i00 + c * i10;
        K1[i] = a * i10 + c * i11;
      }
      T Pn[21];
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
          Pn[ix(i, j)] = (i == 2 || j == 2) ? T(0) : Pt[ix(i, j)] - K0[i] * Pt[ix(0, j)] - K1[i] * Pt[ix(1, j)];
#pragma unroll
      for (int i = 0; i < 6; ++i)
        if (i != 2) q[i] = q[i] + Pt[ix(i, 0)] * t0 + Pt[ix(i, 1)] * t1;
#pragma unroll
      for (int i = 0; i < 21; ++i) Pt[i] = Pn[i];
    } else {
      T K0[6], K1[6], K2[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const T a = Pt[ix(i, 0)], c = Pt[ix(i, 1)], d = Pt[ix(i, 2)];
        K0[i] = a * i00 + c * i10 + d * i20;
        K1[i] = a * i10 + c * i11 + d * i21;
        K2[i] = a * i20 + c * i21 + d * i22;
      }
      T Pn[21];
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
          Pn[ix(i, j)] = Pt[ix(i, j)] - K0[i] * Pt[ix(0, j)] - K1[i] * Pt[ix(1, j)] - K2[i] * Pt[ix(2, j)];
#pragma unroll
      for (int i = 0; i < 6; ++i) q[i] = q[i] + Pt[ix(i, 0)] * t0 + Pt[ix(i, 1)] * t1 + Pt[ix(i, 2)] * t2;
#pragma unroll
      for (int i = 0; i < 21; ++i) Pt[i] = Pn[i];
    }
  } else {
    const Chol3<T> L = chol3(S00, S10, S11, S20, S21, S22);
    pd = L.pd;
    T z0, z1, z2;
    L.solve(r0, r1, r2, z0, z1, z2);
    dchi = z0 * z0 + z1 * z1 + z2 * z2;
    T W0[6], W1[6], W2[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) L.solve(Pt[ix(i, 0)], Pt[ix(i, 1)], Pt[ix(i, 2)], W0[i], W1[i], W2[i]);
    T Pn[21];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) Pn[ix(i, j)] = Pt[ix(i, j)] - W0[i] * W0[j] - W1[i] * W1[j] - W2[i] * W2[j];
#pragma unroll
    for (int i = 0; i < 6; ++i) q[i] = q[i] + W0[i] * z0 + W1[i] * z1 + W2[i] * z2;
#pragma unroll
    for (int i = 0; i < 21; ++i) Pt[i] = Pn[i];
  }
  bool out_ok = fin(dchi);
#pragma unroll
  for (int i = 0; i < 6; ++i) out_ok = out_ok & fin(q[i]) & fin(Pt[ix(i, i)]);
  return !in_ok ? S_NONFINITE : (!pd ? S_NOT_PD : (!out_ok ? S_NONFINITE : 0u));
}

// The precision form: S, S^-1, the gain and the state update in FP64; the
// covariance update in FP64 too, in plain form or, with JOSEPH, as
//   P' = (I - K H) Pt (I - K H)^T + K V K^T
// (symmetric and positive semi-definite by construction).  Bulk state stays FP32.
template <bool JOSEPH, bool ZROW, class T>
__device__ __forceinline__ uint32_t update_f64(T q[6], T Pt[21], const T m[3], const T V[6], T& dchi) {
  // Pt's entries in double; ZROW (planes): row and column 2 are zero, as
  // constants, so that every term they enter drops out at compile time
  auto pt = [&](int i, int j) -> double { return (ZROW && (i == 2 || j == 2)) ? 0.0 : (double)Pt[ix(i, j)]; };
  const double r0 = (double)m[0] - (double)q[0], r1 = (double)m[1] - (double)q[1], r2 = (double)m[2] - (double)q[2];
  const double S00 = pt(0, 0) + V[0], S10 = pt(1, 0) + V[1], S11 = pt(1, 1) + V[2];
  const double S20 = pt(2, 0) + V[3], S21 = pt(2, 1) + V[4], S22 = pt(2, 2) + V[5];
  const bool in_ok = fin(r0) & fin(r1) & fin(r2) & fin(S00) & fin(S10) & fin(S11) & fin(S20) & fin(S21) & fin(S22);
  const double c00 = S11 * S22 - S21 * S21;
  const double c10 = S20 * S21 - S10 * S22;
  const double c11 = S00 * S22 - S20 * S20;
  const double c20 = S10 * S21 - S11 * S20;
  const double c21 = S10 * S20 - S00 * S21;
  const double c22 = S00 * S11 - S10 * S10;
  const double det = S00 * c00 + S10 * c10 + S20 * c20;
  const bool pd = (S00 > 0.0) & (c22 > 0.0) & (det > 0.0);
  const double rdet = 1.0 / det;
  const double i00 = c00 * rdet, i10 = c10 * rdet, i11 = c11 * rdet;
  const double i20 = c20 * rdet, i21 = c21 * rdet, i22 = c22 * rdet;
  const double t0 = i00 * r0 + i10 * r1 + i20 * r2;
  const double t1 = i10 * r0 + i11 * r1 + i21 * r2;
  const double t2 = i20 * r0 + i21 * r1 + i22 * r2;
  const double chi = r0 * t0 + r1 * t1 + r2 * t2;
  double K0[6], K1[6], K2[6];
  T qn[6], Pn[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double a = pt(i, 0), c = pt(i, 1), d = pt(i, 2);
    K0[i] = a * i00 + c * i10 + d * i20;
    K1[i] = a * i10 + c * i11 + d * i21;
    K2[i] = a * i20 + c * i21 + d * i22;
    qn[i] = (T)((double)q[i] + a * t0 + c * t1 + d * t2);
  }
  if (!JOSEPH) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j)
        Pn[ix(i, j)] = (T)(pt(i, j) - K0[i] * pt(0, j) - K1[i] * pt(1, j) - K2[i] * pt(2, j));
  } else {
    const double v00 = V[0], v10 = V[1], v11 = V[2], v20 = V[3], v21 = V[4], v22 = V[5];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      // row i of M = Pt - K Pt_{xyz,:}, then (M - K V)_{i,0:3}
      double M[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) M[j] = pt(i, j) - K0[i] * pt(0, j) - K1[i] * pt(1, j) - K2[i] * pt(2, j);
      const double e0 = M[0] - (K0[i] * v00 + K1[i] * v10 + K2[i] * v20);
      const double e1 = M[1] - (K0[i] * v10 + K1[i] * v11 + K2[i] * v21);
      const double e2 = M[2] - (K0[i] * v20 + K1[i] * v21 + K2[i] * v22);
#pragma unroll
      for (int j = 0; j <= i; ++j) Pn[ix(i, j)] = (T)(M[j] - e0 * K0[j] - e1 * K1[j] - e2 * K2[j]);
    }
  }
  dchi = (T)chi;
  bool out_ok = fin(dchi);
#pragma unroll
  for (int i = 0; i < 6; ++i) out_ok = out_ok & fin(qn[i]) & fin(Pn[ix(i, i)]);
#pragma unroll
  for (int i = 0; i < 6; ++i) q[i] = qn[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) Pt[i] = Pn[i];
  return !in_ok ? S_NONFINITE : (!pd ? S_NOT_PD : (!out_ok ? S_NONFINITE : 0u));
}

// precision variants of the update
enum { PREC_F32 = 0, PREC_F64 = 1, PREC_F64_JOSEPH = 2 };

template <int GEOM, int PREC, class T>
__device__ __forceinline__ uint32_t update(T q[6], T Pt[21], const T m[3], const T V[6], T& dchi) {
  if (PREC == PREC_F32) return update_f32<GEOM == 0, T>(q, Pt, m, V, dchi);
  if (PREC == PREC_F64) return update_f64<false, GEOM == 0, T>(q, Pt, m, V, dchi);
  return update_f64<true, GEOM == 0, T>(q, Pt, m, V, dchi);
}

// ZIN (planes): C has the zero z row and column a plane update leaves.
template <int GEOM, bool ZIN, class T>
__device__ __forceinline__ uint32_t propagate(const T p[6], const T C[21], DirT<T>& d, T target, T b, T q[6],
                                              T Pt[21]) {
  if (GEOM == 0) {
    // a track parallel to the planes (theta within 1e-6 rad of pi/2) never
    // reaches one; theta does not change on the way, so the entering cosine decides
    const uint32_t f = fabs_t(d.ct) < T(1e-6) ? S_NO_CROSSING : 0u;
    propagate_z<ZIN, T>(p, C, d, target, b, q, Pt);
    return f;
  }
  return propagate_r<T>(p, C, d, target, b, q, Pt);
}

}  // namespace kf
