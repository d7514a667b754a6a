// FP64 CPU oracle for the batched Kalman-filter step: propagate each track's
// helix to the next endcap plane (fixed z) or barrel cylinder (fixed r) in a
// uniform solenoid field, transport its covariance with the propagation
// Jacobian, and update the state with a 3D hit (Sec. 3, "Description of
// algorithm", steps 1 and 2; Sec. 3.2, "Computations and data structure").
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no code, header
// or constant table with the GPU library; the two meet only through the
// seeded synthetic inputs.
//
// It is written to be checked by eye, not to be fast:
//   * full 6x6 and 3x3 matrices, plain triple loops, no use of sparsity;
//   * the propagation map is the helix definition written out, and its
//     Jacobian F is obtained by forward-mode differentiation (dual numbers)
//     of that map, so no hand-derived derivative enters the oracle;
//   * the cylinder crossing is the closed-form circle/circle intersection
//     (the first positive crossing), i.e. the exact point that the paper's
//     iterative propagation converges to;
//   * the update is the textbook Kalman update with measurement matrix
//     H = [I3 | 0] (optionally in Joseph form);
//   * one template over the scalar type gives the FP64 reference, an FP32
//     build used only to calibrate tolerances, and nested dual numbers for
//     the reference gradient of the summed chi-square.
//
// Conventions (the paper gives none; these are the readings this project
// takes):
//   p = (x, y, z, kappa = q/pT, phi, theta), cm / GeV / rad; Bz in tesla.
//   Transverse curvature omega = -b * kappa with b = 0.00299792458 * Bz, so
//   d(phi)/ds = omega along the transverse arc length s.
//   Covariances are exchanged as packed lower triangles, row-major:
//   element (i, j), i >= j, sits at i*(i+1)/2 + j (21 entries for 6x6,
//   6 for 3x3: xx, yx, yy, zx, zy, zz).
//   Per-track status: bit 0 non-finite value, bit 1 residual covariance not
//   positive definite, bit 2 surface not reachable (a cylinder beyond the
//   helix's reach, or a plane parallel to the track's direction), bit 3 the
//   method's crossing search (at most five Newton steps) ends off the
//   cylinder or on a crossing other than the first ahead (see
//   newton_crossing_f32); bits 16..31 hold the number of layers applied.  A
//   track stops at its first failing layer and keeps the state from before
//   that layer.  Within a layer the checks run in this order: surface
//   reachable; the crossing search lands on the first crossing; hit,
//   propagated state and Jacobian
//   finite; residual covariance positive definite; updated state finite.
//   Process noise is zero (no material effects).

#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace kfo {

using std::sin; using std::cos; using std::tan; using std::sqrt;
using std::atan2; using std::asin; using std::fabs; using std::isfinite;

constexpr double kCLight = 0.00299792458;
constexpr double kPi = 3.14159265358979323846;

enum : uint32_t { ST_NONFINITE = 1u, ST_NOT_PD = 2u, ST_NO_CROSSING = 4u, ST_NEWTON_RESIDUAL = 8u };

// ---------------------------------------------------------------- dual numbers
// a + sum_i d_i eps_i with eps_i eps_j = 0: exact first derivatives.
template <class T, int N>
struct Dual {
  T v;
  std::array<T, N> d;
  Dual() : v(0.0) { d.fill(T(0.0)); }
  Dual(double c) : v(c) { d.fill(T(0.0)); }
  Dual(const T& c, int) : v(c) { d.fill(T(0.0)); }
};

inline double val(double x) { return x; }
inline double val(float x) { return x; }
template <class T, int N> double val(const Dual<T, N>& x) { return val(x.v); }

inline bool finite_all(double x) { return std::isfinite(x); }
inline bool finite_all(float x) { return std::isfinite(x); }
template <class T, int N> bool finite_all(const Dual<T, N>& x) {
  if (!finite_all(x.v)) return false;
  for (int i = 0; i < N; ++i) if (!finite_all(x.d[i])) return false;
  return true;
}

template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r;
}
template <class T, int N> Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r;
}
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r;
}
template <class T, int N> Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <class T, int N> Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
template <class T, int N> Dual<T, N> operator+(const Dual<T, N>& a, double b) { Dual<T, N> r = a; r.v = a.v + b; return r; }
template <class T, int N> Dual<T, N> operator+(double a, const Dual<T, N>& b) { return b + a; }
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a, double b) { Dual<T, N> r = a; r.v = a.v - b; return r; }
template <class T, int N> Dual<T, N> operator-(double a, const Dual<T, N>& b) { return -b + a; }
template <class T, int N> Dual<T, N> operator*(const Dual<T, N>& a, double b) {
  Dual<T, N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r;
}
template <class T, int N> Dual<T, N> operator*(double a, const Dual<T, N>& b) { return b * a; }
template <class T, int N> Dual<T, N> operator/(const Dual<T, N>& a, double b) {
  Dual<T, N> r; r.v = a.v / b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / b; return r;
}
template <class T, int N> Dual<T, N> operator/(double a, const Dual<T, N>& b) { return Dual<T, N>(a) / b; }

// chain rule: f(a) with f' evaluated at a.v
template <class T, int N, class D>
Dual<T, N> chain(const Dual<T, N>& a, const T& fv, const D& dfv) {
  Dual<T, N> r; r.v = fv; for (int i = 0; i < N; ++i) r.d[i] = dfv * a.d[i]; return r;
}
template <class T, int N> Dual<T, N> sin(const Dual<T, N>& a) { return chain(a, T(sin(a.v)), T(cos(a.v))); }
template <class T, int N> Dual<T, N> cos(const Dual<T, N>& a) { return chain(a, T(cos(a.v)), T(-sin(a.v))); }
template <class T, int N> Dual<T, N> tan(const Dual<T, N>& a) {
  T c = cos(a.v); return chain(a, T(tan(a.v)), T(1.0 / (c * c)));
}
template <class T, int N> Dual<T, N> sqrt(const Dual<T, N>& a) {
  T s = sqrt(a.v); return chain(a, s, T(0.5 / s));
}
template <class T, int N> Dual<T, N> asin(const Dual<T, N>& a) {
  return chain(a, T(asin(a.v)), T(1.0 / sqrt(1.0 - a.v * a.v)));
}
template <class T, int N> Dual<T, N> atan2(const Dual<T, N>& y, const Dual<T, N>& x) {
  Dual<T, N> r; r.v = atan2(y.v, x.v);
  T den = x.v * x.v + y.v * y.v;
  for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
  return r;
}

// ------------------------------------------------------------- linear algebra
template <class S> using V3 = std::array<S, 3>;
template <class S> using V6 = std::array<S, 6>;
template <class S> using M3 = std::array<std::array<S, 3>, 3>;
template <class S> using M6 = std::array<std::array<S, 6>, 6>;

enum { IX = 0, IY = 1, IZ = 2, IK = 3, IPHI = 4, ITH = 5 };

inline int pk(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

template <class S, size_t R, size_t K, size_t C>
std::array<std::array<S, C>, R> matmul(const std::array<std::array<S, K>, R>& a,
                                       const std::array<std::array<S, C>, K>& b) {
  std::array<std::array<S, C>, R> r;
  for (size_t i = 0; i < R; ++i)
    for (size_t j = 0; j < C; ++j) {
      S acc(0.0);
      for (size_t l = 0; l < K; ++l) acc = acc + a[i][l] * b[l][j];
      r[i][j] = acc;
    }
  return r;
}

template <class S, size_t R, size_t C>
std::array<std::array<S, R>, C> transpose(const std::array<std::array<S, C>, R>& a) {
  std::array<std::array<S, R>, C> r;
  for (size_t i = 0; i < R; ++i) for (size_t j = 0; j < C; ++j) r[j][i] = a[i][j];
  return r;
}

// ------------------------------------------------------------------- the helix
// sin(u)/u; for |u| < 1e-2 its Taylor series through u^8 (same function to
// double rounding, and free of the 0/0 at u = 0).
template <class S> S sinc(const S& u) {
  if (fabs(val(u)) < 1e-2) {
    S u2 = u * u;
    return 1.0 - u2 / 6.0 * (1.0 - u2 / 20.0 * (1.0 - u2 / 42.0 * (1.0 - u2 / 72.0)));
  }
  return sin(u) / u;
}

// The helix after transverse arc length s (Sec. 3: a charged particle in a
// constant field travels on a helix).  Direction angle phi(s) = phi0 + omega*s;
// x(s) - x0 = integral_0^s cos(phi(t)) dt = s * sinc(omega*s/2) * cos(phi0 + omega*s/2)
// (product-to-sum identity), likewise y with sin; z(s) = z0 + s*cot(theta).
// kappa and theta are constants of motion.
template <class S> V6<S> helix_at(const V6<S>& p, const S& s, double b) {
  S om = -b * p[IK];
  S u = 0.5 * om * s;
  S a = p[IPHI] + u;
  S chord = s * sinc(u);
  V6<S> q = p;
  q[IX] = p[IX] + chord * cos(a);
  q[IY] = p[IY] + chord * sin(a);
  q[IZ] = p[IZ] + s / tan(p[ITH]);
  q[IPHI] = p[IPHI] + om * s;
  return q;
}

// Propagate to the endcap plane z = zk (the "propagation to z" benchmark):
// the helix reaches it after s = (zk - z0) * tan(theta).  A track whose
// direction is parallel to the planes never reaches one; the reading taken
// here is that a plane is out of reach when |cos theta| < 1e-6 (within 1e-6
// rad of theta = pi/2, where reaching a plane 1 cm away takes 10 km of
// transverse path).
constexpr double kPlaneCosMin = 1e-6;
template <class S> V6<S> to_plane(const V6<S>& p, double zk, double b, uint32_t& flags) {
  if (!(fabs(std::cos(val(p[ITH]))) >= kPlaneCosMin)) { flags |= ST_NO_CROSSING; return p; }
  S s = (zk - p[IZ]) * tan(p[ITH]);
  return helix_at(p, s, b);
}

// The method's own cylinder-crossing search (Sec. 3.2: the barrel
// propagation is iterative), as the FP32 path runs it: Newton's method on
// g(s) = x(s)^2 + y(s)^2 - rk^2, g'(s) = 2 (x(s) cos phi(s) + y(s) sin phi(s)).
// The start is the first positive root of g's second-order expansion
// g(0) + 2 beta s + a s^2 with beta = x cos(phi) + y sin(phi),
// gam = y cos(phi) - x sin(phi) and a = 1 + omega gam (clamped to >= 1/2), in
// forms free of cancellation: from inside the cylinder (g(0) < 0) the positive
// root -g(0) / (beta + sqrt(beta^2 - a g(0))), from outside (g(0) > 0, moving
// inward) the near root g(0) / (sqrt(beta^2 - a g(0)) - beta); when that
// denominator is not positive, the straight line's crossing
// -beta + sqrt(beta^2 - g(0)) (square roots' arguments clamped at zero).
// Then at most five Newton steps, stopping after a step that moves s by no
// more than 1e-5 |s| and by no more than a tenth of the step before it (the
// quadratic regime, where the next step would be some 1e-7 of s at most;
// next to a double root the error only halves per step and all five steps
// run).  The oracle's crossing is the closed form below; this
// search only decides status bit 3 (its last iterate is off the cylinder:
// |g| > 1e-4 rk^2, which happens only next to a tangent crossing, where the
// root is nearly double, Newton's method slows down and all five steps run),
// or the iterate is not the first crossing: there g'(s) has the opposite sign
// to g(0) (g rises through zero from inside the cylinder and falls through it
// from outside), it lies ahead (s > 0) and the helix has not yet completed a
// turn (|omega s| < 2 pi); an iterate where any fails is another crossing (a
// strongly curved track entering a cylinder, whose second-order start lies
// past the first crossing and whose steps may run on to a crossing behind
// the track, or one that loops round and enters again).  It runs in single precision, the precision of
// the FP32 path whose flag it mirrors.  Returns the last iterate; *rel =
// |g| / rk^2 there; *steps (if not NULL) the number of Newton steps taken;
// *first (if not NULL) whether the iterate is the first crossing.
inline float newton_crossing_f32(double xd, double yd, double kappa, double phid, double rkd, double bd,
                                 float* rel, int* steps = nullptr, bool* first = nullptr) {
  const float x = float(xd), y = float(yd), phi = float(phid), rk = float(rkd);
  const float om = -float(bd) * float(kappa);
  const float c0 = std::cos(phi), s0 = std::sin(phi);
  const float beta = x * c0 + y * s0;
  const float gam = y * c0 - x * s0;
  const float rk2 = rk * rk;
  const float g0 = x * x + y * y - rk2;
  const float a = std::max(1.0f + om * gam, 0.5f);
  const float sq = std::sqrt(std::max(beta * beta - a * g0, 0.0f));
  const bool inward = g0 > 0.0f;
  const float den = inward ? sq - beta : beta + sq;
  float s = den > 0.0f ? (inward ? g0 : -g0) / den : -beta + std::sqrt(std::max(beta * beta - g0, 0.0f));
  float X = x, Y = y, cph = c0, sph = s0;
  auto point = [&](float t) {
    const float u = 0.5f * om * t;
    const float sincu = u == 0.0f ? 1.0f : std::sin(u) / u;
    X = x + t * sincu * std::cos(phi + u);
    Y = y + t * sincu * std::sin(phi + u);
    cph = std::cos(phi + om * t);
    sph = std::sin(phi + om * t);
  };
  int it = 0;
  float prev = 0.0f;  // the step before (none yet: no stop after the first)
  while (it < 5) {
    point(s);
    const float g = X * X + Y * Y - rk2;
    const float gp = 2.0f * (X * cph + Y * sph);
    const float ds = g / gp;
    s = s - ds;
    ++it;
    if (std::fabs(ds) <= 1e-5f * std::fabs(s) && std::fabs(ds) <= 0.1f * std::fabs(prev)) break;
    prev = ds;
  }
  if (steps) *steps = it;
  point(s);
  *rel = std::fabs(X * X + Y * Y - rk2) / rk2;
  const float gs = X * cph + Y * sph;
  if (first) *first = (g0 > 0.0f ? gs < 0.0f : gs > 0.0f) && s > 0.0f && std::fabs(om * s) < 6.2831853f;
  return s;
}
// Next to tangency five steps leave a residual of 2.0e-4 .. 2.3e-4 rk^2 (the
// error only halves per step at a nearly double root); the threshold sits a
// factor 2 below that cluster, and 4x above the 2.2e-5 of a crossing 1e-3
// from tangency, so that two single-precision evaluations of the search take
// the same decision.
constexpr float kNewtonResidualMax = 1e-4f;

// Propagate to the barrel cylinder r = rk (the "propagation to r" benchmark):
// the first crossing at s > 0.  The transverse circle has centre
// c = (x0 - sin(phi0)/omega, y0 + cos(phi0)/omega) and radius 1/|omega|; the
// point at direction angle psi is c + (sin psi, -cos psi)/omega, so
// |point|^2 = rk^2  <=>  sin(psi - gamma) = omega (rk^2 - |c|^2 - R^2) / (2|c|),
// gamma = atan2(c).  Both roots psi give a family of s spaced by 2 pi/|omega|;
// the smallest positive s wins.  |Q| > 1: the cylinder is out of reach.
template <class S> V6<S> to_cylinder(const V6<S>& p, double rk, double b, uint32_t& flags) {
  S om = -b * p[IK];
  S s;
  if (val(om) == 0.0) {
    S beta = p[IX] * cos(p[IPHI]) + p[IY] * sin(p[IPHI]);
    S disc = beta * beta - (p[IX] * p[IX] + p[IY] * p[IY]) + rk * rk;
    if (!(val(disc) >= 0.0)) { flags |= ST_NO_CROSSING; return p; }
    s = -beta + sqrt(disc);
    if (!(val(s) > 0.0)) { flags |= ST_NO_CROSSING; return p; }
  } else {
    S cx = p[IX] - sin(p[IPHI]) / om;
    S cy = p[IY] + cos(p[IPHI]) / om;
    S d = sqrt(cx * cx + cy * cy);
    S R = val(om) > 0.0 ? 1.0 / om : -1.0 / om;
    S Q = om * (rk * rk - d * d - R * R) / (2.0 * d);
    if (!(fabs(val(Q)) <= 1.0)) { flags |= ST_NO_CROSSING; return p; }
    S gam = atan2(cy, cx);
    S as = asin(Q);
    S period = 2.0 * kPi * R;  // 2 pi / |omega|
    bool have = false;
    for (int root = 0; root < 2; ++root) {
      S psi = root == 0 ? gam + as : gam + kPi - as;
      S t = (psi - p[IPHI]) / om;
      double nper = std::floor(val(t) / val(period));
      t = t - period * nper;
      if (!(val(t) > 0.0)) t = t + period;
      if (!have || val(t) < val(s)) { s = t; have = true; }
    }
  }
  // the crossing exists; flag it if the method's own search misses it (the
  // state returned is still the exact crossing)
  float rel;
  bool first = true;
  newton_crossing_f32(val(p[IX]), val(p[IY]), val(p[IK]), val(p[IPHI]), rk, b, &rel, nullptr, &first);
  if (!(rel <= kNewtonResidualMax) || !first) flags |= ST_NEWTON_RESIDUAL;
  return helix_at(p, s, b);
}

// Propagated state and its Jacobian F = d(propagated p)/d(p), by forward-mode
// differentiation of the propagation map (the path length's dependence on p
// is included automatically).
template <class S>
V6<S> propagate(int geom, const V6<S>& p, double target, double b, M6<S>& F, uint32_t& flags) {
  using D = Dual<S, 6>;
  V6<D> pd;
  for (int i = 0; i < 6; ++i) { pd[i] = D(p[i], 0); pd[i].d[i] = S(1.0); }
  V6<D> q = geom == 0 ? to_plane(pd, target, b, flags) : to_cylinder(pd, target, b, flags);
  V6<S> out;
  for (int i = 0; i < 6; ++i) {
    out[i] = q[i].v;
    for (int j = 0; j < 6; ++j) F[i][j] = q[i].d[j];
  }
  return out;
}

// ------------------------------------------------------------- Kalman update
// Textbook update with a 3D position hit m (covariance V); H = [I3 | 0]
// (Sec. 3.2: a hit has three coordinates and a 3x3 covariance; the update
// needs small products and a 3x3 inverse).
//   r = m - H p;  S = H P H^T + V;  K = P H^T S^-1;
//   p' = p + K r;  P' = (I - K H) P   or, Joseph form,
//   P' = (I - K H) P (I - K H)^T + K V K^T;  chi2 = r^T S^-1 r.
// S must be positive definite (Sylvester's criterion on its leading minors).
template <class S>
bool kalman_update(V6<S>& p, M6<S>& P, const V3<S>& m, const M3<S>& V, bool joseph,
                   S& chi2, uint32_t& flags) {
  V3<S> r;
  M3<S> Sm;
  for (int i = 0; i < 3; ++i) {
    r[i] = m[i] - p[i];
    for (int j = 0; j < 3; ++j) Sm[i][j] = P[i][j] + V[i][j];
  }
  S m1 = Sm[0][0];
  S m2 = Sm[0][0] * Sm[1][1] - Sm[0][1] * Sm[1][0];
  // cofactor matrix; S^-1 = cof^T / det
  M3<S> cof;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      cof[i][j] = Sm[i1][j1] * Sm[i2][j2] - Sm[i1][j2] * Sm[i2][j1];
    }
  S det = Sm[0][0] * cof[0][0] + Sm[0][1] * cof[0][1] + Sm[0][2] * cof[0][2];
  if (!(val(m1) > 0.0 && val(m2) > 0.0 && val(det) > 0.0)) { flags |= ST_NOT_PD; return false; }
  M3<S> Si;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Si[i][j] = cof[j][i] / det;

  std::array<std::array<S, 3>, 6> PHt;  // P H^T = first three columns of P
  for (int i = 0; i < 6; ++i) for (int j = 0; j < 3; ++j) PHt[i][j] = P[i][j];
  std::array<std::array<S, 3>, 6> K = matmul<S, 6, 3, 3>(PHt, Si);
  std::array<std::array<S, 6>, 3> H{};
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 6; ++j) H[i][j] = S(i == j ? 1.0 : 0.0);
  M6<S> KH = matmul<S, 6, 3, 6>(K, H);
  M6<S> A;  // I - K H
  for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) A[i][j] = S(i == j ? 1.0 : 0.0) - KH[i][j];

  V6<S> pn;
  for (int i = 0; i < 6; ++i) {
    S acc = p[i];
    for (int j = 0; j < 3; ++j) acc = acc + K[i][j] * r[j];
    pn[i] = acc;
  }
  M6<S> Pn;
  if (!joseph) {
    Pn = matmul<S, 6, 6, 6>(A, P);
  } else {
    M6<S> APA = matmul<S, 6, 6, 6>(matmul<S, 6, 6, 6>(A, P), transpose<S, 6, 6>(A));
    std::array<std::array<S, 3>, 6> KV = matmul<S, 6, 3, 3>(K, V);
    M6<S> KVK = matmul<S, 6, 3, 6>(KV, transpose<S, 6, 3>(K));
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Pn[i][j] = APA[i][j] + KVK[i][j];
  }
  S c(0.0);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) c = c + r[i] * Si[i][j] * r[j];
  p = pn;
  P = Pn;
  chi2 = c;
  return true;
}

template <class S, size_t R, size_t C> bool finite_mat(const std::array<std::array<S, C>, R>& a) {
  for (size_t i = 0; i < R; ++i) for (size_t j = 0; j < C; ++j) if (!finite_all(a[i][j])) return false;
  return true;
}
template <class S, size_t N> bool finite_vec(const std::array<S, N>& a) {
  for (size_t i = 0; i < N; ++i) if (!finite_all(a[i])) return false;
  return true;
}

// What the filter passes through on layer k, kept for the smoother: the
// predicted state (before the update), the Jacobian of the propagation into
// layer k, and the filtered state (after the update).
template <class S>
struct LayerRecord {
  V6<S> pred_p;
  M6<S> pred_P;
  M6<S> F;
  V6<S> filt_p;
  M6<S> filt_P;
};

// One track through its layers (Sec. 3.1: propagate the seed to the next
// layer, update with the one hit on that layer, repeat).  rec: NULL, or room
// for nl records (filled for the layers applied).
template <class S>
void run_track(int geom, V6<S>& p, M6<S>& P, const V3<S>* hits, const M3<S>* hcov,
               const double* layers, int nl, double b, bool joseph, S& chi2, uint32_t& status,
               LayerRecord<S>* rec = nullptr) {
  uint32_t flags = 0;
  int done = 0;
  chi2 = S(0.0);
  if (!finite_vec(p) || !finite_mat(P)) flags |= ST_NONFINITE;
  for (int k = 0; k < nl && !flags; ++k) {
    // order of the checks: the surface must be reachable; then every value
    // entering the update must be finite; then S must be positive definite;
    // then the updated state must be finite.
    M6<S> F;
    uint32_t f = 0;
    V6<S> pt = propagate(geom, p, layers[k], b, F, f);
    if (f) { flags |= f; break; }
    if (!finite_vec(hits[k]) || !finite_mat(hcov[k]) || !finite_vec(pt) || !finite_mat(F)) {
      flags |= ST_NONFINITE;
      break;
    }
    M6<S> Pt = matmul<S, 6, 6, 6>(matmul<S, 6, 6, 6>(F, P), transpose<S, 6, 6>(F));
    if (rec) {
      rec[k].pred_p = pt;
      rec[k].pred_P = Pt;
      rec[k].F = F;
    }
    S dchi;
    if (!kalman_update(pt, Pt, hits[k], hcov[k], joseph, dchi, f)) { flags |= f; break; }
    if (!finite_vec(pt) || !finite_mat(Pt) || !finite_all(dchi)) { flags |= ST_NONFINITE; break; }
    if (rec) {
      rec[k].filt_p = pt;
      rec[k].filt_P = Pt;
    }
    p = pt;
    P = Pt;
    chi2 = chi2 + dchi;
    done = k + 1;
  }
  status = flags | (uint32_t(done) << 16);
}

// ------------------------------------------------------------- batch drivers
template <class S, class In>
void load_track(int64_t i, int64_t n, int L, const In* par, const In* cov, const In* hp,
                const In* hc, V6<S>& p, M6<S>& P, V3<S>* m, M3<S>* V) {
  for (int a = 0; a < 6; ++a) p[a] = S(par[i * 6 + a]);
  for (int a = 0; a < 6; ++a) for (int c = 0; c < 6; ++c) P[a][c] = S(cov[i * 21 + pk(a, c)]);
  for (int k = 0; k < L; ++k) {
    for (int a = 0; a < 3; ++a) m[k][a] = S(hp[(k * n + i) * 3 + a]);
    for (int a = 0; a < 3; ++a) for (int c = 0; c < 3; ++c) V[k][a][c] = S(hc[(k * n + i) * 6 + pk(a, c)]);
  }
}

template <class S>
void run_batch(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
               const S* par_in, const S* cov_in, const S* hit_pos, const S* hit_cov, int joseph,
               S* par_out, S* cov_out, S* chi2_out, int32_t* status_out, int nthreads) {
  const double b = kCLight * bz;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    std::vector<V3<S>> m(L > 0 ? L : 1);
    std::vector<M3<S>> V(L > 0 ? L : 1);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      V6<S> p; M6<S> P;
      load_track<S, S>(i, n, L, par_in, cov_in, hit_pos, hit_cov, p, P, m.data(), V.data());
      int nl = nlay ? nlay[i] : L;
      nl = std::max(0, std::min(nl, L));
      S chi2; uint32_t st;
      run_track<S>(geom, p, P, m.data(), V.data(), layers, nl, b, joseph != 0, chi2, st);
      for (int a = 0; a < 6; ++a) par_out[i * 6 + a] = p[a];
      for (int a = 0; a < 6; ++a) for (int c = 0; c <= a; ++c) cov_out[i * 21 + pk(a, c)] = P[a][c];
      if (chi2_out) chi2_out[i] = chi2;
      if (status_out) status_out[i] = int32_t(st);
    }
  }
}

// The filter pass with its per-layer records written out (input to the
// smoother): pred_p, filt_p [L][n][6]; pred_P, filt_P [L][n][21] packed;
// F [L][n][36] row-major.  Records of layers a track did not apply are left
// as they are.  S: the arithmetic (double; float only to size tolerances).
template <class S>
void record_batch(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                  const double* par_in, const double* cov_in, const double* hit_pos, const double* hit_cov,
                  int joseph, double* pred_p, double* pred_P, double* F, double* filt_p, double* filt_P,
                  double* chi2_out, int32_t* status_out, int nthreads) {
  const double b = kCLight * bz;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    std::vector<V3<S>> m(L > 0 ? L : 1);
    std::vector<M3<S>> V(L > 0 ? L : 1);
    std::vector<LayerRecord<S>> rec(L > 0 ? L : 1);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      V6<S> p; M6<S> P;
      load_track<S, double>(i, n, L, par_in, cov_in, hit_pos, hit_cov, p, P, m.data(), V.data());
      int nl = nlay ? nlay[i] : L;
      nl = std::max(0, std::min(nl, L));
      S chi2; uint32_t st;
      run_track<S>(geom, p, P, m.data(), V.data(), layers, nl, b, joseph != 0, chi2, st, rec.data());
      const int done = int(st >> 16);
      for (int k = 0; k < done; ++k) {
        const int64_t o = int64_t(k) * n + i;
        const LayerRecord<S>& r = rec[size_t(k)];
        for (int a = 0; a < 6; ++a) {
          pred_p[o * 6 + a] = double(r.pred_p[a]);
          filt_p[o * 6 + a] = double(r.filt_p[a]);
          for (int c = 0; c < 6; ++c) F[o * 36 + a * 6 + c] = double(r.F[a][c]);
          for (int c = 0; c <= a; ++c) {
            pred_P[o * 21 + pk(a, c)] = double(r.pred_P[a][c]);
            filt_P[o * 21 + pk(a, c)] = double(r.filt_P[a][c]);
          }
        }
      }
      if (chi2_out) chi2_out[i] = double(chi2);
      if (status_out) status_out[i] = int32_t(st);
    }
  }
}

// Hit selection on layers with several candidate hits (the search step of
// track finding that runs between propagation and update, Sec. 3.1): after
// the propagation, every candidate j gets the chi-square a Kalman update
// with it would add; a candidate whose residual covariance is not positive
// definite, or with non-finite values, takes no part.  The candidate with
// the smallest chi-square not above `gate` (the first of equal ones) updates
// the state; if none qualifies the layer is passed without update (a hole)
// and the state is the prediction.  forced (if not NULL): the choice of
// every layer is taken from it instead (-1: a hole) -- used to follow a
// given sequence of choices.  Track failures as in run_track.
// cand_chi2 (if not NULL): [nl][M] each candidate's chi-square, NaN if it
// takes no part; chosen: [nl] the index used, -1 for a hole.
template <class S>
void run_track_gated(int geom, V6<S>& p, M6<S>& P, const V3<S>* cand, const M3<S>* ccov, int M,
                     const double* layers, int nl, double b, double gate, const int32_t* forced,
                     bool joseph, S& chi2, uint32_t& status, int32_t* chosen, double* cand_chi2) {
  uint32_t flags = 0;
  int done = 0;
  chi2 = S(0.0);
  if (!finite_vec(p) || !finite_mat(P)) flags |= ST_NONFINITE;
  for (int k = 0; k < nl && !flags; ++k) {
    M6<S> F;
    uint32_t f = 0;
    V6<S> pt = propagate(geom, p, layers[k], b, F, f);
    if (f) { flags |= f; break; }
    if (!finite_vec(pt) || !finite_mat(F)) { flags |= ST_NONFINITE; break; }
    M6<S> Pt = matmul<S, 6, 6, 6>(matmul<S, 6, 6, 6>(F, P), transpose<S, 6, 6>(F));
    int best = -1;
    double bchi = 0.0;
    for (int j = 0; j < M; ++j) {
      V6<S> q = pt;
      M6<S> Q = Pt;
      S c;
      uint32_t fj = 0;
      const V3<S>& m = cand[size_t(k) * M + j];
      const M3<S>& V = ccov[size_t(k) * M + j];
      const bool ok = finite_vec(m) && finite_mat(V) && kalman_update(q, Q, m, V, false, c, fj) &&
                      finite_all(c);
      if (cand_chi2) cand_chi2[size_t(k) * M + j] = ok ? val(c) : NAN;
      if (ok && val(c) <= gate && (best < 0 || val(c) < bchi)) {
        best = j;
        bchi = val(c);
      }
    }
    if (forced) best = forced[k];
    if (chosen) chosen[k] = best;
    if (best >= 0) {
      S dchi;
      if (!kalman_update(pt, Pt, cand[size_t(k) * M + best], ccov[size_t(k) * M + best], joseph, dchi, f)) {
        flags |= f;
        break;
      }
      if (!finite_vec(pt) || !finite_mat(Pt) || !finite_all(dchi)) { flags |= ST_NONFINITE; break; }
      chi2 = chi2 + dchi;
    }
    p = pt;
    P = Pt;
    done = k + 1;
  }
  status = flags | (uint32_t(done) << 16);
}

// cand_pos [L][n][M][3], cand_cov [L][n][M][6] packed; forced, chosen [L][n];
// cand_chi2 [L][n][M] (or NULL).
template <class S>
void gate_batch(int geom, int64_t n, int L, int M, const double* layers, double bz, const int32_t* nlay,
                const double* par_in, const double* cov_in, const double* cand_pos, const double* cand_cov,
                double gate, const int32_t* forced, int joseph, double* par_out, double* cov_out, double* chi2_out,
                int32_t* status_out, int32_t* chosen_out, double* cand_chi2_out, int nthreads) {
  const double b = kCLight * bz;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    const size_t LM = size_t(L > 0 ? L : 1) * size_t(M);
    std::vector<V3<S>> m(LM);
    std::vector<M3<S>> V(LM);
    std::vector<int32_t> fc(size_t(L > 0 ? L : 1)), ch(size_t(L > 0 ? L : 1));
    std::vector<double> cc(LM);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      V6<S> p; M6<S> P;
      for (int a = 0; a < 6; ++a) p[a] = S(par_in[i * 6 + a]);
      for (int a = 0; a < 6; ++a) for (int c = 0; c < 6; ++c) P[a][c] = S(cov_in[i * 21 + pk(a, c)]);
      for (int k = 0; k < L; ++k) {
        for (int j = 0; j < M; ++j) {
          const int64_t o = (int64_t(k) * n + i) * M + j;
          for (int a = 0; a < 3; ++a) m[size_t(k) * M + j][a] = S(cand_pos[o * 3 + a]);
          for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) V[size_t(k) * M + j][a][c] = S(cand_cov[o * 6 + pk(a, c)]);
        }
        if (forced) fc[size_t(k)] = forced[int64_t(k) * n + i];
      }
      int nl = nlay ? nlay[i] : L;
      nl = std::max(0, std::min(nl, L));
      S chi2; uint32_t st;
      std::fill(cc.begin(), cc.end(), NAN);
      run_track_gated<S>(geom, p, P, m.data(), V.data(), M, layers, nl, b, gate, forced ? fc.data() : nullptr,
                         joseph != 0, chi2, st, ch.data(), cc.data());
      const int done = int(st >> 16);
      for (int a = 0; a < 6; ++a) par_out[i * 6 + a] = double(p[a]);
      for (int a = 0; a < 6; ++a) for (int c = 0; c <= a; ++c) cov_out[i * 21 + pk(a, c)] = double(P[a][c]);
      if (chi2_out) chi2_out[i] = double(chi2);
      if (status_out) status_out[i] = int32_t(st);
      for (int k = 0; k < done; ++k) {
        if (chosen_out) chosen_out[int64_t(k) * n + i] = ch[size_t(k)];
        if (cand_chi2_out)
          for (int j = 0; j < M; ++j) cand_chi2_out[(int64_t(k) * n + i) * M + j] = cc[size_t(k) * M + j];
      }
    }
  }
}

// Reference gradient of sum_i w_i chi2_i with respect to the seed parameters
// and the hit positions, by forward-mode dual numbers through the whole
// chain (the Jacobian's own dependence on p enters through nested duals).
// Instantiated in double (the reference) and in float (only to size the
// tolerance of a float-arithmetic gradient); inputs and outputs are double.
constexpr int kGradChunk = 6;
template <class R>
void grad_batch(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                const double* par_in, const double* cov_in, const double* hit_pos,
                const double* hit_cov, int joseph, const double* w, double* g_hit, double* g_par,
                int nthreads) {
  using D = Dual<R, kGradChunk>;
  const double b = kCLight * bz;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    std::vector<V3<double>> m0(L > 0 ? L : 1);
    std::vector<M3<double>> V0(L > 0 ? L : 1);
    std::vector<V3<D>> m(L > 0 ? L : 1);
    std::vector<M3<D>> V(L > 0 ? L : 1);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
    for (int64_t i = 0; i < n; ++i) {
      V6<double> p0; M6<double> P0;
      load_track<double, double>(i, n, L, par_in, cov_in, hit_pos, hit_cov, p0, P0, m0.data(), V0.data());
      int nl = nlay ? nlay[i] : L;
      nl = std::max(0, std::min(nl, L));
      for (int k = 0; k < L; ++k) for (int a = 0; a < 3; ++a) g_hit[(k * n + i) * 3 + a] = 0.0;
      for (int a = 0; a < 6; ++a) g_par[i * 6 + a] = 0.0;
      const int nin = 6 + 3 * nl;  // inputs: seed parameters, then hit k coordinate a at 6 + 3k + a
      for (int c0 = 0; c0 < nin; c0 += kGradChunk) {
        V6<D> p; M6<D> P;
        for (int a = 0; a < 6; ++a) {
          p[a] = D(R(p0[a]), 0);
          for (int c = 0; c < 6; ++c) P[a][c] = D(R(P0[a][c]), 0);
        }
        for (int k = 0; k < nl; ++k)
          for (int a = 0; a < 3; ++a) {
            m[k][a] = D(R(m0[k][a]), 0);
            for (int c = 0; c < 3; ++c) V[k][a][c] = D(R(V0[k][a][c]), 0);
          }
        for (int c = 0; c < kGradChunk && c0 + c < nin; ++c) {
          int idx = c0 + c;
          if (idx < 6) p[idx].d[c] = R(1.0);
          else m[(idx - 6) / 3][(idx - 6) % 3].d[c] = R(1.0);
        }
        D chi2; uint32_t st;
        run_track<D>(geom, p, P, m.data(), V.data(), layers, nl, b, joseph != 0, chi2, st);
        for (int c = 0; c < kGradChunk && c0 + c < nin; ++c) {
          int idx = c0 + c;
          double g = w[i] * double(chi2.d[c]);
          if (idx < 6) g_par[i * 6 + idx] = g;
          else g_hit[(((idx - 6) / 3) * n + i) * 3 + (idx - 6) % 3] = g;
        }
      }
    }
  }
}

}  // namespace kfo

// ------------------------------------------------------------------ C exports
extern "C" {

int kfo_version(void) { return 1; }

// Whole sample through the filter in FP64.  Arrays are host memory, logical
// layout: par [n][6], cov [n][21], hit_pos [L][n][3], hit_cov [L][n][6],
// layers [L] (z for geom 0, r for geom 1), nlay [n] or NULL (= L for all).
int kfo_run_f64(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                const double* par_in, const double* cov_in, const double* hit_pos,
                const double* hit_cov, int joseph, double* par_out, double* cov_out,
                double* chi2_out, int32_t* status_out, int nthreads) {
  if (n < 0 || L < 0 || (geom != 0 && geom != 1)) return 1;
  kfo::run_batch<double>(geom, n, L, layers, bz, nlay, par_in, cov_in, hit_pos, hit_cov, joseph,
                         par_out, cov_out, chi2_out, status_out, nthreads);
  return 0;
}

// The same algorithm instantiated in FP32 (used only to size tolerances).
int kfo_run_f32(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                const float* par_in, const float* cov_in, const float* hit_pos,
                const float* hit_cov, int joseph, float* par_out, float* cov_out,
                float* chi2_out, int32_t* status_out, int nthreads) {
  if (n < 0 || L < 0 || (geom != 0 && geom != 1)) return 1;
  kfo::run_batch<float>(geom, n, L, layers, bz, nlay, par_in, cov_in, hit_pos, hit_cov, joseph,
                        par_out, cov_out, chi2_out, status_out, nthreads);
  return 0;
}

// The filter pass with per-layer records (see record_batch); precision 0:
// double, 1: float arithmetic (tolerance sizing only).
int kfo_filter_record(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                      const double* par_in, const double* cov_in, const double* hit_pos, const double* hit_cov,
                      int joseph, double* pred_p, double* pred_P, double* F, double* filt_p, double* filt_P,
                      double* chi2_out, int32_t* status_out, int precision, int nthreads) {
  if (n < 0 || L < 0 || (geom != 0 && geom != 1)) return 1;
  if (precision == 0)
    kfo::record_batch<double>(geom, n, L, layers, bz, nlay, par_in, cov_in, hit_pos, hit_cov, joseph, pred_p,
                              pred_P, F, filt_p, filt_P, chi2_out, status_out, nthreads);
  else
    kfo::record_batch<float>(geom, n, L, layers, bz, nlay, par_in, cov_in, hit_pos, hit_cov, joseph, pred_p,
                             pred_P, F, filt_p, filt_P, chi2_out, status_out, nthreads);
  return 0;
}

// Filter with hit selection among M candidates per layer (see
// run_track_gated); the chosen candidate's update in Joseph form if joseph;
// precision 0 double, 1 float (tolerance sizing only).
int kfo_gate_run(int geom, int64_t n, int L, int M, const double* layers, double bz, const int32_t* nlay,
                 const double* par_in, const double* cov_in, const double* cand_pos, const double* cand_cov,
                 double gate, const int32_t* forced, int joseph, double* par_out, double* cov_out, double* chi2_out,
                 int32_t* status_out, int32_t* chosen_out, double* cand_chi2_out, int precision, int nthreads) {
  if (n < 0 || L < 0 || M < 1 || (geom != 0 && geom != 1)) return 1;
  if (precision == 0)
    kfo::gate_batch<double>(geom, n, L, M, layers, bz, nlay, par_in, cov_in, cand_pos, cand_cov, gate, forced,
                            joseph, par_out, cov_out, chi2_out, status_out, chosen_out, cand_chi2_out, nthreads);
  else
    kfo::gate_batch<float>(geom, n, L, M, layers, bz, nlay, par_in, cov_in, cand_pos, cand_cov, gate, forced,
                           joseph, par_out, cov_out, chi2_out, status_out, chosen_out, cand_chi2_out, nthreads);
  return 0;
}

// One propagation: p [6] -> p_out [6], F [6][6] row-major, flags.
int kfo_propagate(int geom, const double* p, double target, double bz, double* p_out,
                  double* F_out, uint32_t* flags) {
  kfo::V6<double> q;
  for (int i = 0; i < 6; ++i) q[i] = p[i];
  kfo::M6<double> F;
  uint32_t f = 0;
  kfo::V6<double> r = kfo::propagate(geom, q, target, kfo::kCLight * bz, F, f);
  for (int i = 0; i < 6; ++i) {
    p_out[i] = r[i];
    for (int j = 0; j < 6; ++j) F_out[i * 6 + j] = F[i][j];
  }
  *flags = f;
  return 0;
}

// The method's crossing search on its own (newton_crossing_f32):
// p [6], cylinder radius rk; returns the last iterate s, |g(s)| / rk^2, the
// number of Newton steps taken and whether the iterate is the first crossing.
int kfo_newton_r(const double* p, double rk, double bz, double* s_out, double* rel_out, int32_t* steps_out,
                 int32_t* first_out) {
  float rel = 0.0f;
  int steps = 0;
  bool first = true;
  const float s = kfo::newton_crossing_f32(p[kfo::IX], p[kfo::IY], p[kfo::IK], p[kfo::IPHI], rk,
                                           kfo::kCLight * bz, &rel, &steps, &first);
  *s_out = double(s);
  *rel_out = double(rel);
  if (steps_out) *steps_out = steps;
  if (first_out) *first_out = first ? 1 : 0;
  return 0;
}

// One Kalman update: p [6], P [21] packed, m [3], V [6] packed.
int kfo_update(const double* p, const double* P21, const double* m, const double* V6p, int joseph,
               double* p_out, double* P21_out, double* chi2, uint32_t* flags) {
  kfo::V6<double> q; kfo::M6<double> P; kfo::V3<double> mm; kfo::M3<double> V;
  for (int i = 0; i < 6; ++i) { q[i] = p[i]; for (int j = 0; j < 6; ++j) P[i][j] = P21[kfo::pk(i, j)]; }
  for (int i = 0; i < 3; ++i) { mm[i] = m[i]; for (int j = 0; j < 3; ++j) V[i][j] = V6p[kfo::pk(i, j)]; }
  uint32_t f = 0;
  double c = 0.0;
  bool ok = kfo::kalman_update(q, P, mm, V, joseph != 0, c, f);
  for (int i = 0; i < 6; ++i) { p_out[i] = q[i]; for (int j = 0; j <= i; ++j) P21_out[kfo::pk(i, j)] = P[i][j]; }
  *chi2 = c;
  *flags = f;
  return ok ? 0 : 1;
}

// Reference gradient of sum_i w[i]*chi2_i: g_hit [L][n][3], g_par [n][6].
int kfo_grad_chi2(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                  const double* par_in, const double* cov_in, const double* hit_pos,
                  const double* hit_cov, int joseph, const double* w, double* g_hit,
                  double* g_par, int nthreads) {
  if (n < 0 || L < 0 || (geom != 0 && geom != 1)) return 1;
  kfo::grad_batch<double>(geom, n, L, layers, bz, nlay, par_in, cov_in, hit_pos, hit_cov, joseph, w,
                          g_hit, g_par, nthreads);
  return 0;
}

// The same gradient evaluated in float arithmetic (tolerance sizing only).
int kfo_grad_chi2_f32(int geom, int64_t n, int L, const double* layers, double bz, const int32_t* nlay,
                      const double* par_in, const double* cov_in, const double* hit_pos,
                      const double* hit_cov, int joseph, const double* w, double* g_hit,
                      double* g_par, int nthreads) {
  if (n < 0 || L < 0 || (geom != 0 && geom != 1)) return 1;
  kfo::grad_batch<float>(geom, n, L, layers, bz, nlay, par_in, cov_in, hit_pos, hit_cov, joseph, w,
                         g_hit, g_par, nthreads);
  return 0;
}

}  // extern "C"
