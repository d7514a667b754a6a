// Hand-written adjoint of L = sum_i w_i chi2_i for the filter through planes
// (z) or cylinders (r): dL/d(hit positions) and dL/d(seed parameters) (and
// dL/d(seed covariance)).
//
// One lane per track walks its applied layers backwards.  For layer k it
// needs the state (p, P) that entered the layer -- read from the forward's
// per-layer checkpoint, or recomputed from the seed by re-running layers
// 0..k-1 -- and rebuilds the layer's forward quantities: propagated q, the
// Jacobian F (with dF/dp from dual numbers over the same formulas), Pt =
// F P F^T, S = Pt_xyz + V, S^-1, K = Pt_{:,xyz} S^-1, r = m - q_xyz,
// t = S^-1 r.  With the adjoints (ap, aP) of the state after the layer
// (aP symmetric) and w = dL/dchi2:
//   r_bar = 2 w t + K^T ap                        (= dL/dm_k)
//   q_bar = ap - H^T r_bar
//   S_bar = -w t t^T + K^T aP K - sym((K^T ap) t^T)
//   G     = aP + sym([-2 aP K + ap t^T | 0]) + H^T S_bar H   (adjoint of Pt)
//   aP   <- F^T G F
//   ap   <- F^T q_bar + sum_ij (2 G F P)_ij dF_ij/dp
// where sym(X) = (X + X^T)/2 and H = [I3 | 0].  On cylinders the path length
// s to the crossing depends on p implicitly (x(s)^2 + y(s)^2 = r^2): dual
// numbers take ds/dp = -g_p / g_s at the search's s, which is the forward's
// own Jacobian term, and carry it through the crossing's formulas to dF/dp.
#include "kf_dual.h"
#include "kf_internal.h"
#include "kf_lanes.h"
#include "kf_track.h"

namespace kf {

// sum_l F[l][j] v[l]: column j of the plane Jacobian against v
__device__ __forceinline__ float fcol(const PlaneJac<float>& J, int j, const float v[6]) {
  switch (j) {
    case 0: return v[0];
    case 1: return v[1];
    case 2: return J.a0 * v[0] + J.b0 * v[1] + J.c0 * v[4];
    case 3: return J.a1 * v[0] + J.b1 * v[1] + v[3] + J.c1 * v[4];
    case 4: return J.a2 * v[0] + J.b2 * v[1] + v[4];
    default: return J.a3 * v[0] + J.b3 * v[1] + J.c3 * v[4] + v[5];
  }
}

// sum_l F[i][l] v[l]: row i of the plane Jacobian against v
__device__ __forceinline__ float frow(const PlaneJac<float>& J, int i, const float v[6]) {
  switch (i) {
    case 0: return v[0] + J.a0 * v[2] + J.a1 * v[3] + J.a2 * v[4] + J.a3 * v[5];
    case 1: return v[1] + J.b0 * v[2] + J.b1 * v[3] + J.b2 * v[4] + J.b3 * v[5];
    case 2: return 0.0f;
    case 3: return v[3];
    case 4: return J.c0 * v[2] + J.c1 * v[3] + v[4] + J.c3 * v[5];
    default: return v[5];
  }
}

// The adjoint of the Kalman update with hit (m, V) on the prediction (q, Pt):
// from ap, aP (adjoints of the updated state) to gm = dL/dm, qb (adjoint of
// q) and G (adjoint of Pt, symmetric, as a full 6x6 array).
__device__ __forceinline__ void adjoint_update(const float q[6], const float Pt[21], const float m[3],
                                               const float V[6], float w, const float ap[6], const float aP[21],
                                               float gm[3], float qb[6], float G[6][6]) {
  const float S00 = Pt[0] + V[0], S10 = Pt[1] + V[1], S11 = Pt[2] + V[2];
  const float S20 = Pt[3] + V[3], S21 = Pt[4] + V[4], S22 = Pt[5] + V[5];
  const float c00 = S11 * S22 - S21 * S21, c10 = S20 * S21 - S10 * S22, c11 = S00 * S22 - S20 * S20;
  const float c20 = S10 * S21 - S11 * S20, c21 = S10 * S20 - S00 * S21, c22 = S00 * S11 - S10 * S10;
  const float rdet = rcp(S00 * c00 + S10 * c10 + S20 * c20);
  float Si[3][3];
  Si[0][0] = c00 * rdet;
  Si[1][0] = Si[0][1] = c10 * rdet;
  Si[1][1] = c11 * rdet;
  Si[2][0] = Si[0][2] = c20 * rdet;
  Si[2][1] = Si[1][2] = c21 * rdet;
  Si[2][2] = c22 * rdet;
  float r[3], t[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = m[c] - q[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) t[c] = Si[c][0] * r[0] + Si[c][1] * r[1] + Si[c][2] * r[2];
  float K[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      K[i][c] = Pt[ix(i, 0)] * Si[0][c] + Pt[ix(i, 1)] * Si[1][c] + Pt[ix(i, 2)] * Si[2][c];

  float Kp[3], rb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) acc += K[i][c] * ap[i];
    Kp[c] = acc;
    rb[c] = 2.0f * w * t[c] + acc;
    gm[c] = rb[c];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) qb[i] = ap[i] - (i < 3 ? rb[i] : 0.0f);
  float aPK[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = 0.0f;
#pragma unroll
      for (int l = 0; l < 6; ++l) acc += aP[ix(i, l)] * K[l][c];
      aPK[i][c] = acc;
    }
  float Sb[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c <= a; ++c) {
      float acc = -w * t[a] * t[c] - 0.5f * (Kp[a] * t[c] + t[a] * Kp[c]);
#pragma unroll
      for (int i = 0; i < 6; ++i) acc += K[i][a] * aPK[i][c];
      Sb[a][c] = Sb[c][a] = acc;
    }
  float A[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) A[i][c] = -2.0f * aPK[i][c] + ap[i] * t[c];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float g = aP[ix(i, j)] + 0.5f * ((j < 3 ? A[i][j] : 0.0f) + (i < 3 ? A[j][i] : 0.0f));
      if (i < 3 && j < 3) g += Sb[i][j];
      G[i][j] = G[j][i] = g;
    }
}

// One plane layer backwards (see the file comment).  p, P: state entering
// the layer; m, V: its hit; ap, aP: adjoints of the state leaving the layer
// on entry, of the state entering it on return; gm: dL/dm.
__device__ __forceinline__ void adjoint_layer_z(const float p[6], const float P[21], const float m[3],
                                                const float V[6], float zk, float b, float w, float ap[6],
                                                float aP[21], float gm[3]) {
  // forward quantities, with dF/dp along (z, kappa, phi, theta)
  D4 pd[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) pd[i] = D4(p[i]);
  pd[2].d[0] = 1.0f;
  pd[3].d[1] = 1.0f;
  pd[4].d[2] = 1.0f;
  pd[5].d[3] = 1.0f;
  D4 qd[6];
  PlaneJac<D4> Jd;
  helix_to_plane<D4>(pd, zk, b, qd, Jd);
  const PlaneJac<float> J{Jd.a0.v, Jd.a1.v, Jd.a2.v, Jd.a3.v, Jd.b0.v, Jd.b1.v,
                          Jd.b2.v, Jd.b3.v, Jd.c0.v, Jd.c1.v, Jd.c3.v};
  float Pt[21];
  transport_plane<false>(J, P, Pt);
  float q[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) q[i] = qd[i].v;
  float qb[6], G[6][6];
  adjoint_update(q, Pt, m, V, w, ap, aP, gm, qb, G);

  // adjoint of the transport: aP <- F^T G F, and F_bar = 2 G F P
  float GF[6][6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int j = 0; j < 6; ++j) GF[k][j] = fcol(J, j, G[k]);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float col[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) col[k] = GF[k][j];
      aP[ix(i, j)] = fcol(J, i, col);
    }
  // (F P)[k][j] for j = 2..5, all k
  float FP[6][4];
#pragma unroll
  for (int j = 2; j < 6; ++j) {
    float col[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) col[l] = P[ix(l, j)];
#pragma unroll
    for (int k = 0; k < 6; ++k) FP[k][j - 2] = frow(J, k, col);
  }
  // F_bar on the entries of F that depend on p: rows x, y, phi; columns z..theta
  float Fb[3][4];
  const int rows[3] = {0, 1, 4};
#pragma unroll
  for (int ri = 0; ri < 3; ++ri)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 6; ++k) acc += G[rows[ri]][k] * FP[k][j];
      Fb[ri][j] = 2.0f * acc;
    }

  // adjoint of the propagation
  float apn[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) apn[j] = fcol(J, j, qb);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    apn[2 + d] += Fb[0][0] * Jd.a0.d[d] + Fb[0][1] * Jd.a1.d[d] + Fb[0][2] * Jd.a2.d[d] + Fb[0][3] * Jd.a3.d[d] +
                  Fb[1][0] * Jd.b0.d[d] + Fb[1][1] * Jd.b1.d[d] + Fb[1][2] * Jd.b2.d[d] + Fb[1][3] * Jd.b3.d[d] +
                  Fb[2][0] * Jd.c0.d[d] + Fb[2][1] * Jd.c1.d[d] + Fb[2][3] * Jd.c3.d[d];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) ap[j] = apn[j];
}

// The cylinder Jacobian's rows, as a full matrix:
//   x   = (x0, x1, 0, x3, x4, 0)      y = (y0, y1, 0, y3, y4, 0)
//   z   = (z0, z1, 1, z3, z4, z5)     kappa = e_kappa
//   phi = (f0, f1, 0, f3, f4, 0)      theta = e_theta
// sum_l F[l][j] v[l]: column j against v
__device__ __forceinline__ float fcol_r(const CylJac<float>& J, int j, const float v[6]) {
  switch (j) {
    case 0: return J.x0 * v[0] + J.y0 * v[1] + J.z0 * v[2] + J.f0 * v[4];
    case 1: return J.x1 * v[0] + J.y1 * v[1] + J.z1 * v[2] + J.f1 * v[4];
    case 2: return v[2];
    case 3: return J.x3 * v[0] + J.y3 * v[1] + J.z3 * v[2] + v[3] + J.f3 * v[4];
    case 4: return J.x4 * v[0] + J.y4 * v[1] + J.z4 * v[2] + J.f4 * v[4];
    default: return J.z5 * v[2] + v[5];
  }
}
// sum_l F[i][l] v[l]: row i against v
__device__ __forceinline__ float frow_r(const CylJac<float>& J, int i, const float v[6]) {
  switch (i) {
    case 0: return J.x0 * v[0] + J.x1 * v[1] + J.x3 * v[3] + J.x4 * v[4];
    case 1: return J.y0 * v[0] + J.y1 * v[1] + J.y3 * v[3] + J.y4 * v[4];
    case 2: return J.z0 * v[0] + J.z1 * v[1] + v[2] + J.z3 * v[3] + J.z4 * v[4] + J.z5 * v[5];
    case 3: return v[3];
    case 4: return J.f0 * v[0] + J.f1 * v[1] + J.f3 * v[3] + J.f4 * v[4];
    default: return v[5];
  }
}

// dual directions of the cylinder step: p index of each (z does not enter)
__device__ __forceinline__ constexpr int cyl_dir_par(int d) { return d < 2 ? d : d + 1; }

// One cylinder layer backwards; arguments as adjoint_layer_z, rk the radius.
__device__ __forceinline__ void adjoint_layer_r(const float p[6], const float P[21], const float m[3],
                                                const float V[6], float rk, float b, float w, float ap[6],
                                                float aP[21], float gm[3]) {
  // the forward's search in float, from freshly evaluated sin and cos of phi
  float sp, cp, sth, cth;
  sincos_r(p[4], &sp, &cp);
  sincos_r(p[5], &sth, &cth);
  bool reachable;
  const float s = cylinder_search(p, sp, cp, rk, b, reachable);
  // dual state along (x, y, kappa, phi, theta), and ds/dp = -g_p / g_s at s
  D5 pd[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) pd[i] = D5(p[i]);
#pragma unroll
  for (int d = 0; d < 5; ++d) pd[cyl_dir_par(d)].d[d] = 1.0f;
  D5 spd, cpd, sthd, cthd;
  sincos_t(pd[4], &spd, &cpd);
  sincos_t(pd[5], &sthd, &cthd);
  D5 sd(s);
  {
    const D5 om = -b * pd[3];
    const D5 u = 0.5f * om * sd;
    D5 su, cu, sinc, g;
    helix_trig_t(u, su, cu, sinc, g);
    const D5 cA = cpd * cu - spd * su;
    const D5 sA = spd * cu + cpd * su;
    const D5 ch = sd * sinc;
    const D5 X = pd[0] + ch * cA;
    const D5 Y = pd[1] + ch * sA;
    const D5 gg = X * X + Y * Y - rk * rk;
    const float cPv = cA.v * cu.v - sA.v * su.v, sPv = sA.v * cu.v + cA.v * su.v;
    const float rgs = rcp(2.0f * (X.v * cPv + Y.v * sPv));
#pragma unroll
    for (int d = 0; d < 5; ++d) sd.d[d] = -gg.d[d] * rgs;
  }
  D5 qd[6], sPd, cPd;
  CylJac<D5> Jd;
  cylinder_at<D5, float>(pd, sthd, cthd, spd, cpd, sd, rk, b, qd, Jd, sPd, cPd);
  const CylJac<float> J{Jd.x0.v, Jd.x1.v, Jd.x3.v, Jd.x4.v, Jd.y0.v, Jd.y1.v, Jd.y3.v, Jd.y4.v, Jd.z0.v,
                        Jd.z1.v, Jd.z3.v, Jd.z4.v, Jd.z5.v, Jd.f0.v, Jd.f1.v, Jd.f3.v, Jd.f4.v};
  float Pt[21];
  transport_cylinder(J, P, Pt);
  float q[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) q[i] = qd[i].v;
  float qb[6], G[6][6];
  adjoint_update(q, Pt, m, V, w, ap, aP, gm, qb, G);

  // adjoint of the transport: aP <- F^T G F
  float GF[6][6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int j = 0; j < 6; ++j) GF[k][j] = fcol_r(J, j, G[k]);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float col[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) col[k] = GF[k][j];
      aP[ix(i, j)] = fcol_r(J, i, col);
    }
  // F_bar = 2 G F P on the entries of F that depend on p: rows x, y, phi in
  // columns (x, y, kappa, phi); row z in (x, y, kappa, phi, theta)
  const int cols[5] = {0, 1, 3, 4, 5};
  float FP[6][5];
#pragma unroll
  for (int jj = 0; jj < 5; ++jj) {
    float col[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) col[l] = P[ix(l, cols[jj])];
#pragma unroll
    for (int k = 0; k < 6; ++k) FP[k][jj] = frow_r(J, k, col);
  }
  float Fb[4][5];
  const int rows[4] = {0, 1, 2, 4};
#pragma unroll
  for (int ri = 0; ri < 4; ++ri)
#pragma unroll
    for (int jj = 0; jj < 5; ++jj) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 6; ++k) acc += G[rows[ri]][k] * FP[k][jj];
      Fb[ri][jj] = 2.0f * acc;
    }

  // adjoint of the propagation
  float apn[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) apn[j] = fcol_r(J, j, qb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    apn[cyl_dir_par(d)] +=
        Fb[0][0] * Jd.x0.d[d] + Fb[0][1] * Jd.x1.d[d] + Fb[0][2] * Jd.x3.d[d] + Fb[0][3] * Jd.x4.d[d] +
        Fb[1][0] * Jd.y0.d[d] + Fb[1][1] * Jd.y1.d[d] + Fb[1][2] * Jd.y3.d[d] + Fb[1][3] * Jd.y4.d[d] +
        Fb[2][0] * Jd.z0.d[d] + Fb[2][1] * Jd.z1.d[d] + Fb[2][2] * Jd.z3.d[d] + Fb[2][3] * Jd.z4.d[d] +
        Fb[2][4] * Jd.z5.d[d] +
        Fb[3][0] * Jd.f0.d[d] + Fb[3][1] * Jd.f1.d[d] + Fb[3][2] * Jd.f3.d[d] + Fb[3][3] * Jd.f4.d[d];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) ap[j] = apn[j];
}

// Cylinders: the dual-number crossing needs 180 VGPRs (2 waves per SIMD);
// compiled for 3 waves it spills 20 bytes per lane and runs faster (barrel
// sample, checkpoints every layer: 0.954 -> 0.882 ms; every 2nd layer:
// 1.064 -> 0.911 ms; for 4 waves it spills enough to take 1.95 ms).
template <int GEOM, int KIND, bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GEOM == 1 ? 3 : 1, 8)))
kf_adjoint_kernel(const AdjointArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Lanes<KIND, WIDE> ln(i, a.n, a.L, a.lay, a.Lck);
  const int L = a.L;
  int done = int(uint32_t(a.status[i]) >> KF_S_LAYERS_SHIFT);
  done = done > L ? L : done;
  const float w = a.grad_chi2[i];
  float ap[6], aP[21];
#pragma unroll
  for (int e = 0; e < 6; ++e) ap[e] = 0.0f;
#pragma unroll
  for (int e = 0; e < 21; ++e) aP[e] = 0.0f;
  // Layers run in step across the wave (the same k in every lane, lanes past
  // their track's end idle), so each dL/dm row, hit row and checkpoint row is
  // one access of the whole wave.  With each lane at its own k the accesses
  // scatter over rows and every 4-byte word costs a line (10x the bytes on
  // the barrel sample).  Layers a track did not apply get dL/dm = 0 in the
  // same store.
  for (int k = L - 1; k >= 0; --k) {
    float gm[3] = {0.0f, 0.0f, 0.0f};
    if (k < done) {
      // the state entering layer k: from the checkpoint slot that covers it
      // (or the seed), then forward through layers j0 .. k-1
      float p[6], P[21];
      int j0 = 0;
      if (a.ckpt) {
        const int c = k >> a.ck_shift;
        j0 = c << a.ck_shift;
        float s[27];
        ln.template ld_all<27>(ln.ck, a.ckpt, c, s);
#pragma unroll
        for (int e = 0; e < 6; ++e) p[e] = s[e];
#pragma unroll
        for (int e = 0; e < 21; ++e) P[e] = s[6 + e];
      } else {
        ln.template ld_all<6>(ln.par, a.par_in, 0, p);
        ln.template ld_all<21>(ln.cov, a.cov_in, 0, P);
      }
      if (j0 < k) {
        float chi2 = 0.0f;
        Dir d;
        dir_init(p, d);
        for (int j = j0; j < k; ++j) {
          float m[3], V[6];
          ln.template ld_all<3>(ln.hp, a.hit_pos, j, m);
          ln.template ld_all<6>(ln.hc, a.hit_cov, j, V);
          layer_at<GEOM, PREC_F32>(j, p, P, d, m, V, a.layer[j], a.b, chi2);
        }
      }
      float m[3], V[6];
      ln.template ld_all<3>(ln.hp, a.hit_pos, k, m);
      ln.template ld_all<6>(ln.hc, a.hit_cov, k, V);
      if (GEOM == 0)
        adjoint_layer_z(p, P, m, V, a.layer[k], a.b, w, ap, aP, gm);
      else
        adjoint_layer_r(p, P, m, V, a.layer[k], a.b, w, ap, aP, gm);
    }
    ln.template st_all<3>(ln.hp, a.grad_hit, k, gm);
  }
  ln.template st_all<6>(ln.par, a.grad_par, 0, ap);
  if (a.grad_cov) ln.template st_all<21>(ln.cov, a.grad_cov, 0, aP);
}

template <int GEOM, int KIND, bool WIDE>
static hipError_t launch_adj(int block, const AdjointArgs& a, hipStream_t s) {
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL((kf_adjoint_kernel<GEOM, KIND, WIDE>), dim3(unsigned(grid)), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int GEOM>
static hipError_t launch_adj_geom(int block, const AdjointArgs& a, hipStream_t s) {
  const bool wide = needs_wide(a.n, a.L, a.lay);
  if (a.lay.kind == KF_AOS)
    return wide ? launch_adj<GEOM, KF_AOS, true>(block, a, s) : launch_adj<GEOM, KF_AOS, false>(block, a, s);
  if (a.lay.kind == KF_AOSOA)
    return wide ? launch_adj<GEOM, KF_AOSOA, true>(block, a, s) : launch_adj<GEOM, KF_AOSOA, false>(block, a, s);
  return wide ? launch_adj<GEOM, KF_SOA, true>(block, a, s) : launch_adj<GEOM, KF_SOA, false>(block, a, s);
}

hipError_t launch_adjoint(int geom, int block, const AdjointArgs& a, hipStream_t s) {
  return geom == 0 ? launch_adj_geom<0>(block, a, s) : launch_adj_geom<1>(block, a, s);
}

}  // namespace kf
