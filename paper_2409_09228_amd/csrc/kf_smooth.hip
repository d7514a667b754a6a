// Rauch-Tung-Striebel smoother after the filter: one lane per track walks
// back over the layers its filter applied and writes the smoothed state of
// every layer -- the backward pass that completes a track fit on top of the
// paper's forward step (Sec. 3.1).
//
// With the filtered state (p_k, C_k) on layer k, the prediction q and
// Jacobian F of the propagation from layer k to k + 1, and the smoothed
// state (p', C') on layer k + 1, the smoother takes
//   p'_k = p_k + A (p'_{k+1} - q),   C'_k = C_k + A (C'_{k+1} - F C_k F^T) A^T,
//   A = C_k F^T (F C_k F^T)^-1,
// every matrix in the five local coordinates of its surface (a state on a
// surface cannot leave it, so its 6x6 covariance is singular along the
// normal).  The filter has no process noise, so F C_k F^T is the whole
// predicted covariance and, whenever C_k is invertible, A = F^-1 exactly:
//   p'_k = p_k + F^-1 (p'_{k+1} - q),   C'_k = F^-1 C'_{k+1} F^-T.
// That is what is evaluated here: F^-1 in closed form from the sparsity of
// the propagation Jacobian (better conditioned in FP32 than inverting the
// predicted covariance, and C_k is never read -- only the filtered
// parameters are).
//
// Local coordinates: on a plane (x, y, kappa, phi, theta), z fixed; on a
// cylinder (t, z, kappa, phi, theta), t along (-y, x)/r at the surface point
// the filter predicted (the point whose normal the covariance is singular
// along).  For layer k that point is the propagation of the filtered state
// of layer k - 1 (of the seed for layer 0), so the cylinder pass runs one
// propagation ahead: each propagation serves as layer k's frame and then as
// the Jacobian of the next step back.
//
// Precision: positions of tens of cm and unwrapped angles of several rad
// carry FP32 rounding of ~1e-6 of their size, and an angle's rounding error
// moves the positions of all earlier layers through the lever arm.  So the
// pass carries the smoothing correction D = p' - p (small) rather than p':
//   D_k = F^-1 (D_{k+1} + (p_{k+1} - p_k) - (q - p_k)),
// with the prediction's increments q - p_k taken from the propagation at
// full precision and p_{k+1} - p_k a difference of neighbouring states; the
// smoothed parameters p_k + D_k are rounded once, on output.
//
// The loop runs over a wave-uniform layer index (from the last layer down),
// each lane taking part for its own applied layers, so that every array
// access keeps a wave-uniform layer offset.
//
// Reads per layer: the filtered parameters (6 of the checkpoint slot's 27
// numbers); writes per layer: the smoothed state (27).  Every slot is read
// before it is written, so the output may be the checkpoint array itself.
#include "kf_device.h"
#include "kf_internal.h"
#include "kf_lanes.h"

namespace kf {

namespace {

// --------------------------------------------------------------------- plane
// F restricted to (x, y, kappa, phi, theta) is
//   x' = x + a1 kappa + a2 phi + a3 theta,  y' = y + b1 kappa + b2 phi + b3 theta,
//   phi' = phi + c1 kappa + c3 theta,       kappa' = kappa, theta' = theta,
// whose inverse has the same pattern: phi = phi' - c1 kappa' - c3 theta',
// x = x' - a1 kappa' - a2 phi - a3 theta', y likewise.  It is returned as a
// PlaneJac so that the plane transport applies it to covariances.
__device__ __forceinline__ PlaneJac<float> plane_inverse(const PlaneJac<float>& J) {
  PlaneJac<float> G;
  G.a0 = G.b0 = G.c0 = 0.0f;  // z column: unused (z row and column are zero)
  G.c1 = -J.c1;
  G.c3 = -J.c3;
  G.a1 = J.a2 * J.c1 - J.a1;
  G.a2 = -J.a2;
  G.a3 = J.a2 * J.c3 - J.a3;
  G.b1 = J.b2 * J.c1 - J.b1;
  G.b2 = -J.b2;
  G.b3 = J.b2 * J.c3 - J.b3;
  return G;
}

// D <- G (D + dp - dq) on (x, y, kappa, phi, theta): dp = p_{k+1} - p_k,
// dq = the prediction's increments; G as plane_inverse returns it
__device__ __forceinline__ void plane_back(const PlaneJac<float>& G, const float dp[6], const float dq[6],
                                           float D[6]) {
  const float dx = D[0] + (dp[0] - dq[0]), dy = D[1] + (dp[1] - dq[1]);
  const float dk = D[3] + dp[3], df = D[4] + (dp[4] - dq[4]), dt = D[5] + dp[5];
  D[0] = dx + G.a1 * dk + G.a2 * df + G.a3 * dt;
  D[1] = dy + G.b1 * dk + G.b2 * df + G.b3 * dt;
  D[2] = 0.0f;
  D[3] = dk;
  D[4] = df + G.c1 * dk + G.c3 * dt;
  D[5] = dt;
}

// The prediction from p to the plane zk: its increments dq (x, y, phi; the
// others are not used) and the Jacobian.  The propagation of a copy of p at
// x = y = phi = 0, with the direction of p, returns exactly the increments.
__device__ __forceinline__ void plane_predict(const float p[6], float zk, float b, float dq[6], PlaneJac<float>& J) {
  float sth, cth, sp, cp, sP, cP;
  sincos_t(p[5], &sth, &cth);
  sincos_t(p[4], &sp, &cp);
  const float p0[6] = {0.0f, 0.0f, p[2], p[3], 0.0f, p[5]};
  helix_to_plane_dir<float, float>(p0, sth, cth, sp, cp, zk, b, dq, J, sP, cP);
}

// ------------------------------------------------------------------ cylinder
// Local covariances: packed 5x5 (15 entries, ix order) over (t, z, kappa,
// phi, theta).
struct Frame {
  float tx, ty;  // unit tangent (-y, x)/r
};

__device__ __forceinline__ Frame frame_at(float x, float y) {
  const float r2 = x * x + y * y;
  const float ri = r2 > 0.0f ? rcp(sqrtf(r2)) : 0.0f;
  return {-y * ri, x * ri};
}

// C (6x6 packed) -> U^T C U
__device__ __forceinline__ void to_local(const Frame& f, const float C[21], float L5[15]) {
  L5[ix(0, 0)] = f.tx * f.tx * C[ix(0, 0)] + 2.0f * f.tx * f.ty * C[ix(1, 0)] + f.ty * f.ty * C[ix(1, 1)];
#pragma unroll
  for (int j = 1; j < 5; ++j) {
    L5[ix(j, 0)] = f.tx * C[ix(j + 1, 0)] + f.ty * C[ix(j + 1, 1)];
#pragma unroll
    for (int k = 1; k <= j; ++k) L5[ix(j, k)] = C[ix(j + 1, k + 1)];
  }
}

// U L5 U^T -> C (6x6 packed)
__device__ __forceinline__ void from_local(const Frame& f, const float L5[15], float C[21]) {
  const float tt = L5[ix(0, 0)];
  C[ix(0, 0)] = f.tx * f.tx * tt;
  C[ix(1, 0)] = f.tx * f.ty * tt;
  C[ix(1, 1)] = f.ty * f.ty * tt;
#pragma unroll
  for (int j = 1; j < 5; ++j) {
    C[ix(j + 1, 0)] = f.tx * L5[ix(j, 0)];
    C[ix(j + 1, 1)] = f.ty * L5[ix(j, 0)];
#pragma unroll
    for (int k = 1; k <= j; ++k) C[ix(j + 1, k + 1)] = L5[ix(j, k)];
  }
}

// F^-1 in local coordinates.  F (from frame f0 at layer k to frame f1 at
// layer k + 1) has rows t = (Mtt, 0, Mtk, Mtf, 0), z = (Mzt, 1, Mzk, Mzf, Mzh),
// phi = (Mft, 0, Mfk, Mff, 0) and identity rows kappa, theta; inverting the
// (t, phi) block M gives
//   (t, phi) = M^-1 ((t', phi') - (Mtk, Mfk) kappa'),
//   z = z' - Mzt t - Mzk kappa' - Mzf phi - Mzh theta'.
struct CylInverse {
  float tt, tk, tf;           // row t:   (tt, 0, tk, tf, 0)
  float zt, zk, zf, zh;       // row z:   (zt, 1, zk, zf, zh)
  float ft, fk, ff;           // row phi: (ft, 0, fk, ff, 0)
};

__device__ __forceinline__ CylInverse cyl_inverse(const CylJac<float>& J, const Frame& f0, const Frame& f1) {
  const float Mtt = f1.tx * (J.x0 * f0.tx + J.x1 * f0.ty) + f1.ty * (J.y0 * f0.tx + J.y1 * f0.ty);
  const float Mtk = f1.tx * J.x3 + f1.ty * J.y3;
  const float Mtf = f1.tx * J.x4 + f1.ty * J.y4;
  const float Mft = J.f0 * f0.tx + J.f1 * f0.ty;
  const float Mzt = J.z0 * f0.tx + J.z1 * f0.ty;
  const float rdet = rcp(Mtt * J.f4 - Mtf * Mft);
  CylInverse G;
  G.tt = J.f4 * rdet;
  G.tf = -Mtf * rdet;
  G.ft = -Mft * rdet;
  G.ff = Mtt * rdet;
  G.tk = -(G.tt * Mtk + G.tf * J.f3);
  G.fk = -(G.ft * Mtk + G.ff * J.f3);
  G.zt = -(Mzt * G.tt + J.z4 * G.ft);
  G.zk = -(Mzt * G.tk + J.z4 * G.fk) - J.z3;
  G.zf = -(Mzt * G.tf + J.z4 * G.ff);
  G.zh = -J.z5;
  return G;
}

// L5 <- G L5 G^T
__device__ __forceinline__ void cyl_congruence(const CylInverse& G, float L5[15]) {
  float C[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) C[i][j] = C[j][i] = L5[ix(i, j)];
  float Wt[5], Wz[5], Wf[5];  // rows t, z, phi of G C
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    Wt[j] = G.tt * C[0][j] + G.tk * C[2][j] + G.tf * C[3][j];
    Wf[j] = G.ft * C[0][j] + G.fk * C[2][j] + G.ff * C[3][j];
    Wz[j] = G.zt * C[0][j] + C[1][j] + G.zk * C[2][j] + G.zf * C[3][j] + G.zh * C[4][j];
  }
  L5[ix(0, 0)] = G.tt * Wt[0] + G.tk * Wt[2] + G.tf * Wt[3];
  L5[ix(1, 0)] = G.tt * Wz[0] + G.tk * Wz[2] + G.tf * Wz[3];
  L5[ix(1, 1)] = G.zt * Wz[0] + Wz[1] + G.zk * Wz[2] + G.zf * Wz[3] + G.zh * Wz[4];
  L5[ix(2, 0)] = Wt[2];
  L5[ix(2, 1)] = Wz[2];
  L5[ix(2, 2)] = C[2][2];
  L5[ix(3, 0)] = G.tt * Wf[0] + G.tk * Wf[2] + G.tf * Wf[3];
  L5[ix(3, 1)] = G.zt * Wf[0] + Wf[1] + G.zk * Wf[2] + G.zf * Wf[3] + G.zh * Wf[4];
  L5[ix(3, 2)] = Wf[2];
  L5[ix(3, 3)] = G.ft * Wf[0] + G.fk * Wf[2] + G.ff * Wf[3];
  L5[ix(4, 0)] = Wt[4];
  L5[ix(4, 1)] = Wz[4];
  L5[ix(4, 2)] = C[4][2];
  L5[ix(4, 3)] = Wf[4];
  L5[ix(4, 4)] = C[4][4];
}

// D <- U0 G U1^T (D + dp - dq): dp = p_{k+1} - p_k, dq = the prediction's
// increments (x, y, z, phi)
__device__ __forceinline__ void cyl_back(const CylInverse& G, const Frame& f0, const Frame& f1, const float dp[6],
                                         const float dq[6], float D[6]) {
  const float dt = f1.tx * (D[0] + (dp[0] - dq[0])) + f1.ty * (D[1] + (dp[1] - dq[1]));
  const float dz = D[2] + (dp[2] - dq[2]), dk = D[3] + dp[3], df = D[4] + (dp[4] - dq[4]), dh = D[5] + dp[5];
  const float et = G.tt * dt + G.tk * dk + G.tf * df;
  const float ez = G.zt * dt + dz + G.zk * dk + G.zf * df + G.zh * dh;
  const float ef = G.ft * dt + G.fk * dk + G.ff * df;
  D[0] = f0.tx * et;
  D[1] = f0.ty * et;
  D[2] = ez;
  D[3] = dk;
  D[4] = ef;
  D[5] = dh;
}

// the crossing q, its increments dq (x, y, z, phi) and Jacobian
__device__ __forceinline__ void cyl_predict(const float p[6], float rk, float b, float q[6], float dq[6],
                                            CylJac<float>& J) {
  DirT<float> d;
  dir_init(p, d);
  (void)helix_to_cylinder(p, d, rk, b, q, J, dq);
}

// Default cache policy: the waves of tracks with different layer counts
// read and write partial rows, for which the non-temporal hint costs more
// than it saves (measured: 1.29 against 0.94 ms on the barrel sample, 2 %
// gained on planes).
template <int KIND, bool WIDE>
using SmoothLanes = Lanes<KIND, WIDE>;

template <int KIND, bool WIDE>
__device__ __forceinline__ void store_state(const SmoothLanes<KIND, WIDE>& ln, float* base, int k, const float p[6],
                                            const float C[21]) {
  float s[27];
#pragma unroll
  for (int e = 0; e < 6; ++e) s[e] = p[e];
#pragma unroll
  for (int e = 0; e < 21; ++e) s[6 + e] = C[e];
  ln.template st_all<27>(ln.ck, base, k, s);
}

}  // namespace

// Cylinders: compiled for 4 waves per SIMD (128 VGPRs, no spill; 156 and 3
// waves otherwise: 557 -> 551 us on the barrel sample).
template <int GEOM, int KIND, bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GEOM == 1 ? 4 : 1, 8)))
kf_smooth_kernel(const SmoothArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const SmoothLanes<KIND, WIDE> ln(i, a.n, a.L, a.lay, a.L);
  int nd = int(uint32_t(a.status[i]) >> 16);
  nd = nd > a.L ? a.L : nd;
  if (nd <= 0) return;
  float C[21];      // the smoothed covariance (on planes its z row and column are zero)
  float L5[15];     // cylinder: the smoothed covariance in local coordinates
  float p1[6];      // filtered parameters of the layer above (k + 1)
  float pk[6] = {};  // filtered parameters of layer k (from checkpoint slot k + 1)
  float D[6] = {};  // smoothing correction of layer k + 1
  // cylinder: the prediction into layer k + 1 (increments, Jacobian, frame)
  float dqn[6] = {};
  CylJac<float> Jn;
  Frame f1{0.0f, 0.0f};
  ln.template ld_all<6>(ln.par, a.par, 0, p1);
  ln.template ld_all<21>(ln.cov, a.cov, 0, C);
  // checkpoint slot k's parameters, fetched one iteration ahead of their use
  // (planes do not need slot 0: zeros)
  float nx[6] = {};
  if (nd == a.L && (GEOM == 1 || a.L - 1 > 0)) ln.template ld_first<27, 6>(ln.ck, a.ckpt, a.L - 1, nx);
  for (int k = a.L - 1; k >= 0; --k) {
    // layer k - 1's filtered parameters (checkpoint slot k), or the seed
    float pm[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) pm[e] = nx[e];
    if (k - 1 >= 0 && k - 1 < nd) {
      if (GEOM == 1 || k - 1 > 0) {
        ln.template ld_first<27, 6>(ln.ck, a.ckpt, k - 1, nx);
      } else {
#pragma unroll
        for (int e = 0; e < 6; ++e) nx[e] = 0.0f;
      }
    }
    // the row of layer k: the smoothed state, or (k >= nd, element-major
    // layouts) the track's final state, so that no line of the output is
    // written in part (memory completes partial lines by read-modify-write:
    // 0.94 -> 0.74 ms on the barrel sample; AoS records share their lines
    // with neighbouring lanes either way and only lose, 0.92 -> 1.09 ms).
    // One store per row after the branches: a store in each branch would
    // write every row of a divergent wave in two parts at different times.
    float ps[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) ps[e] = p1[e];
    if (k < nd) {
      // cylinder: the prediction into layer k gives layer k's frame and the
      // Jacobian of the next step back (one propagation per layer and lane,
      // whichever branch below the lane takes)
      float dqk[6] = {};
      CylJac<float> Jk;
      Frame f0{0.0f, 0.0f};
      if constexpr (GEOM == 1) {
        float qk[6];
        cyl_predict(pm, a.layer[k], a.b, qk, dqk, Jk);
        f0 = frame_at(qk[0], qk[1]);
      }
      if (k == nd - 1) {
        // the last layer applied: smoothed = filtered
        if constexpr (GEOM == 1) to_local(f0, C, L5);
      } else {
        // step back from layer k + 1 (p1) to layer k (pk)
        float dp[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) dp[e] = p1[e] - pk[e];
        if constexpr (GEOM == 0) {
          float dq[6];
          PlaneJac<float> J;
          plane_predict(pk, a.layer[k + 1], a.b, dq, J);
          const PlaneJac<float> G = plane_inverse(J);
          plane_back(G, dp, dq, D);
          float Cn[21];
          transport_plane<true>(G, C, Cn);
#pragma unroll
          for (int e = 0; e < 21; ++e) C[e] = Cn[e];
        } else {
          const CylInverse G = cyl_inverse(Jn, f0, f1);
          cyl_back(G, f0, f1, dp, dqn, D);
          cyl_congruence(G, L5);
          from_local(f0, L5, C);
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) ps[e] = pk[e] + D[e];
#pragma unroll
        for (int e = 0; e < 6; ++e) p1[e] = pk[e];
      }
#pragma unroll
      for (int e = 0; e < 6; ++e) pk[e] = pm[e];
      if constexpr (GEOM == 1) {
#pragma unroll
        for (int e = 0; e < 6; ++e) dqn[e] = dqk[e];
        Jn = Jk;
        f1 = f0;
      }
    }
    if (KIND != KF_AOS || k < nd) store_state(ln, a.smoothed, k, ps, C);
  }
}

template <int GEOM, bool WIDE>
static hipError_t launch_kind(int block, const SmoothArgs& a, hipStream_t s) {
  const dim3 grid(unsigned((a.n + block - 1) / block));
  if (a.lay.kind == KF_AOS)
    hipLaunchKernelGGL((kf_smooth_kernel<GEOM, KF_AOS, WIDE>), grid, dim3(block), 0, s, a);
  else if (a.lay.kind == KF_AOSOA)
    hipLaunchKernelGGL((kf_smooth_kernel<GEOM, KF_AOSOA, WIDE>), grid, dim3(block), 0, s, a);
  else
    hipLaunchKernelGGL((kf_smooth_kernel<GEOM, KF_SOA, WIDE>), grid, dim3(block), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_smooth(int geom, int block, const SmoothArgs& a, hipStream_t s) {
  const bool wide = needs_wide(a.n, a.L, a.lay);
  if (geom == 0) return wide ? launch_kind<0, true>(block, a, s) : launch_kind<0, false>(block, a, s);
  return wide ? launch_kind<1, true>(block, a, s) : launch_kind<1, false>(block, a, s);
}

}  // namespace kf
