/*
 * kf.h -- C ABI of libkf.so, a batched Kalman-filter step for charged-particle
 * tracks on AMD Instinct MI355X (gfx950).
 *
 * The step is the one the p2z / p2r tracking mini-apps time (arXiv 2409.09228,
 * Sec. 3 "Description of algorithm" and Sec. 3.2 "Computations and data
 * structure"): for every track, propagate the helix from its current state to
 * the next detector layer -- an endcap plane at fixed z ("propagate to z") or a
 * barrel cylinder at fixed radius r ("propagate to r") -- carrying the 6x6
 * covariance along with the propagation Jacobian F (C -> F C F^T), then update
 * state and covariance with the single hit on that layer (3 coordinates and a
 * 3x3 covariance), and repeat over the track's layers (Sec. 3.1, one hit per
 * layer).
 *
 * Conventions shared by every entry point
 *   Units: cm, GeV, tesla, rad.
 *   Track parameters p = (x, y, z, kappa = q/pT [1/GeV], phi, theta), where phi
 *   is the transverse direction angle and theta the polar angle.  The
 *   transverse curvature is omega = -0.00299792458 * Bz * kappa [1/cm]
 *   (d phi / ds = omega along the transverse arc length s).
 *   Covariances are symmetric and stored as packed lower triangles, row-major:
 *   element (i, j) with i >= j is number i*(i+1)/2 + j.  Track covariance: 21
 *   numbers; hit covariance: 6 (xx, yx, yy, zx, zy, zz).
 *   The hit measures global (x, y, z): H = [I3 | 0].  No process noise.
 *
 * Memory
 *   Every array argument is DEVICE memory (hipMalloc'd or a torch CUDA tensor)
 *   unless its comment says HOST.  Buffers are owned by the caller; the library
 *   keeps no pointer after the call returns (work already enqueued aside) and
 *   allocates nothing except where a function says so.  All calls enqueue on
 *   `stream` (a hipStream_t; NULL = the null stream) and return without
 *   synchronising.  Outputs may alias the matching inputs exactly (in-place);
 *   any other overlap is undefined.  Float arrays must be 4-byte aligned.
 *
 * Track layouts (kf_layout_t), n = n_tracks, element e of track i:
 *   KF_SOA           per-track arrays with e elements per track are stored
 *                    element-major: offset e*n + i.
 *   KF_AOSOA, B      blocks of B tracks (B in {16, 32, 64, 128, 256}):
 *                    offset (i/B)*(E*B) + e*B + i%B for an array of E
 *                    elements per track; the buffer holds ceil(n/B) blocks
 *                    and the padding slots of the last block are neither read
 *                    nor written.
 *   KF_AOS           track-major: offset i*E + e.
 *   Per-layer arrays (hits, checkpoints) add the layer l (0 <= l < n_layers):
 *     KF_SOA          offset (l*E + e)*n + i
 *     KF_AOSOA, B     offset ((i/B)*n_layers + l)*(E*B) + e*B + i%B
 *     KF_AOS          offset (l*n + i)*E + e
 *   This is the array-of-structures-of-arrays organisation of Sec. 3.2 with a
 *   free batch width B.
 *
 * Errors
 *   Argument problems are reported synchronously through kf_status_t before
 *   anything is enqueued; no exception crosses the ABI.  Numerical trouble of
 *   one track is reported in its status word (below); that track stops at the
 *   failing layer and keeps the state it had before it.
 */
#ifndef KF_H
#define KF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KF_ABI_VERSION 7
#define KF_MAX_LAYERS 64

typedef enum {
  KF_OK = 0,
  KF_E_NULL = 1,      /* a required pointer is NULL */
  KF_E_SHAPE = 2,     /* n_tracks < 0, n_layers outside [0, KF_MAX_LAYERS], ... */
  KF_E_LAYOUT = 3,    /* unknown layout kind or block width */
  KF_E_ALIGN = 4,     /* a float pointer is not 4-byte aligned */
  KF_E_DEVICE = 5,    /* no usable gfx950 device */
  KF_E_LAUNCH = 6,    /* the HIP runtime refused the launch */
  KF_E_WORKSPACE = 7, /* workspace missing or too small */
  KF_E_FLAGS = 8,     /* unknown flag bits or tuning values */
  KF_E_UNSUPPORTED = 9 /* valid request the library does not implement */
} kf_status_t;

enum { KF_SOA = 0, KF_AOSOA = 1, KF_AOS = 2 };
typedef struct {
  int32_t kind;  /* KF_SOA, KF_AOSOA or KF_AOS */
  int32_t block; /* AoSoA block width B; ignored for KF_SOA */
} kf_layout_t;

/* Launch shape; pass NULL for the built-in default: (256, 1, dynamic, 1), and
 * (128, 1, static, 2) for kf_propagate_update_batched.
 *   block_threads      64, 128 or 256
 *   tracks_per_thread  1 or 2; the plain kernels use 1 whatever is asked;
 *                      the batched kernel gives each lane this many tracks of a
 *                      work item, one after the other
 *   schedule           batched kernel only: KF_SCHED_DYNAMIC (atomic work queue)
 *                      or KF_SCHED_STATIC (round-robin over the waves)
 *   waves_mult         batched kernel only: 1..8 (0 = 1), grid size in units
 *                      of the blocks that fit on the GPU at once */
enum { KF_SCHED_DYNAMIC = 0, KF_SCHED_STATIC = 1 };
typedef struct {
  int32_t block_threads;
  int32_t tracks_per_thread;
  int32_t schedule;
  int32_t waves_mult;
} kf_tune_t;

/* flags */
enum {
  KF_F_FP64_INVERSE = 1u << 0, /* S = H P H^T + V, S^-1, the gain K and the updates in FP64 */
  KF_F_JOSEPH = 1u << 1,       /* as KF_F_FP64_INVERSE, and the covariance update in Joseph
                                  form (I-KH) P (I-KH)^T + K V K^T */
  KF_F_NO_GRAPH = 1u << 8      /* kf_propagate_update_batched only: enqueue the kernels
                                  directly instead of replaying a cached hipGraph */
};
#define KF_F_PRECISION (KF_F_FP64_INVERSE | KF_F_JOSEPH)
#define KF_BATCHED_MAX_TRACKS ((int64_t)2147483647 - 65536)

/* per-track status word: flag bits, plus the number of layers applied in
 * bits 16..31 */
enum {
  KF_S_NONFINITE = 1,       /* a NaN or Inf entered or came out of the update */
  KF_S_NOT_PD = 2,          /* S failed Sylvester's criterion */
  KF_S_NO_CROSSING = 4,     /* the helix never reaches the surface: a cylinder beyond its
                               reach, or a plane parallel to its direction
                               (|cos theta| < 1e-6) */
  KF_S_NEWTON_RESIDUAL = 8, /* the cylinder iteration ended off the surface, or
                               on a crossing other than the first ahead */
  KF_S_BAD_HITS = 16        /* kf_propagate_update_batched: the track's hit rows fall
                               outside [0, n_hits); the track is left as it came in */
};
#define KF_S_LAYERS_SHIFT 16

/*
 * kf_propagate_update_z -- filter n_tracks tracks through endcap planes
 * z = layer_z[l] (Sec. 3.2, "propagation to z": the expected helical
 * trajectory to layer N+1, then the Kalman update with that layer's hit).
 *
 *   par_in, cov_in    track parameters (6) and covariance (21) per track, in `layout`
 *   par_out, cov_out  results, same layout; may equal par_in / cov_in
 *   hit_pos, hit_cov  per layer and track: hit position (3) and covariance (6),
 *                     in `layout` (per-layer form)
 *   layer_z           HOST [n_layers], plane positions in cm
 *   n_layers          0 .. KF_MAX_LAYERS
 *   n_layers_per_track  [n_tracks] int32 or NULL: track i uses its first
 *                     min(max(n,0), n_layers) layers (NULL: all n_layers).
 *                     With NULL every staged hit is read exactly once and
 *                     the SoA / AoSoA kernels stream the hits with the
 *                     non-temporal cache hint; pass NULL rather than an
 *                     array of n_layers for the fastest form.
 *   n_tracks          >= 0 (0: nothing is enqueued)
 *   bz_tesla          uniform solenoid field
 *   flags             0 (FP32 throughout) or KF_F_* bits
 *   chi2_out          [n_tracks] summed chi-square of the applied layers, or NULL
 *   status_out        [n_tracks] status words, or NULL
 *   ckpt_out          NULL, or [ceil(n_layers / ckpt_every)][27] per track in
 *                     `layout` (per-layer form, E = 27): slot j holds the state
 *                     (6 parameters, then the 21 covariance numbers) that
 *                     entered layer j * ckpt_every; slots of layers a track
 *                     does not reach receive unspecified values (with per-track
 *                     counts in SoA / AoSoA the library writes whole rows).
 *                     Used by kf_chi2_backward and kf_smooth.
 *   ckpt_every        1, 2, 4, .. 64 (0 means 1): the checkpoint stride in layers
 *                     (anything else: KF_E_SHAPE)
 *   tune              NULL or a launch shape
 *
 * The plane is reached after the transverse path s = (z_l - z) tan(theta);
 * the propagated z equals z_l exactly and the covariance's z row and column
 * become zero (a plane fixes z).  A track within 1e-6 rad of theta = pi/2
 * (|cos theta| < 1e-6) runs parallel to the planes: KF_S_NO_CROSSING.
 */
kf_status_t kf_propagate_update_z(
    const float* par_in, const float* cov_in, float* par_out, float* cov_out,
    const float* hit_pos, const float* hit_cov, const float* layer_z, int32_t n_layers,
    const int32_t* n_layers_per_track, int64_t n_tracks, float bz_tesla, kf_layout_t layout,
    uint32_t flags, float* chi2_out, int32_t* status_out, float* ckpt_out, int32_t ckpt_every,
    const kf_tune_t* tune, void* stream);

/*
 * kf_propagate_update_r -- the same through barrel cylinders r = layer_r[l]
 * (Sec. 3.2, "propagation to r": an iterative approach that advances the
 * track state to the next radius).  The crossing is the first one at positive
 * path length; it is found by Newton steps on g(s) = x(s)^2 + y(s)^2 - r^2
 * from the first positive root of g's second-order expansion (at most five
 * steps; a track stops once its steps have converged), after a closed-form
 * test that the helix reaches the cylinder at all (KF_S_NO_CROSSING
 * otherwise).  Layers may lie inside the track (decreasing radii): the search
 * then starts at the near root.  KF_S_NEWTON_RESIDUAL (and the track stops
 * there) when the last iterate misses the cylinder by more than
 * |g| = 1e-4 r^2 (a radius off by about 5e-5 r: next to tangency), or is not
 * the first crossing ahead (g' not of the opposite sign to g(0), s <= 0, or
 * a full turn made: strongly curved tracks entering a cylinder).  Arguments as kf_propagate_update_z (the checkpoints
 * feed kf_smooth); the longer barrel step prefetches each lane's hits into
 * registers in every layout, so the non-temporal form of the planes does not
 * apply here.
 */
kf_status_t kf_propagate_update_r(
    const float* par_in, const float* cov_in, float* par_out, float* cov_out,
    const float* hit_pos, const float* hit_cov, const float* layer_r, int32_t n_layers,
    const int32_t* n_layers_per_track, int64_t n_tracks, float bz_tesla, kf_layout_t layout,
    uint32_t flags, float* chi2_out, int32_t* status_out, float* ckpt_out, int32_t ckpt_every,
    const kf_tune_t* tune, void* stream);

/* Most candidate hits per layer kf_propagate_gate_update accepts. */
#define KF_MAX_CANDIDATES 64

/*
 * kf_propagate_gate_update -- the filter with hit selection: every layer
 * holds n_cand candidate hits per track instead of one; after the
 * propagation each candidate gets the chi-square r^T S^-1 r that an update
 * with it would add (r = m - H q, S = H P H^T + V, H = [I3|0]), and the
 * candidate with the smallest one not above chi2_gate (the first of equal
 * ones) updates the state -- the search step of track finding that runs
 * between propagation and update (Sec. 3.1; the paper's benchmark gives each
 * layer one hit).  If no candidate qualifies the layer is a hole: the state
 * is the prediction and no chi-square is added.  A candidate with non-finite
 * values or an S that is not positive definite takes no part (it does not
 * fail the track).
 *
 *   geometry      0: planes z = layers[l], 1: cylinders r = layers[l]
 *   par_in .. cov_out, layers, n_layers, n_layers_per_track, n_tracks,
 *   bz_tesla, layout, chi2_out, status_out, tune   as in kf_propagate_update_z
 *                 (the status word counts the layers processed, holes
 *                 included; failures as there)
 *   cand_pos      per layer 3 * n_cand floats per track in `layout`
 *                 (candidate j's x, y, z at elements 3j .. 3j+2), i.e. an
 *                 array of E = 3 n_cand elements and n_layers layers
 *   cand_cov      per layer 6 * n_cand floats (candidate j's packed 3x3
 *                 covariance at elements 6j .. 6j+5)
 *   n_cand        1 .. KF_MAX_CANDIDATES
 *   chi2_gate     the largest chi-square accepted (+inf: no gate; NaN is
 *                 KF_E_SHAPE)
 *   flags         0 (FP32 update) or the precision bits of
 *                 kf_propagate_update_z: KF_F_FP64_INVERSE takes every
 *                 candidate's S^-1, the decision's chi-square, the gain and
 *                 the update in FP64; KF_F_JOSEPH adds the Joseph covariance
 *                 update (the form for tracks updated after several holes,
 *                 whose plain FP32 covariance update cancels badly)
 *   chosen_out    [n_layers][n_tracks] int32 or NULL: the candidate used on
 *                 each layer processed, -1 for a hole (layers not processed
 *                 are left untouched)
 * Errors: KF_E_SHAPE, KF_E_LAYOUT, KF_E_FLAGS, KF_E_NULL, KF_E_ALIGN,
 * KF_E_DEVICE, KF_E_LAUNCH; nothing is enqueued on error.
 */
kf_status_t kf_propagate_gate_update(int32_t geometry, const float* par_in, const float* cov_in, float* par_out,
                                     float* cov_out, const float* cand_pos, const float* cand_cov, int32_t n_cand,
                                     float chi2_gate, const float* layers, int32_t n_layers,
                                     const int32_t* n_layers_per_track, int64_t n_tracks, float bz_tesla,
                                     kf_layout_t layout, uint32_t flags, float* chi2_out, int32_t* status_out,
                                     int32_t* chosen_out, const kf_tune_t* tune, void* stream);

/*
 * kf_smooth -- Rauch-Tung-Striebel smoother after the filter: the backward
 * pass that turns the filter (Sec. 3.1: propagate to the next layer, update
 * with its hit, repeat) into a complete track fit, giving every layer the
 * estimate that uses all of the track's hits.  With the filtered state
 * (p_k, C_k) on layer k, the prediction q and Jacobian F of the propagation
 * to layer k + 1 and the smoothed state on layer k + 1:
 *   p'_k = p_k + A (p'_{k+1} - q),  C'_k = C_k + A (C'_{k+1} - F C_k F^T) A^T,
 *   A = C_k F^T (F C_k F^T)^-1,
 * in the five local coordinates of each surface (plane: x, y, kappa, phi,
 * theta; cylinder: the tangent (-y, x)/r, z, kappa, phi, theta).  The filter
 * has no process noise, so A = F^-1 and C'_k = F^-1 C'_{k+1} F^-T: the
 * library evaluates that form (F^-1 in closed form) and never reads C_k.
 *
 *   geometry     0: planes (kf_propagate_update_z), 1: cylinders (_r)
 *   ckpt         the filter's ckpt_out written with ckpt_every = 1 (slot k =
 *                the state entering layer k): slots 0 .. applied - 1 are read,
 *                their first six numbers only (parameters)
 *   par_out, cov_out   the filter's outputs (state after its last layer)
 *   status       the filter's status words: track i is smoothed over its
 *                first (status >> 16) layers; the flags are not looked at
 *   layers, n_layers, n_tracks, bz_tesla, layout   as in the filter call
 *   smoothed     [n_layers] slots of 27 numbers per track in `layout`
 *                (kf_checkpoint_floats(n, L, 1, layout) floats): slot k
 *                receives the smoothed state on layer k (parameters, then the
 *                packed covariance) for k < applied; other slots receive
 *                unspecified values (SoA / AoSoA: the library writes whole
 *                rows).  May be `ckpt` itself (each slot is read before
 *                it is written); must not overlap it otherwise.
 *   tune         NULL or a launch shape (block_threads 64, 128 or 256)
 * Errors: KF_E_SHAPE (geometry, sizes), KF_E_LAYOUT, KF_E_NULL, KF_E_ALIGN,
 * KF_E_FLAGS (tune), KF_E_DEVICE, KF_E_LAUNCH; nothing is enqueued on error.
 * A degenerate step (F not invertible: a crossing tangent to the cylinder)
 * gives non-finite smoothed values for that track.
 */
kf_status_t kf_smooth(int32_t geometry, const float* ckpt, const float* par_out, const float* cov_out,
                      const int32_t* status, const float* layers, int32_t n_layers, int64_t n_tracks,
                      float bz_tesla, kf_layout_t layout, float* smoothed, const kf_tune_t* tune, void* stream);

/*
 * kf_chi2_backward -- adjoint of L = sum_i grad_chi2[i] * chi2_i for the
 * filter through planes (geometry 0, kf_propagate_update_z) or cylinders
 * (geometry 1, kf_propagate_update_r), FP32, flags 0: dL/d(hit positions),
 * dL/d(seed parameters) and, optionally, dL/d(seed covariance).  chi2_i sums
 * r^T S^-1 r over the layers track i applied (the paper's step, Sec. 3.2;
 * the chi-square itself is this project's addition).  The derivative is the
 * full one, including the covariance's dependence on the parameters through
 * the Jacobian (whose own derivative is taken by dual numbers).  On
 * cylinders the path length to the crossing depends on the parameters
 * implicitly (Sec. 3.2: the barrel propagation is an iteration); its
 * derivative is the implicit-function one at the iteration's result,
 * -g_p / g_s of g = x(s)^2 + y(s)^2 - r^2, which is also what the forward's
 * Jacobian uses.
 *
 *   geometry       0 planes, 1 cylinders (else KF_E_SHAPE)
 *   par_in .. n_tracks, bz_tesla, layout   the forward call's inputs
 *                  (layers: layer_z or layer_r, HOST)
 *   status_fwd     [n_tracks] the forward's status words: track i's
 *                  gradient runs over its first (status >> 16) layers
 *   ckpt           the forward's ckpt_out, or NULL to recompute the entering
 *                  state of every layer from the seed (no extra memory,
 *                  O(layers^2) work instead of O(layers))
 *   ckpt_every     the forward's checkpoint stride s: the state entering layer
 *                  k is recomputed from slot k / s through layers
 *                  s * (k / s) .. k - 1 (up to s - 1 forward steps; s times
 *                  less memory than s = 1)
 *   grad_chi2      [n_tracks] dL/dchi2_i
 *   grad_hit_pos   per-layer [n_layers][3] in `layout`; layers a track did not
 *                  apply get 0
 *   grad_par_in    [6] per track in `layout`
 *   grad_cov_in    [21] per track in `layout`, or NULL
 */
kf_status_t kf_chi2_backward(
    int32_t geometry, const float* par_in, const float* cov_in, const float* hit_pos, const float* hit_cov,
    const float* layers, int32_t n_layers, int64_t n_tracks, float bz_tesla, kf_layout_t layout,
    const int32_t* status_fwd, const float* ckpt, int32_t ckpt_every, const float* grad_chi2,
    float* grad_hit_pos, float* grad_par_in, float* grad_cov_in, const kf_tune_t* tune, void* stream);
/* kf_chi2_backward_z -- kf_chi2_backward with geometry 0 (planes). */
kf_status_t kf_chi2_backward_z(
    const float* par_in, const float* cov_in, const float* hit_pos, const float* hit_cov,
    const float* layer_z, int32_t n_layers, int64_t n_tracks, float bz_tesla, kf_layout_t layout,
    const int32_t* status_fwd, const float* ckpt, int32_t ckpt_every, const float* grad_chi2,
    float* grad_hit_pos, float* grad_par_in, float* grad_cov_in, const kf_tune_t* tune, void* stream);
/* Floats of a checkpoint buffer for kf_propagate_update_z / _r and kf_chi2_backward:
 * ceil(n_layers / ckpt_every) per-layer slots of 27 floats per track in
 * `layout`; 0 for invalid arguments. */
int64_t kf_checkpoint_floats(int64_t n_tracks, int32_t n_layers, int32_t ckpt_every, kf_layout_t layout);

/*
 * kf_propagate_update_batched -- tracks of both geometries and uneven layer
 * counts in one persistent launch (the paper's benchmarks give every track the
 * same number of layers, Sec. 3.2; real events do not).
 *
 *   par_in .. cov_out   as kf_propagate_update_z, in `layout`
 *   hit_pos, hit_cov    ragged per-track runs: track i's hit on its layer k
 *                       (k < n_layers_per_track[i]) is row hit_offset[i] + k of
 *                       hit_pos [n_hits][3] and hit_cov [n_hits][6]
 *   hit_offset          [n_tracks] int64, 8-byte aligned; a track whose rows do
 *                       not lie inside [0, n_hits) gets KF_S_BAD_HITS and no layer
 *   n_hits              rows of hit_pos and hit_cov (>= 0)
 *   geom                [n_tracks] uint8: 0 plane (layer_z), any other value cylinder (layer_r)
 *   n_layers_per_track  [n_tracks] int32, clamped to [0, max_layers]
 *   layer_z, layer_r    HOST [max_layers] each: layer k of a track is plane
 *                       layer_z[k] or cylinder layer_r[k]
 *   max_layers          0 .. KF_MAX_LAYERS
 *   n_tracks            0 .. KF_BATCHED_MAX_TRACKS
 *   flags               precision bits as kf_propagate_update_z, plus KF_F_NO_GRAPH
 *   chi2_out, status_out  as kf_propagate_update_z
 *   workspace           DEVICE scratch of at least kf_batched_workspace_size(n_tracks)
 *                       bytes, 8-byte aligned, owned by the caller; calls that share a
 *                       workspace must not overlap in time
 *   tune                NULL or a launch shape (tracks_per_thread = tracks a lane
 *                       takes from each work item)
 *
 * On the device each call sorts the tracks into work items of 64 (x
 * tracks_per_thread) tracks with one geometry and one layer count, ordered by
 * decreasing cost, and a grid that just fills the GPU pulls items from an
 * atomic counter.  Unless KF_F_NO_GRAPH is set the four kernels of a call are
 * captured once into a hipGraph, cached by the call's arguments (up to 32
 * graphs), and replayed on `stream` by later identical calls -- so buffers
 * passed once must stay valid while their graph is cached (kf_batched_release
 * drops the cache).  Results per track are identical to
 * kf_propagate_update_z / _r on the same track.
 */
int64_t kf_batched_workspace_size(int64_t n_tracks);
kf_status_t kf_propagate_update_batched(
    const float* par_in, const float* cov_in, float* par_out, float* cov_out,
    const float* hit_pos, const float* hit_cov, const int64_t* hit_offset, int64_t n_hits, const uint8_t* geom,
    const int32_t* n_layers_per_track, const float* layer_z, const float* layer_r, int32_t max_layers,
    int64_t n_tracks, float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
    int32_t* status_out, void* workspace, int64_t workspace_bytes, const kf_tune_t* tune, void* stream);
/* Destroy every cached batched-call graph. */
void kf_batched_release(void);

/*
 * kf_propagate_update_batched_noalloc -- kf_propagate_update_batched for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  It computes exactly what
 * kf_propagate_update_batched computes (the same kernels, bit for bit) but
 * takes no workspace: its planning workspace is a fixed device array inside
 * the library, about 4 MiB per GPU, sized for KF_NOALLOC_MAX_TRACKS tracks and
 * held by each GPU the library runs on until the process ends.  It calls no
 * allocating routine: no hipMalloc, no graph is built (the four kernels are
 * enqueued on `stream` directly, so a caller capturing that stream records
 * them in its own graph).  KF_F_NO_GRAPH is accepted and changes nothing.
 *
 * Arguments as kf_propagate_update_batched without workspace and
 * workspace_bytes.  n_tracks above KF_NOALLOC_MAX_TRACKS: KF_E_WORKSPACE,
 * nothing enqueued.  Every call on one GPU shares that GPU's array, and the
 * planning kernels clear what must start at zero on every call: calls that
 * overlap in time on one GPU (different streams, or different host threads)
 * race and must be serialised by the caller.
 */
#define KF_NOALLOC_MAX_TRACKS ((int64_t)1 << 20)
kf_status_t kf_propagate_update_batched_noalloc(
    const float* par_in, const float* cov_in, float* par_out, float* cov_out,
    const float* hit_pos, const float* hit_cov, const int64_t* hit_offset, int64_t n_hits, const uint8_t* geom,
    const int32_t* n_layers_per_track, const float* layer_z, const float* layer_r, int32_t max_layers,
    int64_t n_tracks, float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
    int32_t* status_out, const kf_tune_t* tune, void* stream);

/*
 * kf_propagate_update_z_f64 / kf_propagate_update_r_f64 -- the same steps in
 * FP64 end to end: double arrays (same layouts, 8-byte elements, 8-byte
 * aligned), field constant and layer table in double, all arithmetic in
 * double (the paper's CPU and non-A770 GPU runs; MI355X issues FP64 FMA at
 * the non-packed FP32 rate).  flags: 0 (plain covariance update) or
 * KF_F_JOSEPH (Joseph form); KF_F_FP64_INVERSE alone changes nothing here.
 * Status words and failure handling as the FP32 calls; no checkpoints.
 */
kf_status_t kf_propagate_update_z_f64(
    const double* par_in, const double* cov_in, double* par_out, double* cov_out, const double* hit_pos,
    const double* hit_cov, const double* layer_z, int32_t n_layers, const int32_t* n_layers_per_track,
    int64_t n_tracks, double bz_tesla, kf_layout_t layout, uint32_t flags, double* chi2_out, int32_t* status_out,
    const kf_tune_t* tune, void* stream);
kf_status_t kf_propagate_update_r_f64(
    const double* par_in, const double* cov_in, double* par_out, double* cov_out, const double* hit_pos,
    const double* hit_cov, const double* layer_r, int32_t n_layers, const int32_t* n_layers_per_track,
    int64_t n_tracks, double bz_tesla, kf_layout_t layout, uint32_t flags, double* chi2_out, int32_t* status_out,
    const kf_tune_t* tune, void* stream);

/*
 * kf_propagate_update_host -- the step on HOST-resident arrays, transfers
 * included (the paper times its kernels both with and without the host-device
 * copies, Sec. 5).  Arguments as kf_propagate_update_z / _r (geometry 0:
 * planes layer[], 1: cylinders; no checkpoints), but every array pointer is a
 * HOST pointer -- page-locked memory (hipHostMalloc) lets the copies overlap
 * the kernels, pageable memory works but serialises them.
 *
 * The tracks are cut into chunks of chunk_tracks (0: 131072; rounded up to a
 * whole AoSoA block); chunk j is copied in, filtered by the same kernels as the
 * device-resident calls, and copied out on stream j mod n_streams (1 .. 8, 0:
 * 3), so the copies of one chunk overlap the kernel of another.  The call
 * returns when every result is in host memory; results are identical to the
 * device-resident call's.  The library keeps the chunk buffers and streams of
 * the last configuration per device (about n_streams * chunk_tracks *
 * (54 + 36 n_layers) * 4 bytes) until kf_host_release.  Not thread-safe
 * against itself: concurrent calls are serialised.
 */
kf_status_t kf_propagate_update_host(
    int32_t geometry, const float* par_in, const float* cov_in, float* par_out, float* cov_out,
    const float* hit_pos, const float* hit_cov, const float* layers, int32_t n_layers,
    const int32_t* n_layers_per_track, int64_t n_tracks, float bz_tesla, kf_layout_t layout, uint32_t flags,
    float* chi2_out, int32_t* status_out, int64_t chunk_tracks, int32_t n_streams, const kf_tune_t* tune);
/* Free the host pipeline's device buffers and streams. */
void kf_host_release(void);

/* Copy between KF_SOA and another layout for an array of n_elem elements per
 * track (n_layers_or_1 = 1 for per-track arrays, the layer count for
 * per-layer arrays).  dst and src must not overlap. */
kf_status_t kf_pack(const float* src_soa, float* dst, int32_t n_elem, int32_t n_layers_or_1,
                    int64_t n_tracks, kf_layout_t layout, void* stream);
kf_status_t kf_unpack(const float* src, float* dst_soa, int32_t n_elem, int32_t n_layers_or_1,
                      int64_t n_tracks, kf_layout_t layout, void* stream);

/* Number of floats an array of n_elem per track (and n_layers_or_1 layers)
 * occupies in `layout`; 0 for an invalid layout. */
int64_t kf_array_floats(int32_t n_elem, int32_t n_layers_or_1, int64_t n_tracks, kf_layout_t layout);

const char* kf_status_string(kf_status_t status);
int kf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KF_H */
