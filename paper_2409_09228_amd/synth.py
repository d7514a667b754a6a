"""Seeded synthetic workloads for the batched Kalman-filter step.

The paper feeds its benchmark with an artificial sample: one seed track
smeared with a Gaussian so that no two tracks repeat the same arithmetic, and
one hit per layer smeared per track the same way (Sec. 3.1, "Input data").
Nothing else about the sample is published, so this module builds an
equivalent sample from stated distributions:

* truth parameters p = (x, y, z, q/pT, phi, theta) drawn per track;
* hits at the points where the true helix crosses each layer, smeared;
* the filter's seed = truth + Gaussian smear of sigma 0.01 on every
  component, with initial covariance C0 = diag(1e-4).

This module is shared by the tests, the benchmark and the oracle-based
checks.  It holds no part of the filter itself (no propagation Jacobian, no
covariance transport, no gain or chi-square).  The layer crossings of the
*true* trajectory are computed here with the circle-centre construction
(rotation of the radius vector about the helix axis and a circle-circle
intersection), in float64, which is independent of both the oracle's and
the GPU kernels' helix code.

Random numbers come from numpy's Philox counter-based generator keyed by
(seed, event), drawn in a fixed order per event, so the output does not
depend on thread count or device.

Units: cm, GeV, tesla, rad.  Curvature convention: the transverse direction
angle advances as d(phi)/ds = omega = -b * (q/pT) with b = 0.00299792458*Bz
(a positive track in +Bz turns clockwise seen from +z).
"""
from __future__ import annotations

import dataclasses
import numpy as np

# Speed of light factor: transverse curvature [1/cm] = C_LIGHT * Bz[T] * q/pT[1/GeV]
C_LIGHT = 0.00299792458

GEOM_Z = 0  # endcap plane at fixed z ("propagate to z")
GEOM_R = 1  # barrel cylinder at fixed radius ("propagate to r")

SIGMA_SEED = 0.01   # seed smear, every component (cm, 1/GeV, rad)
SIGMA_HIT = 0.01    # hit smear (cm)
C0_DIAG = 1e-4      # initial covariance diagonal
V_DIAG = 1e-4       # hit covariance diagonal (cm^2)
BASE_SEED = 240909228
N_LAYER_TABLE = 64  # longest layer table the library accepts


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and distributions of one synthetic sample."""
    name: str
    geom: str            # "z", "r" or "mixed"
    nevts: int
    ntrks: int           # tracks per event
    n_layers: int        # layers per track (max for "mixed")
    bz: float = 3.8
    seed_index: int = 0
    kappa_lo_z: float = 0.5
    kappa_hi_z: float = 5.0
    theta_lo_z: float = 0.4
    theta_hi_z: float = 1.2
    kappa_lo_r: float = 0.3
    kappa_hi_r: float = 5.0
    theta_lo_r: float = 0.5
    theta_hi_r: float = 2.6
    reach_margin: float = 0.9   # p2r: keep layers with r_k <= margin * max radius
    min_layers: int = 5         # "mixed": requested layer count ~ U{min..max}

    @property
    def n_tracks(self) -> int:
        return self.nevts * self.ntrks


# The paper's event shapes: p2z 9600 tracks per event, 32-track batches
# (Sec. 3.2); ~800k-track runs (Sec. 5).  Layer tables z_k = 10 + 5k cm and
# r_k = 5 + 5k cm.
WORKLOADS = {
    "p2z_1x8192": Workload("p2z_1x8192", "z", 1, 8192, 20, seed_index=1),
    "p2z_100x9600": Workload("p2z_100x9600", "z", 100, 9600, 20, seed_index=2),
    "p2r_100x9600": Workload("p2r_100x9600", "r", 100, 9600, 20, seed_index=3),
    "uneven_250k": Workload("uneven_250k", "mixed", 1, 250000, 30, seed_index=4),
    "p2z_64x9600": Workload("p2z_64x9600", "z", 64, 9600, 20, seed_index=5),
}


def layer_table(geom: int, n: int) -> np.ndarray:
    """Layer positions: z_k = 10 + 5k cm (planes) or r_k = 5 + 5k cm (cylinders)."""
    k = np.arange(n, dtype=np.float64)
    return 10.0 + 5.0 * k if geom == GEOM_Z else 5.0 + 5.0 * k


def packed_index(i: int, j: int) -> int:
    """Packed lower-triangle index of symmetric element (i, j)."""
    if i < j:
        i, j = j, i
    return i * (i + 1) // 2 + j


def diag_packed(n: int, value: float, count: int) -> np.ndarray:
    out = np.zeros((count, n * (n + 1) // 2))
    for i in range(n):
        out[:, packed_index(i, i)] = value
    return out


def _curvature(bz: float, kappa: np.ndarray) -> np.ndarray:
    return -C_LIGHT * bz * kappa


def _centre(x0, y0, phi0, omega):
    """Centre of the transverse circle of a helix with direction angle phi0."""
    return x0 - np.sin(phi0) / omega, y0 + np.cos(phi0) / omega


def truth_cross_plane(truth: np.ndarray, zk: float, bz: float) -> np.ndarray:
    """Where the true helix crosses the plane z = zk: (x, y, z) [n, 3].

    Rotation of the start point about the helix axis by the turning angle
    omega * s, with s = (zk - z0) * tan(theta) the transverse path length.
    """
    x0, y0, z0, kap, phi0, th = truth.T
    om = _curvature(bz, kap)
    s = (zk - z0) * np.tan(th)
    cx, cy = _centre(x0, y0, phi0, om)
    a = om * s
    dx, dy = x0 - cx, y0 - cy
    ca, sa = np.cos(a), np.sin(a)
    x = cx + dx * ca - dy * sa
    y = cy + dx * sa + dy * ca
    return np.stack([x, y, np.full_like(x, zk)], axis=1)


def truth_max_radius(truth: np.ndarray, bz: float) -> np.ndarray:
    """Largest transverse radius the true helix reaches: |centre| + R."""
    x0, y0, _, kap, phi0, _ = truth.T
    om = _curvature(bz, kap)
    cx, cy = _centre(x0, y0, phi0, om)
    return np.hypot(cx, cy) + 1.0 / np.abs(om)


def truth_cross_cylinder(truth: np.ndarray, rk: float, bz: float) -> np.ndarray:
    """First crossing (smallest positive path) of the true helix with r = rk.

    Circle-circle intersection of the transverse circle (centre c, radius R)
    with the cylinder's circle, then the candidate reached first moving in
    the track's direction.  Rows with no crossing hold NaN.
    """
    x0, y0, z0, kap, phi0, th = truth.T
    om = _curvature(bz, kap)
    R = 1.0 / np.abs(om)
    cx, cy = _centre(x0, y0, phi0, om)
    d = np.hypot(cx, cy)
    a = (rk * rk - R * R + d * d) / (2.0 * d)
    h2 = rk * rk - a * a
    h = np.sqrt(np.where(h2 >= 0.0, h2, np.nan))
    ux, uy = cx / d, cy / d
    v0x, v0y = x0 - cx, y0 - cy
    best = np.full_like(x0, np.inf)
    bx = np.full_like(x0, np.nan)
    by = np.full_like(x0, np.nan)
    for sgn in (1.0, -1.0):
        px = a * ux - sgn * h * uy
        py = a * uy + sgn * h * ux
        v1x, v1y = px - cx, py - cy
        ang = np.arctan2(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y)
        turn = np.mod(ang * np.sign(om), 2.0 * np.pi)   # turning in the direction of motion
        turn = np.where(turn <= 0.0, 2.0 * np.pi, turn)
        s = turn / np.abs(om)
        take = s < best
        best = np.where(take, s, best)
        bx = np.where(take, px, bx)
        by = np.where(take, py, by)
    z = z0 + best / np.tan(th)
    return np.stack([bx, by, z], axis=1)


def _draw_truth(g: np.random.Generator, n: int, geom: int, w: Workload) -> np.ndarray:
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    if geom == GEOM_Z:
        kmag = g.uniform(w.kappa_lo_z, w.kappa_hi_z, n)
        th = g.uniform(w.theta_lo_z, w.theta_hi_z, n)
    else:
        kmag = g.uniform(w.kappa_lo_r, w.kappa_hi_r, n)
        th = g.uniform(w.theta_lo_r, w.theta_hi_r, n)
    phi = g.uniform(-np.pi, np.pi, n)
    x = g.normal(0.0, 0.01, n)
    y = g.normal(0.0, 0.01, n)
    z = np.zeros(n)
    return np.stack([x, y, z, sign * kmag, phi, th], axis=1)


def _hits_for(g: np.random.Generator, truth: np.ndarray, geom: int, layers: np.ndarray,
              nlay: np.ndarray, bz: float) -> np.ndarray:
    """Smeared hits [L, n, 3]; layers beyond a track's count hold its unsmeared
    truth crossing if one exists, else zeros (they are never read)."""
    n = truth.shape[0]
    L = layers.shape[0]
    hits = np.zeros((L, n, 3))
    for k in range(L):
        if geom == GEOM_Z:
            pt = truth_cross_plane(truth, layers[k], bz)
            sm = g.normal(0.0, SIGMA_HIT, (n, 3))
            pt = pt + sm
        else:
            pt = truth_cross_cylinder(truth, layers[k], bz)
            d_rphi = g.normal(0.0, SIGMA_HIT, n)
            d_z = g.normal(0.0, SIGMA_HIT, n)
            ang = np.arctan2(pt[:, 1], pt[:, 0]) + d_rphi / layers[k]
            pt = np.stack([layers[k] * np.cos(ang), layers[k] * np.sin(ang), pt[:, 2] + d_z], axis=1)
        valid = (k < nlay)[:, None]
        hits[k] = np.where(valid & np.isfinite(pt), pt, 0.0)
    return hits


def reachable_layers(truth: np.ndarray, layers: np.ndarray, bz: float, margin: float) -> np.ndarray:
    """Number of leading cylinders with r_k <= margin * (largest radius of the true helix)."""
    rmax = truth_max_radius(truth, bz)
    return np.sum(layers[None, :] <= margin * rmax[:, None], axis=1).astype(np.int32)


def generate(name_or_workload, seed: int | None = None, n_events: int | None = None) -> dict:
    """Build the sample for a named workload.

    Returns float64 arrays in logical layout:
      par [n, 6] (seed), cov [n, 21] (packed lower triangle), truth [n, 6],
      hit_pos [L, n, 3], hit_cov [L, n, 6], layer_z [L], layer_r [L],
      nlay [n] int32, geom [n] uint8, bz (float).
    ``n_events`` truncates the sample to its first events (same values).
    """
    w = WORKLOADS[name_or_workload] if isinstance(name_or_workload, str) else name_or_workload
    base = BASE_SEED + w.seed_index if seed is None else seed
    nev = w.nevts if n_events is None else min(n_events, w.nevts)
    L = w.n_layers
    lz = layer_table(GEOM_Z, L)
    lr = layer_table(GEOM_R, L)
    parts = []
    for ev in range(nev):
        g = np.random.Generator(np.random.Philox(key=[base, ev]))
        n = w.ntrks
        if w.geom == "mixed":
            geom = np.zeros(n, np.uint8)
            geom[n // 2:] = GEOM_R
            geom = g.permutation(geom)
            want = g.integers(w.min_layers, L + 1, n).astype(np.int32)
        else:
            geom = np.full(n, GEOM_Z if w.geom == "z" else GEOM_R, np.uint8)
            want = np.full(n, L, np.int32)
        truth = np.zeros((n, 6))
        for gi in (GEOM_Z, GEOM_R):
            sel = geom == gi
            if sel.any():
                truth[sel] = _draw_truth(g, int(sel.sum()), gi, w)
        nlay = want.copy()
        selr = geom == GEOM_R
        if selr.any():
            nlay[selr] = np.minimum(want[selr], reachable_layers(truth[selr], lr, w.bz, w.reach_margin))
        seed_par = truth + g.normal(0.0, SIGMA_SEED, (n, 6))
        hits = np.zeros((L, n, 3))
        for gi, tab in ((GEOM_Z, lz), (GEOM_R, lr)):
            sel = geom == gi
            if sel.any():
                hits[:, sel] = _hits_for(g, truth[sel], gi, tab, nlay[sel], w.bz)
        parts.append((seed_par, truth, hits, nlay, geom))
    par = np.concatenate([p[0] for p in parts])
    truth = np.concatenate([p[1] for p in parts])
    hit_pos = np.concatenate([p[2] for p in parts], axis=1)
    nlay = np.concatenate([p[3] for p in parts])
    geom = np.concatenate([p[4] for p in parts])
    n = par.shape[0]
    return {
        "name": w.name,
        "par": par,
        "cov": diag_packed(6, C0_DIAG, n),
        "truth": truth,
        "hit_pos": hit_pos,
        "hit_cov": np.broadcast_to(diag_packed(3, V_DIAG, 1)[None], (L, n, 6)).copy(),
        "layer_z": lz,
        "layer_r": lr,
        "nlay": nlay,
        "geom": geom,
        "bz": w.bz,
    }


def every_nth_layer(sample: dict, step: int) -> dict:
    """The same tracks on every step-th layer of the table (layers 0, step,
    2 step, ...) with the sample's own hits there; a track keeps the kept
    layers it reached (nlay -> ceil(nlay / step))."""
    keep = np.arange(0, sample["hit_pos"].shape[0], step)
    out = dict(sample)
    for k in ("hit_pos", "hit_cov"):
        out[k] = sample[k][keep].copy()
    for k in ("layer_z", "layer_r"):
        out[k] = np.asarray(sample[k])[keep].copy()
    out["nlay"] = ((np.asarray(sample["nlay"]) + step - 1) // step).astype(np.int32)
    return out


# Strongly curved tracks: low transverse momentum, so that the helix turns by
# up to a radian or more between surfaces -- on the 5 cm plane spacing for
# |q/pT| of 6-9 /GeV, on every third barrel layer (r = 5, 20, 35, ... cm) for
# 4-8 /GeV (curling tracks reach only the first few cylinders).
CURLED = {
    "z": Workload("p2z_curled_4096", "z", 1, 4096, 20, seed_index=11, kappa_lo_z=6.0, kappa_hi_z=9.0),
    "r": Workload("p2r_curled_4096", "r", 1, 4096, 20, seed_index=12, kappa_lo_r=4.0, kappa_hi_r=8.0),
}


def curled(geom: str) -> dict:
    """The strongly curved sample for geometry "z" or "r" (see CURLED)."""
    s = generate(CURLED[geom])
    return s if geom == "z" else every_nth_layer(s, 3)


def multi_hit(sample: dict, n_cand: int, spread: float = 3.0, seed: int = 0) -> dict:
    """Candidate hits for hit selection: on every layer each track gets its
    own hit plus n_cand - 1 decoys, at a random position in the list.  A
    decoy is the track's hit displaced by a Gaussian of sigma
    spread * SIGMA_HIT per coordinate -- in x, y and z on planes, along
    r*phi and z on cylinders (decoys stay on the cylinder) -- with the same
    covariance.  Returns cand_pos [L, n, M, 3], cand_cov [L, n, M, 6] and
    true_index [L, n]."""
    hp = np.asarray(sample["hit_pos"], np.float64)
    L, n = hp.shape[:2]
    M = int(n_cand)
    g = np.random.Generator(np.random.Philox(key=[BASE_SEED + 7919 * (seed + 1), M]))
    true_index = g.integers(0, M, (L, n)).astype(np.int32)
    off = g.normal(0.0, spread * SIGMA_HIT, (L, n, M, 3))
    cand = np.repeat(hp[:, :, None, :], M, axis=2)
    geom = np.asarray(sample["geom"])
    cyl = geom == GEOM_R
    if (~cyl).any():
        cand[:, ~cyl] += off[:, ~cyl]
    if cyl.any():
        x, y = cand[:, cyl, :, 0], cand[:, cyl, :, 1]
        r = np.hypot(x, y)
        ang = np.arctan2(y, x) + off[:, cyl, :, 0] / np.where(r > 0, r, 1.0)
        cand[:, cyl, :, 0] = r * np.cos(ang)
        cand[:, cyl, :, 1] = r * np.sin(ang)
        cand[:, cyl, :, 2] += off[:, cyl, :, 2]
    li, ti = np.meshgrid(np.arange(L), np.arange(n), indexing="ij")
    cand[li, ti, true_index] = hp
    cov = np.repeat(np.asarray(sample["hit_cov"], np.float64)[:, :, None, :], M, axis=2)
    return {"cand_pos": cand, "cand_cov": cov, "true_index": true_index, "n_cand": M, "spread": spread}


def subset(sample: dict, idx: np.ndarray) -> dict:
    """The same sample restricted to tracks ``idx`` (tracks are independent)."""
    out = dict(sample)
    for k in ("par", "cov", "truth", "nlay", "geom"):
        out[k] = sample[k][idx]
    for k in ("hit_pos", "hit_cov"):
        out[k] = sample[k][:, idx]
    return out


def to_ragged(hit_pos: np.ndarray, hit_cov: np.ndarray, nlay: np.ndarray):
    """Padded [L, n, c] hits -> ragged per-track runs.

    Returns (hit_pos [H, 3], hit_cov [H, 6], hit_offset [n] int64) where track
    i's k-th hit sits at row hit_offset[i] + k.
    """
    n = nlay.shape[0]
    off = np.zeros(n, np.int64)
    if n:
        off[1:] = np.cumsum(nlay.astype(np.int64))[:-1]
    H = int(nlay.sum())
    tr = np.repeat(np.arange(n), nlay)
    kk = np.arange(H) - np.repeat(off, nlay)
    return (np.ascontiguousarray(hit_pos[kk, tr]), np.ascontiguousarray(hit_cov[kk, tr]), off)
