"""Python access to the FP64 CPU oracle (``kf_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.

Arrays use the logical layout of the synthetic sample: par [n, 6],
cov [n, 21] (packed lower triangle), hit_pos [L, n, 3], hit_cov [L, n, 6].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kf_oracle.cpp")
_LIB = os.path.join(_HERE, "libkforacle.so")

ST_NONFINITE = 1
ST_NOT_PD = 2
ST_NO_CROSSING = 4
ST_NEWTON_RESIDUAL = 8


# g++ flags: IEEE arithmetic (no fast-math; -std=c++17 keeps multiply-adds
# unfused), OpenMP over tracks.  The in-tree build targets the generic x86-64
# ISA so that it runs on any host it is copied to.
CXXFLAGS = ["-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True, out: str | None = None, native: bool = False) -> str:
    """Compile the oracle with g++.  native=True adds -march=native (the host
    the library is built on must be the one that runs it)."""
    path = _LIB if out is None else out
    if force or not os.path.exists(path):
        cmd = ["g++", *CXXFLAGS, *(["-march=native"] if native else []), "-o", path + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)
    return path


_lib = None
_lib_path = None


def use_native_build(directory: str) -> str:
    """Build the oracle with -march=native for this host into `directory` and
    load that copy instead of the in-tree one (the CPU-baseline timing).
    Returns the library's path."""
    global _lib, _lib_path
    path = build(force=True, out=os.path.join(directory, "libkforacle_native.so"), native=True)
    _lib = None
    _lib_path = path
    lib()
    return path


def lib():
    global _lib
    if _lib is None:
        path = _lib_path or _LIB
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        d, f, i32, u32 = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float),
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32))
        c_int, c_i64, c_dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.kfo_run_f64.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, d, d, d, d, c_int, d, d, d, i32, c_int]
        L.kfo_run_f32.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, f, f, f, f, c_int, f, f, f, i32, c_int]
        L.kfo_propagate.argtypes = [c_int, d, c_dbl, c_dbl, d, d, u32]
        L.kfo_update.argtypes = [d, d, d, d, c_int, d, d, d, u32]
        L.kfo_newton_r.argtypes = [d, c_dbl, c_dbl, d, d, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.kfo_grad_chi2.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, d, d, d, d, c_int, d, d, d, c_int]
        L.kfo_grad_chi2_f32.argtypes = L.kfo_grad_chi2.argtypes
        L.kfo_filter_record.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, d, d, d, d, c_int, d, d, d, d, d, d,
                                        i32, c_int, c_int]
        L.kfo_filter_record.restype = ctypes.c_int
        L.kfo_gate_run.argtypes = [c_int, c_i64, c_int, c_int, d, c_dbl, i32, d, d, d, d, c_dbl, i32, c_int, d, d,
                                   d, i32, i32, d, c_int, c_int]
        L.kfo_gate_run.restype = ctypes.c_int
        for fn in (L.kfo_run_f64, L.kfo_run_f32, L.kfo_propagate, L.kfo_update, L.kfo_grad_chi2,
                   L.kfo_grad_chi2_f32):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def _threads(nthreads):
    if nthreads is not None:
        return int(nthreads)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def run(geom: int, par, cov, hit_pos, hit_cov, layers, bz: float, nlay=None, joseph=False,
        precision: str = "f64", nthreads=None):
    """Filter every track; returns (par_out, cov_out, chi2, status)."""
    dt = np.float64 if precision == "f64" else np.float32
    ct = ctypes.c_double if precision == "f64" else ctypes.c_float
    par = np.ascontiguousarray(par, dt)
    cov = np.ascontiguousarray(cov, dt)
    hit_pos = np.ascontiguousarray(hit_pos, dt)
    hit_cov = np.ascontiguousarray(hit_cov, dt)
    layers = np.ascontiguousarray(layers, np.float64)
    n = par.shape[0]
    L = hit_pos.shape[0]
    assert par.shape == (n, 6) and cov.shape == (n, 21)
    assert hit_pos.shape == (L, n, 3) and hit_cov.shape == (L, n, 6) and layers.shape[0] >= L
    nl = None if nlay is None else np.ascontiguousarray(nlay, np.int32)
    po = np.zeros((n, 6), dt)
    co = np.zeros((n, 21), dt)
    chi2 = np.zeros(n, dt)
    st = np.zeros(n, np.int32)
    fn = lib().kfo_run_f64 if precision == "f64" else lib().kfo_run_f32
    rc = fn(int(geom), n, L, _p(layers, ctypes.c_double), float(bz), _p(nl, ctypes.c_int32),
            _p(par, ct), _p(cov, ct), _p(hit_pos, ct), _p(hit_cov, ct), int(bool(joseph)),
            _p(po, ct), _p(co, ct), _p(chi2, ct), _p(st, ctypes.c_int32), _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return po, co, chi2, st


def run_sample(sample: dict, geom: int | None = None, **kw):
    """``run`` on a synthetic sample (single geometry)."""
    g = int(sample["geom"][0]) if geom is None else geom
    layers = sample["layer_z"] if g == 0 else sample["layer_r"]
    return run(g, sample["par"], sample["cov"], sample["hit_pos"], sample["hit_cov"], layers,
               sample["bz"], nlay=sample["nlay"], **kw)


def propagate(geom: int, p, target: float, bz: float):
    """One propagation: returns (p_out [6], F [6, 6], flags)."""
    p = np.ascontiguousarray(p, np.float64)
    po = np.zeros(6)
    F = np.zeros((6, 6))
    fl = ctypes.c_uint32(0)
    lib().kfo_propagate(int(geom), _p(p, ctypes.c_double), float(target), float(bz),
                        _p(po, ctypes.c_double), _p(F, ctypes.c_double), ctypes.byref(fl))
    return po, F, fl.value


def newton_r(p, rk: float, bz: float, steps: bool = False):
    """The method's crossing search for cylinder rk on its own (single
    precision): (last iterate s, |x(s)^2 + y(s)^2 - rk^2| / rk^2), plus the
    number of Newton steps taken and whether the iterate is the first
    crossing if `steps`.  The oracle's crossing is the closed form; this
    search decides the ST_NEWTON_RESIDUAL flag."""
    p = np.ascontiguousarray(p, np.float64)
    s = ctypes.c_double(0.0)
    rel = ctypes.c_double(0.0)
    n = ctypes.c_int32(0)
    first = ctypes.c_int32(0)
    lib().kfo_newton_r(_p(p, ctypes.c_double), float(rk), float(bz), ctypes.byref(s), ctypes.byref(rel),
                       ctypes.byref(n), ctypes.byref(first))
    return (s.value, rel.value, n.value, bool(first.value)) if steps else (s.value, rel.value)


def update(p, P21, m, V6, joseph=False):
    """One Kalman update: returns (p_out, P21_out, chi2, flags)."""
    p = np.ascontiguousarray(p, np.float64)
    P21 = np.ascontiguousarray(P21, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    V6 = np.ascontiguousarray(V6, np.float64)
    po = np.zeros(6)
    Po = np.zeros(21)
    c = ctypes.c_double(0.0)
    fl = ctypes.c_uint32(0)
    lib().kfo_update(_p(p, ctypes.c_double), _p(P21, ctypes.c_double), _p(m, ctypes.c_double),
                     _p(V6, ctypes.c_double), int(bool(joseph)), _p(po, ctypes.c_double),
                     _p(Po, ctypes.c_double), ctypes.byref(c), ctypes.byref(fl))
    return po, Po, c.value, fl.value


def grad_chi2(geom: int, par, cov, hit_pos, hit_cov, layers, bz: float, w=None, nlay=None,
              joseph=False, nthreads=None, precision: str = "f64"):
    """Reference gradient of sum_i w_i chi2_i: (g_hit [L, n, 3], g_par [n, 6]).
    precision="f32" evaluates the same algorithm in float (tolerance sizing)."""
    par = np.ascontiguousarray(par, np.float64)
    cov = np.ascontiguousarray(cov, np.float64)
    hit_pos = np.ascontiguousarray(hit_pos, np.float64)
    hit_cov = np.ascontiguousarray(hit_cov, np.float64)
    layers = np.ascontiguousarray(layers, np.float64)
    n = par.shape[0]
    L = hit_pos.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, np.float64)
    nl = None if nlay is None else np.ascontiguousarray(nlay, np.int32)
    gh = np.zeros((L, n, 3))
    gp = np.zeros((n, 6))
    fn = lib().kfo_grad_chi2 if precision == "f64" else lib().kfo_grad_chi2_f32
    rc = fn(int(geom), n, L, _p(layers, ctypes.c_double), float(bz),
                             _p(nl, ctypes.c_int32), _p(par, ctypes.c_double), _p(cov, ctypes.c_double),
                             _p(hit_pos, ctypes.c_double), _p(hit_cov, ctypes.c_double),
                             int(bool(joseph)), _p(w, ctypes.c_double), _p(gh, ctypes.c_double),
                             _p(gp, ctypes.c_double), _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return gh, gp


def filter_record(geom: int, par, cov, hit_pos, hit_cov, layers, bz: float, nlay=None, joseph=False,
                  precision: str = "f64", nthreads=None) -> dict:
    """The filter pass with what it computes on every layer k it applies:
    pred_p [L, n, 6] / pred_P [L, n, 6, 6] (propagated to layer k, before the
    update), F [L, n, 6, 6] (Jacobian of that propagation), filt_p / filt_P
    (after the update); plus chi2 [n] and status [n] as ``run`` returns them.
    Entries of layers a track did not apply are zero.  precision="f32" runs
    the filter in float arithmetic (tolerance sizing)."""
    par = np.ascontiguousarray(par, np.float64)
    cov = np.ascontiguousarray(cov, np.float64)
    hit_pos = np.ascontiguousarray(hit_pos, np.float64)
    hit_cov = np.ascontiguousarray(hit_cov, np.float64)
    layers = np.ascontiguousarray(layers, np.float64)
    n = par.shape[0]
    L = hit_pos.shape[0]
    nl = None if nlay is None else np.ascontiguousarray(nlay, np.int32)
    out = {k: np.zeros((L, n, w)) for k, w in (("pred_p", 6), ("pred_P", 21), ("F", 36), ("filt_p", 6),
                                               ("filt_P", 21))}
    chi2 = np.zeros(n)
    status = np.zeros(n, np.int32)
    c = ctypes.c_double
    rc = lib().kfo_filter_record(int(geom), n, L, _p(layers, c), float(bz), _p(nl, ctypes.c_int32), _p(par, c),
                                 _p(cov, c), _p(hit_pos, c), _p(hit_cov, c), int(bool(joseph)),
                                 _p(out["pred_p"], c), _p(out["pred_P"], c), _p(out["F"], c),
                                 _p(out["filt_p"], c), _p(out["filt_P"], c), _p(chi2, c),
                                 _p(status, ctypes.c_int32), 0 if precision == "f64" else 1, _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    out["pred_P"] = unpack_sym(out["pred_P"])
    out["filt_P"] = unpack_sym(out["filt_P"])
    out["F"] = out["F"].reshape(L, n, 6, 6)
    out["chi2"] = chi2
    out["status"] = status
    return out


def surface_basis(geom: int, p) -> np.ndarray:
    """[..., 6, 5]: orthonormal basis of the directions in which a state on
    its surface can vary -- the surface's five local coordinates.  On a plane
    z is fixed (x, y, kappa, phi, theta remain); on a cylinder the position
    moves along the tangent (-y, x)/r and along z."""
    p = np.asarray(p, np.float64)
    U = np.zeros(p.shape[:-1] + (6, 5))
    if geom == 0:
        for j, a in enumerate((0, 1, 3, 4, 5)):
            U[..., a, j] = 1.0
    else:
        r = np.hypot(p[..., 0], p[..., 1])
        r = np.where(r > 0, r, 1.0)
        U[..., 0, 0] = -p[..., 1] / r
        U[..., 1, 0] = p[..., 0] / r
        for j, a in enumerate((2, 3, 4, 5)):
            U[..., a, j + 1] = 1.0
    return U


def smooth(geom: int, par, cov, hit_pos, hit_cov, layers, bz: float, nlay=None, joseph=False,
           precision: str = "f64", nthreads=None, rec=None):
    """Rauch-Tung-Striebel smoother after the filter (the backward pass that
    turns the filter of Sec. 3.1 into a complete track fit): with the filtered
    state (p_k, C_k) on layer k, the prediction (q, P) and Jacobian F of the
    propagation from layer k to k + 1, and the smoothed state on k + 1,

        A    = C_k F^T P^-1
        p_k' = p_k + A (p_{k+1}' - q)
        C_k' = C_k + A (C_{k+1}' - P) A^T,

    starting from the filtered state of the last layer applied.  A state on a
    surface has five free coordinates (its covariance is singular along the
    surface normal in the six global ones), so every matrix above is taken in
    the local coordinates of its surface (``surface_basis`` at the predicted
    point: C_loc = U^T C U, F_loc = U_{k+1}^T F U_k, a displacement d maps to
    U^T d, and back by U).  Process noise is zero, as in the filter.

    Returns (sm_p [L, n, 6], sm_P [L, n, 21] packed, status [n], rec); layers
    a track did not apply are zero.  precision="f32": the filter and the
    recursion in float arithmetic (tolerance sizing)."""
    if rec is None:
        rec = filter_record(geom, par, cov, hit_pos, hit_cov, layers, bz, nlay, joseph, precision, nthreads)
    dt = np.float64 if precision == "f64" else np.float32
    L, n = rec["filt_p"].shape[:2]
    done = (rec["status"] >> 16).astype(np.int64)
    sm_p = np.zeros((L, n, 6))
    sm_P = np.zeros((L, n, 6, 6))
    last = done - 1
    have = done > 0
    idx = np.nonzero(have)[0]
    sm_p[last[idx], idx] = rec["filt_p"][last[idx], idx]
    sm_P[last[idx], idx] = rec["filt_P"][last[idx], idx]
    for k in range(L - 2, -1, -1):
        t = np.nonzero(k < done - 1)[0]
        if t.size == 0:
            continue
        Uk = surface_basis(geom, rec["pred_p"][k, t]).astype(dt)
        Un = surface_basis(geom, rec["pred_p"][k + 1, t]).astype(dt)
        UkT = np.swapaxes(Uk, -1, -2)
        UnT = np.swapaxes(Un, -1, -2)
        Ck = UkT @ rec["filt_P"][k, t].astype(dt) @ Uk
        Fl = UnT @ rec["F"][k + 1, t].astype(dt) @ Uk
        Pn = UnT @ rec["pred_P"][k + 1, t].astype(dt) @ Un
        A = Ck @ np.swapaxes(Fl, -1, -2) @ np.linalg.inv(Pn)
        d = UnT @ (sm_p[k + 1, t] - rec["pred_p"][k + 1, t]).astype(dt)[..., None]
        sm_p[k, t] = rec["filt_p"][k, t] + (Uk @ (A @ d))[..., 0]
        Cs = Ck + A @ (UnT @ sm_P[k + 1, t].astype(dt) @ Un - Pn) @ np.swapaxes(A, -1, -2)
        sm_P[k, t] = Uk @ Cs @ UkT
    return sm_p, pack_sym(sm_P), rec["status"], rec


def smooth_sample(sample: dict, **kw):
    """``smooth`` on a synthetic sample (single geometry)."""
    g = int(sample["geom"][0])
    layers = sample["layer_z"] if g == 0 else sample["layer_r"]
    return smooth(g, sample["par"], sample["cov"], sample["hit_pos"], sample["hit_cov"], layers, sample["bz"],
                  nlay=sample["nlay"], **kw)


def gate_run(geom: int, par, cov, cand_pos, cand_cov, layers, bz: float, gate: float, nlay=None, forced=None,
             joseph=False, precision: str = "f64", nthreads=None) -> dict:
    """The filter with hit selection among M candidate hits per layer: on
    every layer the candidate with the smallest update chi-square not above
    `gate` updates the state, or none (a hole: the state is the prediction);
    joseph=True takes that update in Joseph form.  cand_pos [L, n, M, 3], cand_cov [L, n, M, 6]; forced [L, n] int (the
    choices to follow instead, -1 a hole).  Returns par [n, 6], cov [n, 21],
    chi2 [n], status [n], chosen [L, n] (-2 where a layer was not processed)
    and cand_chi2 [L, n, M] (NaN for candidates that take no part)."""
    par = np.ascontiguousarray(par, np.float64)
    cov = np.ascontiguousarray(cov, np.float64)
    cand_pos = np.ascontiguousarray(cand_pos, np.float64)
    cand_cov = np.ascontiguousarray(cand_cov, np.float64)
    layers = np.ascontiguousarray(layers, np.float64)
    L, n, M = cand_pos.shape[:3]
    nl = None if nlay is None else np.ascontiguousarray(nlay, np.int32)
    fc = None if forced is None else np.ascontiguousarray(forced, np.int32)
    out = {"par": np.zeros((n, 6)), "cov": np.zeros((n, 21)), "chi2": np.zeros(n),
           "status": np.zeros(n, np.int32), "chosen": np.full((L, n), -2, np.int32),
           "cand_chi2": np.full((L, n, M), np.nan)}
    c = ctypes.c_double
    rc = lib().kfo_gate_run(int(geom), n, L, M, _p(layers, c), float(bz), _p(nl, ctypes.c_int32), _p(par, c),
                            _p(cov, c), _p(cand_pos, c), _p(cand_cov, c), float(gate), _p(fc, ctypes.c_int32),
                            int(bool(joseph)), _p(out["par"], c), _p(out["cov"], c), _p(out["chi2"], c),
                            _p(out["status"], ctypes.c_int32), _p(out["chosen"], ctypes.c_int32),
                            _p(out["cand_chi2"], c), 0 if precision == "f64" else 1, _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def gate_sample(sample: dict, mh: dict, gate: float, **kw) -> dict:
    """``gate_run`` on a synthetic sample and its candidate hits (synth.multi_hit)."""
    g = int(sample["geom"][0])
    layers = sample["layer_z"] if g == 0 else sample["layer_r"]
    return gate_run(g, sample["par"], sample["cov"], mh["cand_pos"], mh["cand_cov"], layers, sample["bz"], gate,
                    nlay=sample["nlay"], **kw)


def unpack_sym(P21) -> np.ndarray:
    """[..., 21] packed lower triangle -> [..., 6, 6] symmetric."""
    P21 = np.asarray(P21)
    n = int(round((np.sqrt(8 * P21.shape[-1] + 1) - 1) / 2))
    out = np.zeros(P21.shape[:-1] + (n, n), P21.dtype)
    k = 0
    for i in range(n):
        for j in range(i + 1):
            out[..., i, j] = P21[..., k]
            out[..., j, i] = P21[..., k]
            k += 1
    return out


def pack_sym(P) -> np.ndarray:
    """[..., n, n] -> [..., n(n+1)/2] packed lower triangle."""
    P = np.asarray(P)
    n = P.shape[-1]
    return np.stack([P[..., i, j] for i in range(n) for j in range(i + 1)], axis=-1)
