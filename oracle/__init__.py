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


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math: IEEE results)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, f, i32, u32 = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float),
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32))
        c_int, c_i64, c_dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.kfo_run_f64.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, d, d, d, d, c_int, d, d, d, i32, c_int]
        L.kfo_run_f32.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, f, f, f, f, c_int, f, f, f, i32, c_int]
        L.kfo_propagate.argtypes = [c_int, d, c_dbl, c_dbl, d, d, u32]
        L.kfo_update.argtypes = [d, d, d, d, c_int, d, d, d, u32]
        L.kfo_grad_chi2.argtypes = [c_int, c_i64, c_int, d, c_dbl, i32, d, d, d, d, c_int, d, d, d, c_int]
        L.kfo_grad_chi2_f32.argtypes = L.kfo_grad_chi2.argtypes
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
