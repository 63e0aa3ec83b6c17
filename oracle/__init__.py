"""CPU oracle for the layer-wise WLS reference-map extrapolation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline
leg are the only callers.  The product path never imports this package.  The compiled
part (``rmx_oracle.c``) shares no code with the GPU library; this module only marshals
numpy arrays into it.

What it computes follows Lin, Derr & Rycroft (arXiv 2104.00095): section "Extrapolation
of xi(x,t)" and the SI section "Weighting scheme for weighted least squares-based
extrapolation", eq. (weight).  See ``rmx_oracle.c`` for the step-by-step account.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmx_oracle.c")
_LIB = os.path.join(_HERE, "librmx_oracle.so")

# Decision codes (one per cell): 0 = not a band cell, r = fitted with search radius r,
# 32 = F1 (normal factor dropped), 33 = F2 (kernel-weighted mean); +64 = no normal.
DEC_F1 = 32
DEC_F2 = 33
DEC_NO_NORMAL = 64
N_STATS = 21

OK, W_EMPTY, E_ARG, E_BOX, E_LAYERS, E_SHAPE, E_TRUNCATED = 0, 1, -1, -2, -3, -4, -7


class Shape(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("centre", ctypes.c_double * 3),
        ("semi", ctypes.c_double * 3),
        ("rot", ctypes.c_double * 9),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("grid_n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_int32 * 3),
        ("ext", ctypes.c_int32 * 3),
        ("shape", Shape),
        ("n_layers", ctypes.c_int32),
        ("r_s", ctypes.c_int32),
        ("r_max", ctypes.c_int32),
        ("normal_layers", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
             "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        L.orc_extrapolate.argtypes = [P(Problem), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int32]
        L.orc_extrapolate.restype = ctypes.c_int
        L.orc_label.argtypes = [P(Problem), ctypes.c_void_p, ctypes.c_void_p,
                                P(ctypes.c_int32)]
        L.orc_label.restype = ctypes.c_int64
        L.orc_phi0.argtypes = [P(Shape), ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_phi0.restype = ctypes.c_double
        L.orc_is_interior.argtypes = [P(Shape), ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double]
        L.orc_is_interior.restype = ctypes.c_int
        L.orc_full_rank.argtypes = [ctypes.c_int32, ctypes.c_void_p]
        L.orc_full_rank.restype = ctypes.c_int
        L.orc_normal.argtypes = [P(Problem), ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_void_p]
        L.orc_normal.restype = None
        _lib = L
    return _lib


def make_shape(kind, centre, semi, rot=None) -> Shape:
    s = Shape()
    s.kind = int(kind)
    s.centre[:] = [float(v) for v in centre]
    semi = list(semi) + [0.0] * (3 - len(semi))
    s.semi[:] = [float(v) for v in semi]
    r = np.eye(3) if rot is None else np.asarray(rot, dtype=np.float64).reshape(3, 3)
    s.rot[:] = [float(v) for v in r.reshape(-1)]
    return s


def make_problem(grid_n, lo, ext, shape: Shape, n_layers, r_s=2, r_max=4,
                 normal_layers=2) -> Problem:
    p = Problem()
    p.grid_n[:] = [int(v) for v in grid_n]
    p.lo[:] = [int(v) for v in lo]
    p.ext[:] = [int(v) for v in ext]
    p.shape = shape
    p.n_layers = int(n_layers)
    p.r_s, p.r_max, p.normal_layers = int(r_s), int(r_max), int(normal_layers)
    return p


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def extrapolate(problem: Problem, xi: np.ndarray, xi_normal: np.ndarray | None = None,
                nthreads: int = 0):
    """Run the oracle on one solid.  ``xi`` is float64 [3, ext2, ext1, ext0] and is NOT
    modified; returns (status, xi_out, labels, decisions, stats)."""
    e = tuple(int(v) for v in problem.ext)
    xi_out = np.ascontiguousarray(xi, dtype=np.float64).copy()
    assert xi_out.shape == (3, e[2], e[1], e[0]), xi_out.shape
    xn = None
    if xi_normal is not None:
        xn = np.ascontiguousarray(xi_normal, dtype=np.float64)
        assert xn.shape == xi_out.shape
    labels = np.empty((e[2], e[1], e[0]), dtype=np.int8)
    dec = np.empty((e[2], e[1], e[0]), dtype=np.int8)
    stats = np.zeros(N_STATS, dtype=np.int64)
    st = lib().orc_extrapolate(ctypes.byref(problem), _ptr(xi_out), _ptr(xn), _ptr(labels),
                               _ptr(dec), _ptr(stats), int(nthreads))
    return st, xi_out, labels, dec, stats


def label(problem: Problem, xi: np.ndarray):
    """Classification and breadth-first layer labels only: (n_interior or status,
    labels, truncated)."""
    e = tuple(int(v) for v in problem.ext)
    x = np.ascontiguousarray(xi, dtype=np.float64)
    labels = np.empty((e[2], e[1], e[0]), dtype=np.int8)
    tr = ctypes.c_int32(0)
    n = lib().orc_label(ctypes.byref(problem), _ptr(x), _ptr(labels), ctypes.byref(tr))
    return int(n), labels, bool(tr.value)


def phi0(shape: Shape, v) -> float:
    return float(lib().orc_phi0(ctypes.byref(shape), float(v[0]), float(v[1]), float(v[2])))


def is_interior(shape: Shape, v) -> bool:
    return bool(lib().orc_is_interior(ctypes.byref(shape), float(v[0]), float(v[1]),
                                      float(v[2])))


def full_rank(points) -> bool:
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int32).reshape(-1, 3))
    return bool(lib().orc_full_rank(int(pts.shape[0]), _ptr(pts)))


def normal(problem: Problem, field: np.ndarray, i: int, j: int, k: int) -> np.ndarray:
    g = np.zeros(3, dtype=np.float64)
    f = np.ascontiguousarray(field, dtype=np.float64)
    lib().orc_normal(ctypes.byref(problem), _ptr(f), int(i), int(j), int(k), _ptr(g))
    return g
