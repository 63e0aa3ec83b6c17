"""CPU oracle for the layer-wise WLS reference-map extrapolation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline
leg are the only callers.  The product path never imports this package.  The compiled
part (``rmx_oracle.c``) shares no code with the GPU library; this module only marshals
numpy arrays into it.

What it computes follows Lin, Derr & Rycroft (arXiv 2104.00095): section "Extrapolation
of xi(x,t)" and the SI section "Weighting scheme for weighted least squares-based
extrapolation", eq. (weight) (``rmx_oracle.c``); the SI "Timestepping algorithm",
steps 5-7 and 11, with the advective term of eq. (adv_terms) and the Godunov face states
of "Evaluating the advective term" (``rmx_step_oracle.c``); and the blur-zone consumers:
eq. (sm_heavi), eq. (mod_heaviside) and the neo-Hookean solid stress of SI "Stress
calculations" (``rmx_blur_oracle.c``).  See the C files for the
step-by-step account.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmx_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "rmx_step_oracle.c"), os.path.join(_HERE, "rmx_blur_oracle.c")]
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
        ("adjacency", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("spacing", ctypes.c_double * 3),
    ]


class BlurSolid(ctypes.Structure):
    _fields_ = [
        ("lo", ctypes.c_int32 * 3),
        ("ext", ctypes.c_int32 * 3),
        ("shape", Shape),
        ("n_layers", ctypes.c_int32),
        ("xi", ctypes.c_void_p),
        ("labels", ctypes.c_void_p),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
             "-Wall", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _stale() -> bool:
    return not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                           for f in _SRCS)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
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
        L.orc_predict.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 8
        L.orc_predict.restype = ctypes.c_int
        L.orc_correct.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 5
        L.orc_correct.restype = None
        L.orc_slope4.argtypes = [ctypes.c_void_p]
        L.orc_slope4.restype = ctypes.c_double
        L.orc_heaviside_eps.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_heaviside_eps.restype = ctypes.c_double
        L.orc_blur.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, P(BlurSolid),
                               ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_blur.restype = None
        L.orc_solid_stress.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       P(BlurSolid), ctypes.c_double, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]
        L.orc_solid_stress.restype = None
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
                 normal_layers=2, adjacency=6, periodic=(0, 0, 0),
                 spacing=(1.0, 1.0, 1.0)) -> Problem:
    """One solid's extrapolation problem.  ``spacing``: the cell sizes along x, y, z
    (only their ratios matter to the extrapolation); ``periodic``: the axes along which
    the grid wraps (no walls there; the box may run past the grid's end)."""
    p = Problem()
    p.grid_n[:] = [int(v) for v in grid_n]
    p.lo[:] = [int(v) for v in lo]
    p.ext[:] = [int(v) for v in ext]
    p.shape = shape
    p.n_layers = int(n_layers)
    p.r_s, p.r_max, p.normal_layers = int(r_s), int(r_max), int(normal_layers)
    p.adjacency = int(adjacency)
    p.periodic[:] = [1 if v else 0 for v in periodic]
    p.spacing[:] = [float(v) for v in spacing]
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


# ---------------------------------------------------------------------------------------
# Time step around the extrapolation (SI "Timestepping algorithm", steps 5-7 and 11).
# ---------------------------------------------------------------------------------------
def slope4(q) -> float:
    """Colella's fourth-order limited slope at the centre of five values."""
    a = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(5))
    return float(lib().orc_slope4(_ptr(a)))


def _spacing(h):
    """A spacing given as one number (isotropic) or as (Delta_x, Delta_y, Delta_z)."""
    v = np.asarray(h, dtype=np.float64).reshape(-1)
    return np.ascontiguousarray(np.repeat(v, 3) if v.size == 1 else v.reshape(3))


def _periodic(periodic):
    return np.ascontiguousarray(np.asarray([1 if v else 0 for v in (periodic or (0, 0, 0))],
                                           dtype=np.int32))


def predict(ext, n_layers, xi_n, labels_n, u, uf, dt, h, xi_next):
    """Step 5: writes the predictor into ``xi_next`` (float64 [3, e2, e1, e0], modified in
    place: predicted cells get the value, the rest of the old band NaN, unmarked cells
    are left as they are).  ``uf`` = (x-faces [e2, e1, e0+1], y-faces [e2, e1+1, e0],
    z-faces [e2+1, e1, e0]).  ``h``: the spacing, one number or one per axis.  Returns 1
    if an interior cell could not be predicted."""
    e = np.ascontiguousarray(np.asarray(ext, dtype=np.int32))
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (xi_n, u) + tuple(uf)]
    lab = np.ascontiguousarray(labels_n, dtype=np.int8)
    assert xi_next.flags.c_contiguous and xi_next.dtype == np.float64
    lam = np.ascontiguousarray([float(dt) / float(d) for d in _spacing(h)])
    return int(lib().orc_predict(_ptr(e), int(n_layers), _ptr(arrs[0]), _ptr(lab),
                                 _ptr(arrs[1]), _ptr(arrs[2]), _ptr(arrs[3]), _ptr(arrs[4]),
                                 _ptr(lam), _ptr(xi_next)))


def correct(ext, n_layers, xi_n, labels_n, xi_next, labels_next, xi_half):
    """Step 7: writes xi^{n+1/2} into ``xi_half`` (modified in place) on the cells labelled
    at step n + 1."""
    e = np.ascontiguousarray(np.asarray(ext, dtype=np.int32))
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (xi_n, xi_next)]
    ln = np.ascontiguousarray(labels_n, dtype=np.int8)
    lx = np.ascontiguousarray(labels_next, dtype=np.int8)
    lib().orc_correct(_ptr(e), int(n_layers), _ptr(a[0]), _ptr(ln), _ptr(a[1]), _ptr(lx),
                      _ptr(xi_half))


def step(problem: Problem, xi_n, labels_n, u, uf, dt, h, xi_next_init, xi_half_init,
         nthreads: int = 0):
    """One time step of the reference map around the extrapolation, in the paper's order:
    predictor (step 5) -> extrapolation from the predicted interior (step 6) -> corrector
    (step 7).  Restoring xi^{n+1} (step 11) is keeping the returned xi_next.

    The extrapolation sees the predicted cells only: every other cell is undefined for
    it, so the interior at n + 1 is the predicted cells with phi0(xi^{n+1}) < 0.  The
    returned xi_next holds the predictor on the predicted cells, NaN on the rest of the
    old band, the extrapolated band at n + 1, and the caller's values elsewhere.
    Returns (status, xi_next, labels_next, decisions, stats, xi_half)."""
    e = tuple(int(v) for v in problem.ext)
    L = int(problem.n_layers)
    xi_next = np.ascontiguousarray(xi_next_init, dtype=np.float64).copy()
    trunc = predict(e, L, xi_n, labels_n, u, uf, dt, h, xi_next)
    # the field the extrapolation is given: the predicted cells, undefined elsewhere
    lab_n = np.asarray(labels_n)
    pred = (lab_n >= 0) & (lab_n <= L - 4)
    kk, jj, ii = np.meshgrid(np.arange(e[2]), np.arange(e[1]), np.arange(e[0]), indexing="ij")
    pred &= (ii >= 3) & (ii <= e[0] - 4) & (jj >= 3) & (jj <= e[1] - 4) & (kk >= 3) & \
        (kk <= e[2] - 4)
    work = np.where(pred[None], xi_next, np.nan)
    st, ext_out, labels_next, dec, stats = extrapolate(problem, work, nthreads=nthreads)
    if trunc and st >= 0:
        st = E_TRUNCATED
    if st == OK:
        band = (labels_next >= 1) & (labels_next <= L)
        xi_next = np.where(band[None], ext_out, xi_next)
    xi_half = np.ascontiguousarray(xi_half_init, dtype=np.float64).copy()
    if st == OK:
        correct(e, L, xi_n, labels_n, xi_next, labels_next, xi_half)
    return st, xi_next, labels_next, dec, stats, xi_half


# ---------------------------------------------------------------------------------------
# Blur-zone consumers (eq. (sm_heavi), eq. (mod_heaviside), SI "Stress calculations").
# ---------------------------------------------------------------------------------------
def heaviside_eps(phi: float, eps: float) -> float:
    return float(lib().orc_heaviside_eps(float(phi), float(eps)))


def _blur_solids(solids):
    """solids: sequence of (lo, ext, Shape, n_layers, xi [3,e2,e1,e0], labels [e2,e1,e0])."""
    keep = []
    arr = (BlurSolid * len(solids))()
    for m, (lo, ext, shape, L, xi, labels) in enumerate(solids):
        x = np.ascontiguousarray(xi, dtype=np.float64)
        lab = np.ascontiguousarray(labels, dtype=np.int8)
        keep += [x, lab]
        arr[m].lo[:] = [int(v) for v in lo]
        arr[m].ext[:] = [int(v) for v in ext]
        arr[m].shape = shape
        arr[m].n_layers = int(L)
        arr[m].xi = x.ctypes.data
        arr[m].labels = lab.ctypes.data
    return arr, keep


def blur(grid_n, solids, eps, H_init, phi_init=None, periodic=None):
    """Modified Heaviside on the grid (written on cells inside some box; H_init elsewhere)
    and, if phi_init (one array per solid) is given, phi_m on each box's labelled cells.
    ``periodic``: the axes along which the grid wraps.  Returns (H, [phi_m])."""
    arr, keep = _blur_solids(solids)
    g = np.ascontiguousarray(np.asarray(grid_n, dtype=np.int32))
    H = np.ascontiguousarray(H_init, dtype=np.float64).copy()
    phis = None
    pp = None
    if phi_init is not None:
        phis = [np.ascontiguousarray(p, dtype=np.float64).copy() for p in phi_init]
        pp = (ctypes.c_void_p * len(phis))(*[p.ctypes.data for p in phis])
    per = _periodic(periodic)
    lib().orc_blur(_ptr(g), _ptr(per), len(solids), arr, float(eps), _ptr(H), pp)
    return H, phis


def solid_stress(grid_n, solids, eps, h, G, tau_init, periodic=None):
    """Blended neo-Hookean stress on the faces: tau_init = three arrays
    [6, n2 + (a==2), n1 + (a==1), n0 + (a==0)], without the extra face along a periodic
    axis a (faces without a cell in any box keep them).  ``h``: the spacing, one number
    or one per axis.  Returns the three arrays."""
    arr, keep = _blur_solids(solids)
    g = np.ascontiguousarray(np.asarray(grid_n, dtype=np.int32))
    Gs = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
    tau = [np.ascontiguousarray(t, dtype=np.float64).copy() for t in tau_init]
    tp = (ctypes.c_void_p * 3)(*[t.ctypes.data for t in tau])
    per = _periodic(periodic)
    hs = _spacing(h)
    for a in range(3):
        want = [int(grid_n[2]), int(grid_n[1]), int(grid_n[0])]
        if not per[a]:
            want[2 - a] += 1
        assert tau[a].shape == (6, *want), (a, tau[a].shape, want)
    lib().orc_solid_stress(_ptr(g), _ptr(per), len(solids), arr, float(eps), _ptr(hs),
                           _ptr(Gs), tp)
    return tau
