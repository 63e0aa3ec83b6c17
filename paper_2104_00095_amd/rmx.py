"""Thin ctypes binding of librmx.so (include/rmx.h).

Argument marshalling only: every step of the extrapolation runs in the HIP library.
Device buffers are torch tensors on a ROCm device (PyTorch provides memory and streams).
The library is loaded from this package directory; if it is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmx.so")

OK, W_EMPTY = 0, 1
E_ARG, E_BOX, E_LAYERS, E_SHAPE, E_WORKSPACE, E_HIP = -1, -2, -3, -4, -5, -6
E_TRUNCATED, E_BUDGET, E_BUSY, E_NOTFOUND, E_DISABLED = -7, -8, -9, -10, -11
SPHERE, ELLIPSOID = 1, 2
FP64, FP32_ACCUM = 0, 1
FLAG_SYNC, FLAG_GRAPH, FLAG_PER_SOLID, FLAG_PROFILE, FLAG_PERSISTENT = 1, 2, 4, 8, 16
FLAG_ADJ26 = 32
N_PHASES = 24
PHASES = ["classify", "label", "normal"] + [f"extrap{l}" for l in range(1, 17)] + \
    ["band", "step_trans", "step_predict", "step_correct", "step_faces"]
MAX_LAYERS = 16
DEC_F1, DEC_F2, DEC_NO_NORMAL = 32, 33, 64

EXPORTS = [
    "rmx_default_options", "rmx_create", "rmx_destroy", "rmx_workspace_size",
    "rmx_extrapolate", "rmx_status_string", "rmx_server_create", "rmx_server_register",
    "rmx_server_field", "rmx_server_submit", "rmx_server_wait", "rmx_server_release",
    "rmx_server_usage", "rmx_server_destroy", "rmx_profile_read", "rmx_autotune",
    "rmx_set_tuning", "rmx_extrapolate_noalloc", "rmx_step", "rmx_blur", "rmx_solid_stress",
    "rmx_layers_for_blur",
    "rmx_layers_for_blur_grid",
]


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("periodic", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32)]


class Shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("centre", ctypes.c_double * 3),
                ("semi_axes", ctypes.c_double * 3), ("rot", ctypes.c_double * 9)]


class Solid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("ext", ctypes.c_int32 * 3), ("phi0", Shape),
                ("n_layers", ctypes.c_int32), ("xi", ctypes.c_void_p),
                ("xi_normal", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("decisions", ctypes.c_void_p)]


class StepSolid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("ext", ctypes.c_int32 * 3), ("phi0", Shape),
                ("n_layers", ctypes.c_int32), ("xi_n", ctypes.c_void_p),
                ("labels_n", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("uf", ctypes.c_void_p * 3), ("xi_next", ctypes.c_void_p),
                ("labels_next", ctypes.c_void_p), ("xi_half", ctypes.c_void_p),
                ("decisions", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("r_s", ctypes.c_int32), ("r_max", ctypes.c_int32),
                ("normal_layers", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("extrap_blocks", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class SolidStats(ctypes.Structure):
    _fields_ = [("n_interior", ctypes.c_int64), ("n_band", ctypes.c_int64 * (MAX_LAYERS + 1)),
                ("n_r_grown", ctypes.c_int64), ("n_no_normal", ctypes.c_int64),
                ("n_f1", ctypes.c_int64), ("n_f2", ctypes.c_int64),
                ("status", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self):
        return {"n_interior": self.n_interior, "n_band": list(self.n_band),
                "n_r_grown": self.n_r_grown, "n_no_normal": self.n_no_normal,
                "n_f1": self.n_f1, "n_f2": self.n_f2, "status": self.status}


class RmxError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: rmx status {status} ({status_string(status)})")


_lib = None


def lib():
    """Load librmx.so; raise loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librmx.so not found at {LIB_PATH}; build it with "
                               "`python -m paper_2104_00095_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.rmx_default_options.argtypes = [P(Options)]
        L.rmx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, P(vp)]
        L.rmx_destroy.argtypes = [vp]
        L.rmx_workspace_size.argtypes = [P(Grid), P(Solid), ctypes.c_int32, P(Options),
                                         P(ctypes.c_size_t)]
        L.rmx_extrapolate.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32, P(Options), vp,
                                      P(SolidStats)]
        L.rmx_status_string.argtypes = [ctypes.c_int]
        L.rmx_status_string.restype = ctypes.c_char_p
        L.rmx_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int32, P(vp)]
        L.rmx_server_register.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32,
                                          P(ctypes.c_int64)]
        L.rmx_server_field.argtypes = [vp, ctypes.c_int64, ctypes.c_int32,
                                       P(P(ctypes.c_double)), P(P(ctypes.c_int8))]
        L.rmx_server_submit.argtypes = [vp, ctypes.c_int64, P(Options), P(ctypes.c_int64)]
        L.rmx_server_wait.argtypes = [vp, ctypes.c_int64, P(SolidStats), P(ctypes.c_double)]
        L.rmx_server_release.argtypes = [vp, ctypes.c_int64]
        L.rmx_server_usage.argtypes = [vp, P(ctypes.c_size_t), P(ctypes.c_size_t)]
        L.rmx_server_destroy.argtypes = [vp]
        L.rmx_profile_read.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
        L.rmx_autotune.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32, P(Options), vp,
                                   ctypes.c_int32, P(Tuning)]
        L.rmx_extrapolate_noalloc.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32,
                                              P(Options), vp, P(SolidStats)]
        L.rmx_set_tuning.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32, P(Options),
                                     P(Tuning)]
        L.rmx_step.argtypes = [vp, P(Grid), P(StepSolid), ctypes.c_int32, P(Options),
                               ctypes.c_double, vp, P(SolidStats)]
        L.rmx_blur.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32, ctypes.c_double, vp, vp,
                               vp]
        L.rmx_layers_for_blur_grid.argtypes = [P(Grid), ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int32, ctypes.c_uint32,
                                               P(ctypes.c_int32)]
        L.rmx_layers_for_blur.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_uint32, P(ctypes.c_int32)]
        L.rmx_solid_stress.argtypes = [vp, P(Grid), P(Solid), ctypes.c_int32, ctypes.c_double,
                                       vp, vp, vp]
        for name in EXPORTS:
            if name != "rmx_status_string":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(st: int) -> str:
    try:
        return lib().rmx_status_string(int(st)).decode()
    except Exception:  # noqa: BLE001 - only used for messages
        return "?"


def options(r_s=2, r_max=4, normal_layers=2, precision=FP64, flags=0) -> Options:
    o = Options()
    o.r_s, o.r_max, o.normal_layers, o.precision, o.flags = (
        int(r_s), int(r_max), int(normal_layers), int(precision), int(flags))
    return o


def grid(n, h, origin=(0.0, 0.0, 0.0), spacing=None, periodic=None) -> Grid:
    """spacing: per-axis cell sizes (0 or None: h); periodic: axes along which the grid
    wraps."""
    g = Grid()
    g.n[:] = [int(v) for v in n]
    g.h = float(h)
    g.origin[:] = [float(v) for v in origin]
    g.spacing[:] = [float(v) for v in (spacing or (0.0, 0.0, 0.0))]
    g.periodic[:] = [1 if v else 0 for v in (periodic or (0, 0, 0))]
    return g


def shape(kind, centre, semi, rot=None) -> Shape:
    s = Shape()
    s.kind = int(kind)
    s.centre[:] = [float(v) for v in centre]
    semi = list(semi) + [0.0] * (3 - len(semi))
    s.semi_axes[:] = [float(v) for v in semi[:3]]
    flat = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    if rot is not None:
        flat = [float(v) for v in (rot.reshape(-1) if hasattr(rot, "reshape") else rot)]
    s.rot[:] = flat
    return s


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(int(t.data_ptr()))


def solid_template(lo, ext, shp: Shape, n_layers) -> Solid:
    """A solid without fields: for rmx_server_register (the server allocates them) and
    rmx_workspace_size."""
    s = Solid()
    s.lo[:] = [int(v) for v in lo]
    s.ext[:] = [int(v) for v in ext]
    s.phi0 = shp
    s.n_layers = int(n_layers)
    return s


def workspace_size(g: Grid, solids: Sequence[Solid], opt: Optional[Options] = None) -> int:
    arr = (Solid * len(solids))(*solids)
    n = ctypes.c_size_t(0)
    st = lib().rmx_workspace_size(ctypes.byref(g), arr, len(solids),
                                  ctypes.byref(opt) if opt else None, ctypes.byref(n))
    if st != OK:
        raise RmxError(st, "rmx_workspace_size")
    return int(n.value)


def solid(lo, ext, shp: Shape, n_layers, xi, labels, xi_normal=None, decisions=None) -> Solid:
    """xi: cuda float64 [3, ext2, ext1, ext0]; labels: cuda int8 [ext2, ext1, ext0]."""
    e = tuple(int(v) for v in ext)
    assert tuple(xi.shape) == (3, e[2], e[1], e[0]) and xi.is_contiguous(), xi.shape
    assert tuple(labels.shape) == (e[2], e[1], e[0]) and labels.is_contiguous()
    s = Solid()
    s.lo[:] = [int(v) for v in lo]
    s.ext[:] = list(e)
    s.phi0 = shp
    s.n_layers = int(n_layers)
    s.xi = _ptr(xi)
    s.xi_normal = _ptr(xi_normal)
    s.labels = _ptr(labels)
    s.decisions = _ptr(decisions)
    # keep the tensors alive with the descriptor
    s._keep = (xi, labels, xi_normal, decisions)
    return s


def layers_for_blur(eps: float, h: float, stretch: float = 1.0, reach: int = 0,
                    flags: int = 0) -> int:
    """Layer count whose band covers the blur zone (rmx_layers_for_blur)."""
    out = ctypes.c_int32(0)
    st = lib().rmx_layers_for_blur(float(eps), float(h), float(stretch), int(reach),
                                   int(flags), ctypes.byref(out))
    if st != OK:
        raise RmxError(st, "rmx_layers_for_blur")
    return int(out.value)


def layers_for_blur_grid(g: Grid, eps: float, stretch: float = 1.0, reach: int = 0,
                         flags: int = 0) -> int:
    """Layer count whose band covers the blur zone on a grid with unequal spacings
    (rmx_layers_for_blur_grid)."""
    out = ctypes.c_int32(0)
    st = lib().rmx_layers_for_blur_grid(ctypes.byref(g), float(eps), float(stretch),
                                        int(reach), int(flags), ctypes.byref(out))
    if st != OK:
        raise RmxError(st, "rmx_layers_for_blur_grid")
    return int(out.value)


def step_solid(lo, ext, shp: Shape, n_layers, xi_n, labels_n, u, uf, xi_next, labels_next,
               xi_half, decisions=None) -> StepSolid:
    """One solid's buffers for rmx_step (cuda tensors): xi_n, u, xi_next, xi_half float64
    [3, e2, e1, e0]; labels_n, labels_next int8 [e2, e1, e0]; uf = (x-faces float64
    [e2, e1, e0+1], y-faces [e2, e1+1, e0], z-faces [e2+1, e1, e0])."""
    e = tuple(int(v) for v in ext)
    f3 = (3, e[2], e[1], e[0])
    for t in (xi_n, u, xi_next, xi_half):
        assert tuple(t.shape) == f3 and t.is_contiguous(), t.shape
    for t in (labels_n, labels_next):
        assert tuple(t.shape) == f3[1:] and t.is_contiguous(), t.shape
    for a, want in enumerate([(e[2], e[1], e[0] + 1), (e[2], e[1] + 1, e[0]),
                              (e[2] + 1, e[1], e[0])]):
        assert tuple(uf[a].shape) == want and uf[a].is_contiguous(), (a, uf[a].shape)
    s = StepSolid()
    s.lo[:] = [int(v) for v in lo]
    s.ext[:] = list(e)
    s.phi0 = shp
    s.n_layers = int(n_layers)
    s.xi_n, s.labels_n, s.u = _ptr(xi_n), _ptr(labels_n), _ptr(u)
    s.uf[:] = [_ptr(t) for t in uf]
    s.xi_next, s.labels_next, s.xi_half = _ptr(xi_next), _ptr(labels_next), _ptr(xi_half)
    s.decisions = _ptr(decisions)
    s._keep = (xi_n, labels_n, u, tuple(uf), xi_next, labels_next, xi_half, decisions)
    return s


def _check_size(t, n, what):
    """A float64 buffer of at least n elements (None passes: the entry point decides)."""
    if t is None or not hasattr(t, "numel"):
        return
    if t.numel() < n or getattr(t, "element_size", lambda: 8)() != 8:
        raise ValueError(f"{what}: need {n} float64 elements, got {t.numel()} of "
                         f"{t.element_size()} bytes")


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _torch_device_first(device: int):  # noqa: ARG001 - every device is initialised
    """Initialise torch's GPU runtime before the library's.  PyTorch wheels for ROCm carry
    their own copy of the HIP and HSA runtimes; when the library's (system) runtime opens
    the device first, torch's copy then finds no GPU.  Initialised in this order, both
    work on the same device, and torch tensors can be passed to the library."""
    try:
        import torch
    except ImportError:   # the C ABI alone needs no torch
        return
    if torch.cuda.is_available():
        torch.cuda.init()


class Context:
    """An rmx context on one device (workspace, graph cache)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        _torch_device_first(device)
        self.h = ctypes.c_void_p()
        st = lib().rmx_create(int(device), int(workspace_bytes), ctypes.byref(self.h))
        if st != OK:
            raise RmxError(st, "rmx_create")

    def close(self):
        if self.h:
            lib().rmx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def workspace_size(self, g: Grid, solids: Sequence[Solid], opt: Optional[Options] = None):
        arr = (Solid * len(solids))(*solids)
        n = ctypes.c_size_t(0)
        st = lib().rmx_workspace_size(ctypes.byref(g), arr, len(solids),
                                      ctypes.byref(opt) if opt else None, ctypes.byref(n))
        if st != OK:
            raise RmxError(st, "rmx_workspace_size")
        return int(n.value)

    def extrapolate(self, g: Grid, solids: Sequence[Solid], opt: Optional[Options] = None,
                    stream=None, want_stats: bool = True, check: bool = True):
        """Run one call; returns (status, [stats dict per solid] or None)."""
        arr = (Solid * len(solids))(*solids)
        stats = (SolidStats * len(solids))() if want_stats else None
        st = lib().rmx_extrapolate(self.h, ctypes.byref(g), arr, len(solids),
                                   ctypes.byref(opt) if opt else None, _stream_handle(stream),
                                   stats)
        if check and st < 0 and st != E_TRUNCATED:
            raise RmxError(st, "rmx_extrapolate")
        return st, ([s.as_dict() for s in stats] if want_stats else None)

    def extrapolate_noalloc(self, g: Grid, solids: Sequence[Solid],
                            opt: Optional[Options] = None, stream=None,
                            want_stats: bool = True, check: bool = True):
        """The allocation-free call (rmx_extrapolate_noalloc): same results, the workspace
        is the library's fixed per-device array; returns (status, [stats] or None)."""
        arr = (Solid * len(solids))(*solids)
        stats = (SolidStats * len(solids))() if want_stats else None
        st = lib().rmx_extrapolate_noalloc(self.h, ctypes.byref(g), arr, len(solids),
                                           ctypes.byref(opt) if opt else None,
                                           _stream_handle(stream), stats)
        if check and st < 0 and st != E_TRUNCATED:
            raise RmxError(st, "rmx_extrapolate_noalloc")
        return st, ([s.as_dict() for s in stats] if want_stats else None)

    def step(self, g: Grid, solids: Sequence[StepSolid], dt: float,
             opt: Optional[Options] = None, stream=None, want_stats: bool = True,
             check: bool = True):
        """One time step of every solid (rmx_step): predictor, extrapolation from the
        predicted interior, corrector; returns (status, [stats dict per solid] or None)."""
        arr = (StepSolid * len(solids))(*solids)
        stats = (SolidStats * len(solids))() if want_stats else None
        st = lib().rmx_step(self.h, ctypes.byref(g), arr, len(solids),
                            ctypes.byref(opt) if opt else None, float(dt),
                            _stream_handle(stream), stats)
        if check and st < 0 and st != E_TRUNCATED:
            raise RmxError(st, "rmx_step")
        return st, ([s.as_dict() for s in stats] if want_stats else None)

    def step_raw(self, g: Grid, arr, n: int, opt: Options, dt: float, stream_handle):
        """rmx_step on a prebuilt StepSolid array, no statistics (timing loops)."""
        return lib().rmx_step(self.h, ctypes.byref(g), arr, n, ctypes.byref(opt), float(dt),
                              stream_handle, None)

    def blur(self, g: Grid, solids: Sequence[Solid], eps: float, H=None, phis=None,
             stream=None):
        """Modified Heaviside on the grid (rmx_blur): H cuda float64 [n2, n1, n0] (cells
        inside some box are written), phis: per solid a cuda float64 [e2, e1, e0] or None."""
        n0, n1, n2 = g.n
        _check_size(H, n0 * n1 * n2, "H")
        for i, p in enumerate(phis or []):
            e = solids[i].ext
            _check_size(p, e[0] * e[1] * e[2], f"phis[{i}]")
        arr = (Solid * len(solids))(*solids)
        pp = None
        if phis is not None:
            pp = (ctypes.c_void_p * len(solids))(*[_ptr(p) for p in phis])
        st = lib().rmx_blur(self.h, ctypes.byref(g), arr, len(solids), float(eps), _ptr(H),
                            pp, _stream_handle(stream))
        if st != OK:
            raise RmxError(st, "rmx_blur")

    def blur_raw(self, g: Grid, arr, n: int, eps: float, H_ptr, phi_ptrs, stream_handle):
        """rmx_blur on a prebuilt Solid array and raw device pointers, no checks (timing
        loops); returns the status."""
        return lib().rmx_blur(self.h, ctypes.byref(g), arr, n, float(eps), H_ptr, phi_ptrs,
                              stream_handle)

    def solid_stress_raw(self, g: Grid, arr, n: int, eps: float, G_arr, tau_ptrs,
                         stream_handle):
        """rmx_solid_stress on prebuilt arrays, no checks (timing loops); returns the
        status."""
        return lib().rmx_solid_stress(self.h, ctypes.byref(g), arr, n, float(eps), G_arr,
                                      tau_ptrs, stream_handle)

    def solid_stress(self, g: Grid, solids: Sequence[Solid], eps: float, G, taus,
                     stream=None):
        """Blended neo-Hookean solid stress on the faces (rmx_solid_stress): taus = three
        cuda float64 arrays [6, n2 + (a==2), n1 + (a==1), n0 + (a==0)], without the extra
        face along a periodic axis a; G: one shear modulus per solid."""
        for a in range(3):
            n = [int(v) for v in g.n]
            if not g.periodic[a]:
                n[a] += 1
            _check_size(taus[a], 6 * n[0] * n[1] * n[2], f"taus[{a}]")
        arr = (Solid * len(solids))(*solids)
        Gs = (ctypes.c_double * len(solids))(*[float(v) for v in G])
        tp = (ctypes.c_void_p * 3)(*[_ptr(t) for t in taus])
        st = lib().rmx_solid_stress(self.h, ctypes.byref(g), arr, len(solids), float(eps), Gs,
                                    tp, _stream_handle(stream))
        if st != OK:
            raise RmxError(st, "rmx_solid_stress")

    def set_tuning(self, g: Grid, solids: Sequence[Solid], tile_w: int, extrap_blocks: int,
                   opt: Optional[Options] = None):
        """Keep the given launch shapes for this batch's shape class (no timing)."""
        arr = (Solid * len(solids))(*solids)
        t = Tuning()
        t.tile_w, t.extrap_blocks, t.ms = int(tile_w), int(extrap_blocks), 0.0
        st = lib().rmx_set_tuning(self.h, ctypes.byref(g), arr, len(solids),
                                  ctypes.byref(opt) if opt else None, ctypes.byref(t))
        if st != OK:
            raise RmxError(st, "rmx_set_tuning")

    def profile_read(self):
        """{phase: (total ms, launches)} for the profiled calls since the last read."""
        ms = (ctypes.c_double * N_PHASES)()
        n = (ctypes.c_int64 * N_PHASES)()
        st = lib().rmx_profile_read(self.h, ms, n)
        if st != OK:
            raise RmxError(st, "rmx_profile_read")
        return {PHASES[i]: (ms[i], n[i]) for i in range(N_PHASES) if n[i]}

    def autotune(self, g: Grid, solids: Sequence[Solid], opt: Optional[Options] = None,
                 reps: int = 5, stream=None):
        """Time the launch-shape candidates on this batch and keep the fastest for its
        shape class; returns {"tile_w", "extrap_blocks", "ms"}."""
        arr = (Solid * len(solids))(*solids)
        best = Tuning()
        st = lib().rmx_autotune(self.h, ctypes.byref(g), arr, len(solids),
                                ctypes.byref(opt) if opt else None, _stream_handle(stream),
                                int(reps), ctypes.byref(best))
        if st != OK:
            raise RmxError(st, "rmx_autotune")
        return {"tile_w": best.tile_w, "extrap_blocks": best.extrap_blocks, "ms": best.ms}

    def extrapolate_raw(self, g: Grid, arr, n: int, opt: Options, stream_handle):
        """Minimal-overhead call for timing loops: prebuilt Solid array, no stats."""
        return lib().rmx_extrapolate(self.h, ctypes.byref(g), arr, n, ctypes.byref(opt),
                                     stream_handle, None)


_HIP = None
H2D, D2H, D2D = 1, 2, 3


def _hip():
    """The HIP runtime library (for copies into and out of server-owned fields)."""
    global _HIP
    if _HIP is None:
        last = None
        for name in ("libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"):
            try:
                L = ctypes.CDLL(name)
                break
            except OSError as e:  # noqa: PERF203
                last = e
        else:
            raise RuntimeError(f"HIP runtime library not found: {last}")
        L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        L.hipMemcpy.restype = ctypes.c_int
        _HIP = L
    return _HIP


def memcpy(dst: int, src: int, nbytes: int, kind: int):
    """Synchronous hipMemcpy between raw addresses (kind: H2D, D2H or D2D)."""
    e = _hip().hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), int(nbytes), int(kind))
    if e != 0:
        raise RuntimeError(f"hipMemcpy failed with HIP error {e}")


class Server:
    """Request loop admitting extrapolation jobs by HBM budget (rmx_server_*)."""

    def __init__(self, device: int, hbm_budget_bytes: int, n_streams: int = 4):
        _torch_device_first(device)
        self.h = ctypes.c_void_p()
        st = lib().rmx_server_create(int(device), int(hbm_budget_bytes), int(n_streams),
                                     ctypes.byref(self.h))
        if st != OK:
            raise RmxError(st, "rmx_server_create")

    def close(self):
        if self.h:
            lib().rmx_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def register(self, g: Grid, templ: Sequence[Solid]) -> int:
        arr = (Solid * len(templ))(*templ)
        sid = ctypes.c_int64(-1)
        st = lib().rmx_server_register(self.h, ctypes.byref(g), arr, len(templ),
                                       ctypes.byref(sid))
        if st != OK:
            raise RmxError(st, "rmx_server_register")
        return int(sid.value)

    def field(self, sim_id: int, solid_idx: int):
        xi = ctypes.POINTER(ctypes.c_double)()
        lab = ctypes.POINTER(ctypes.c_int8)()
        st = lib().rmx_server_field(self.h, int(sim_id), int(solid_idx), ctypes.byref(xi),
                                    ctypes.byref(lab))
        if st != OK:
            raise RmxError(st, "rmx_server_field")
        return ctypes.cast(xi, ctypes.c_void_p).value, ctypes.cast(lab, ctypes.c_void_p).value

    def submit(self, sim_id: int, opt: Optional[Options] = None) -> int:
        t = ctypes.c_int64(-1)
        st = lib().rmx_server_submit(self.h, int(sim_id), ctypes.byref(opt) if opt else None,
                                     ctypes.byref(t))
        if st != OK:
            raise RmxError(st, "rmx_server_submit")
        return int(t.value)

    def wait(self, ticket: int, n_solids: int = 0):
        stats = (SolidStats * max(1, n_solids))() if n_solids else None
        lat = ctypes.c_double(0.0)
        st = lib().rmx_server_wait(self.h, int(ticket), stats, ctypes.byref(lat))
        return st, float(lat.value), ([s.as_dict() for s in stats] if n_solids else None)

    def release(self, sim_id: int):
        st = lib().rmx_server_release(self.h, int(sim_id))
        if st != OK:
            raise RmxError(st, "rmx_server_release")

    def usage(self):
        a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
        lib().rmx_server_usage(self.h, ctypes.byref(a), ctypes.byref(b))
        return int(a.value), int(b.value)

    # Copies into and out of the resident fields; only while no request of the simulation
    # is queued or running.
    def upload(self, sim_id: int, solid_idx: int, xi):
        """xi: float64 [3, ext2, ext1, ext0], a numpy array (host) or a CUDA tensor."""
        dst, _ = self.field(sim_id, solid_idx)
        if hasattr(xi, "is_cuda") and xi.is_cuda:
            import torch
            torch.cuda.synchronize()
            memcpy(dst, xi.data_ptr(), xi.numel() * 8, D2D)
        else:
            import numpy as np
            a = np.ascontiguousarray(xi, dtype=np.float64)
            memcpy(dst, a.ctypes.data, a.nbytes, H2D)

    def download(self, sim_id: int, solid_idx: int, ext):
        """(xi float64 [3, ext2, ext1, ext0], labels int8 [ext2, ext1, ext0]) on the host."""
        import numpy as np
        xp, lp = self.field(sim_id, solid_idx)
        xi = np.empty((3, ext[2], ext[1], ext[0]), dtype=np.float64)
        lab = np.empty((ext[2], ext[1], ext[0]), dtype=np.int8)
        memcpy(xi.ctypes.data, xp, xi.nbytes, D2H)
        memcpy(lab.ctypes.data, lp, lab.nbytes, D2H)
        return xi, lab
