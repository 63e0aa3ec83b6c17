"""Seeded synthetic inputs for the reference-map extrapolation workloads.

This module holds NO arithmetic of the extrapolation method itself: it only builds grids,
solid shapes and reference-map fields xi(x) from seeded random numbers (numpy
``default_rng``), in FP64, on the host.  The same arrays are handed to the GPU library and
to the CPU oracle, so both consume identical bits.

Workloads (the paper's simulation states are not available; these stand in for them):

* ``sphere32``     -- 32^3 unit cube, sphere R=0.25 at the centre, L=4; xi = c + A(x-c)
                      + 0.01 sum_m u_m sin(2 pi k_m.x + theta_m), |k|_inf <= 2.
* ``ellipsoid128`` -- 128^3, ellipsoid (0.3, 0.2, 0.15) with a uniform random rotation,
                      L=6; xi = chi^{-1}(x) for chi(X) = c + A(X-c) + 0.02 sum sin(...),
                      |k|_inf <= 4, inverted per cell by Newton's method.
* ``suspension``   -- 128x128x256 box (the paper's settling box at h = 1/128), 40
                      non-overlapping ellipsoids, semi-axes U[0.04, 0.1], each with its
                      own affine+sine field and its own box; L=4.
* ``cavity256``    -- 256^3, sphere R=0.2 at (0.6, 0.5, 0.5) (the paper's cavity sphere);
                      xi = backward flow map over t=0.5 of u = (sin pi x cos pi y,
                      -cos pi x sin pi y, 0) by RK4 (64 steps), the solution of the
                      reference-map advection equation for that velocity; L=4.
* ``serving_trace``-- 2000 requests from 100 simulations x 20 steps, Poisson arrivals at
                      200/s, grids {32, 64, 96, 128, 192}^3, 1-64 ellipsoids per
                      simulation (semi-axes U[0.05, 0.2]), L in {4, 5, 6}, FP32/FP64.
* ``step_velocity``-- the velocity a time step advects with: the cavity's cellular flow
                      U (sin pi x cos pi y, -cos pi x sin pi y) plus a uniform drift w0 along
                      z (divergence-free), sampled at cell centres and at face centres of
                      each solid's box; dt from a CFL number.
* ``periodic_box`` -- the method variants at once: a 48 x 40 x 56 grid with spacings
                      (1/48, 1/32, 1/64) (unequal), periodic along x and z (the paper's
                      periodic test box), walled along y; six rotated ellipsoids with
                      semi-axes U[0.07, 0.12], each with its own affine+sine field over
                      its unwrapped box, boxes that cross the periodic ends; L=5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SPHERE = 1
ELLIPSOID = 2


@dataclass
class Shape:
    kind: int
    centre: np.ndarray          # (3,) reference coordinates
    semi: np.ndarray            # (3,) semi-axes (sphere: [R, R, R])
    rot: np.ndarray             # (3, 3) columns are the body axes


@dataclass
class Solid:
    lo: tuple
    ext: tuple                  # (ext0, ext1, ext2) = cells along x, y, z
    shape: Shape
    n_layers: int
    xi: np.ndarray              # float64 [3, ext2, ext1, ext0]


@dataclass
class Workload:
    name: str
    grid_n: tuple               # (M, N, O) cells along x, y, z
    h: float
    origin: tuple
    solids: List[Solid] = field(default_factory=list)
    spacing: tuple = (0.0, 0.0, 0.0)   # per-axis cell size; 0 means h
    periodic: tuple = (0, 0, 0)        # 1: the grid wraps along the axis

    @property
    def deltas(self) -> tuple:
        """The cell size along x, y, z."""
        return tuple(float(d) if d > 0.0 else float(self.h) for d in self.spacing)

    @property
    def box_cells(self) -> int:
        return int(sum(int(np.prod(s.ext)) for s in self.solids))


def _unit(v):
    return v / np.linalg.norm(v)


def random_rotation(rng) -> np.ndarray:
    """Uniform rotation from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _modes(rng, n_modes, kmax):
    us, ks, ths = [], [], []
    for _ in range(n_modes):
        u = _unit(rng.standard_normal(3))
        while True:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if np.any(k != 0):
                break
        th = rng.uniform(0.0, 2.0 * math.pi)
        us.append(u)
        ks.append(k.astype(np.float64))
        ths.append(th)
    return us, ks, ths


def cell_centres(lo, ext, h, origin):
    """Coordinates (x, y, z) broadcastable to [ext2, ext1, ext0]; h: one spacing or one
    per axis.  A box past the end of a periodic axis gets its unwrapped coordinates."""
    d = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    x = origin[0] + (np.arange(lo[0], lo[0] + ext[0]) + 0.5) * d[0]
    y = origin[1] + (np.arange(lo[1], lo[1] + ext[1]) + 0.5) * d[1]
    z = origin[2] + (np.arange(lo[2], lo[2] + ext[2]) + 0.5) * d[2]
    return x[None, None, :], y[None, :, None], z[:, None, None]


def affine_sine_field(lo, ext, h, origin, c, A, amp, modes, phase_shift=0.0):
    """xi(x) = c + A (x - c) + amp * sum_m u_m sin(2 pi k_m . x + theta_m)."""
    x, y, z = cell_centres(lo, ext, h, origin)
    X = (x - c[0], y - c[1], z - c[2])
    shape = (ext[2], ext[1], ext[0])
    xi = np.empty((3,) + shape, dtype=np.float64)
    for a in range(3):
        xi[a] = c[a] + (A[a, 0] * X[0] + A[a, 1] * X[1] + A[a, 2] * X[2])
    if amp != 0.0:
        us, ks, ths = modes
        for u, k, th in zip(us, ks, ths):
            s = np.sin(2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + th + phase_shift)
            for a in range(3):
                xi[a] += amp * u[a] * s
    return xi


def sphere_shape(c, R) -> Shape:
    return Shape(SPHERE, np.asarray(c, dtype=np.float64), np.array([R, R, R], dtype=np.float64),
                 np.eye(3))


def ellipsoid_shape(c, semi, rot) -> Shape:
    return Shape(ELLIPSOID, np.asarray(c, dtype=np.float64),
                 np.asarray(semi, dtype=np.float64), np.asarray(rot, dtype=np.float64))


# ------------------------------------------------------------------------------------------
# sphere32
# ------------------------------------------------------------------------------------------
def sphere32(seed: int = 1, n: int = 32, affine: bool = False, n_layers: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    c = np.array([0.5, 0.5, 0.5])
    A = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    modes = _modes(rng, 3, 2)
    lo, ext = (0, 0, 0), (n, n, n)
    xi = affine_sine_field(lo, ext, h, (0.0, 0.0, 0.0), c, A, 0.0 if affine else 0.01, modes)
    w = Workload("sphere32" if n == 32 else f"sphere{n}", (n, n, n), h, (0.0, 0.0, 0.0))
    w.solids.append(Solid(lo, ext, sphere_shape(c, 0.25), n_layers, xi))
    w.affine = (A, c - A @ c)          # xi = A x + b on the affine variant
    return w


# ------------------------------------------------------------------------------------------
# ellipsoid128: xi = chi^{-1}(x), chi(X) = c + A(X - c) + amp sum u sin(2 pi k.X + th)
# ------------------------------------------------------------------------------------------
def _chi_and_jac(Xs, c, A, amp, modes):
    us, ks, ths = modes
    val = [c[a] + A[a, 0] * (Xs[0] - c[0]) + A[a, 1] * (Xs[1] - c[1]) + A[a, 2] * (Xs[2] - c[2])
           for a in range(3)]
    jac = [[np.full_like(Xs[0], A[a, b]) for b in range(3)] for a in range(3)]
    for u, k, th in zip(us, ks, ths):
        arg = 2.0 * math.pi * (k[0] * Xs[0] + k[1] * Xs[1] + k[2] * Xs[2]) + th
        s, co = np.sin(arg), np.cos(arg)
        for a in range(3):
            val[a] = val[a] + amp * u[a] * s
            for b in range(3):
                jac[a][b] = jac[a][b] + amp * u[a] * 2.0 * math.pi * k[b] * co
    return val, jac


def _det3(J):
    return (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
            - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
            + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))


def inverse_deformation(lo, ext, h, origin, c, A, amp, modes, tol=1e-14, max_iter=60):
    """Per-cell Newton inversion of chi; returns xi [3, ...] and min det(grad chi)."""
    x, y, z = cell_centres(lo, ext, h, origin)
    shape = (ext[2], ext[1], ext[0])
    target = [np.broadcast_to(x, shape), np.broadcast_to(y, shape), np.broadcast_to(z, shape)]
    Ainv = np.linalg.inv(A)
    Xs = [c[a] + Ainv[a, 0] * (target[0] - c[0]) + Ainv[a, 1] * (target[1] - c[1])
          + Ainv[a, 2] * (target[2] - c[2]) for a in range(3)]
    Xs = [np.array(v, dtype=np.float64) for v in Xs]
    for _ in range(max_iter):
        val, J = _chi_and_jac(Xs, c, A, amp, modes)
        r = [val[a] - target[a] for a in range(3)]
        err = max(float(np.max(np.abs(r[a]))) for a in range(3))
        if err <= tol:
            break
        det = _det3(J)
        # Cramer's rule for J dX = r
        cof = [[J[1][1] * J[2][2] - J[1][2] * J[2][1], J[0][2] * J[2][1] - J[0][1] * J[2][2],
                J[0][1] * J[1][2] - J[0][2] * J[1][1]],
               [J[1][2] * J[2][0] - J[1][0] * J[2][2], J[0][0] * J[2][2] - J[0][2] * J[2][0],
                J[0][2] * J[1][0] - J[0][0] * J[1][2]],
               [J[1][0] * J[2][1] - J[1][1] * J[2][0], J[0][1] * J[2][0] - J[0][0] * J[2][1],
                J[0][0] * J[1][1] - J[0][1] * J[1][0]]]
        for a in range(3):
            dX = (cof[a][0] * r[0] + cof[a][1] * r[1] + cof[a][2] * r[2]) / det
            Xs[a] = Xs[a] - dX
    val, J = _chi_and_jac(Xs, c, A, amp, modes)
    err = max(float(np.max(np.abs(val[a] - target[a]))) for a in range(3))
    mindet = float(np.min(_det3(J)))
    return np.stack(Xs).astype(np.float64), err, mindet


def ellipsoid128(seed: int = 2, n: int = 128, n_layers: int = 6) -> Workload:
    h = 1.0 / n
    c = np.array([0.5, 0.5, 0.5])
    attempt = 0
    while True:
        rng = np.random.default_rng(seed * 1000 + attempt)
        rot = random_rotation(rng)
        A = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
        modes = _modes(rng, 3, 4)
        lo, ext = (0, 0, 0), (n, n, n)
        xi, err, mindet = inverse_deformation(lo, ext, h, (0.0, 0.0, 0.0), c, A, 0.02, modes)
        if mindet >= 0.25 and err <= 1e-13:
            break
        attempt += 1
    w = Workload("ellipsoid128" if n == 128 else f"ellipsoid{n}", (n, n, n), h, (0.0, 0.0, 0.0))
    w.solids.append(Solid(lo, ext, ellipsoid_shape(c, (0.3, 0.2, 0.15), rot), n_layers, xi))
    w.inversion_residual = err
    w.min_det = mindet
    return w


# ------------------------------------------------------------------------------------------
# suspension: many ellipsoids, each with its own box and field
# ------------------------------------------------------------------------------------------
def place_ellipsoids(rng, n_solids, lengths, h, semi_lo, semi_hi, tries=1000):
    """Rejection sampling: bounding radius rho = 1.3 max semi-axis, pairwise clearance
    2h, wall clearance h.  Returns list of (centre, semi, rot) and the number given up."""
    placed, gave_up = [], 0
    for _ in range(n_solids):
        semi = rng.uniform(semi_lo, semi_hi, size=3)
        rot = random_rotation(rng)
        rho = 1.3 * float(np.max(semi))
        ok = False
        for _t in range(tries):
            cpos = np.array([rng.uniform(rho + h, L - rho - h) if L - 2 * (rho + h) > 0 else L / 2
                             for L in lengths])
            if all(np.linalg.norm(cpos - q[0]) > rho + q[3] + 2 * h for q in placed):
                placed.append((cpos, semi, rot, rho))
                ok = True
                break
        if not ok:
            gave_up += 1
    return [(p[0], p[1], p[2]) for p in placed], gave_up


def solid_box(cpos, amax, h, grid_n, n_layers):
    """Box centred on the solid's cell, half-width ceil(1.3 a_max / h) + L + 1, clipped."""
    hw = int(math.ceil(1.3 * amax / h)) + n_layers + 1
    lo, ext = [], []
    for a in range(3):
        ci = int(math.floor(cpos[a] / h))
        l0 = max(0, ci - hw)
        l1 = min(grid_n[a], ci + hw + 1)
        lo.append(l0)
        ext.append(l1 - l0)
    return tuple(lo), tuple(ext)


@dataclass
class SolidSpec:
    """A solid of an affine+sine workload before its field is evaluated."""
    lo: tuple
    ext: tuple
    shape: Shape
    n_layers: int
    c: np.ndarray               # centre of the affine map (the solid's centre)
    A: np.ndarray               # (3, 3)
    amp: float
    modes: tuple                # (u list, k list, theta list)


def suspension_layout(seed: int = 3, n_solids: int = 40, grid_n=(128, 128, 256),
                      h=1.0 / 128, n_layers: int = 4, semi_lo=0.04, semi_hi=0.1, amp=0.01):
    """Placement, boxes and field parameters of ``suspension`` (no field arrays)."""
    rng = np.random.default_rng(seed)
    lengths = [g * h for g in grid_n]
    placed, gave_up = place_ellipsoids(rng, n_solids, lengths, h, semi_lo, semi_hi)
    specs = []
    for cpos, semi, rot in placed:
        A = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
        modes = _modes(rng, 3, 2)
        lo, ext = solid_box(cpos, float(np.max(semi)), h, grid_n, n_layers)
        specs.append(SolidSpec(lo, ext, ellipsoid_shape(cpos, semi, rot), n_layers, cpos, A,
                               amp, modes))
    return specs, gave_up


def suspension(seed: int = 3, n_solids: int = 40, grid_n=(128, 128, 256), h=1.0 / 128,
               n_layers: int = 4, semi_lo=0.04, semi_hi=0.1, amp=0.01,
               phase_shift=0.0) -> Workload:
    specs, gave_up = suspension_layout(seed, n_solids, grid_n, h, n_layers, semi_lo, semi_hi,
                                       amp)
    w = Workload("suspension", tuple(grid_n), h, (0.0, 0.0, 0.0))
    for sp in specs:
        xi = affine_sine_field(sp.lo, sp.ext, h, (0.0, 0.0, 0.0), sp.c, sp.A, sp.amp, sp.modes,
                               phase_shift)
        w.solids.append(Solid(sp.lo, sp.ext, sp.shape, sp.n_layers, xi))
    w.gave_up = gave_up
    return w


# ------------------------------------------------------------------------------------------
# cavity256: backward flow map of a cellular shear flow (z-invariant)
# ------------------------------------------------------------------------------------------
def _u2(x, y):
    return (np.sin(math.pi * x) * np.cos(math.pi * y), -np.cos(math.pi * x) * np.sin(math.pi * y))


def backward_flow_map_xy(xs, ys, t=0.5, steps=64):
    """X such that the flow of u carries X to (x, y) in time t: integrate dX/ds = -u(X)."""
    X, Y = np.meshgrid(xs, ys, indexing="xy")   # [ny, nx]
    X = X.astype(np.float64).copy()
    Y = Y.astype(np.float64).copy()
    dt = t / steps
    for _ in range(steps):
        k1 = _u2(X, Y)
        k2 = _u2(X - 0.5 * dt * k1[0], Y - 0.5 * dt * k1[1])
        k3 = _u2(X - 0.5 * dt * k2[0], Y - 0.5 * dt * k2[1])
        k4 = _u2(X - dt * k3[0], Y - dt * k3[1])
        X = X - dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        Y = Y - dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    return X, Y


def cavity256(seed: int = 4, n: int = 256, n_layers: int = 4, t: float = 0.5) -> Workload:
    # The flow is deterministic; the seed is kept for the naming convention only.
    del seed
    h = 1.0 / n
    lo, ext = (0, 0, 0), (n, n, n)
    x, y, z = cell_centres(lo, ext, h, (0.0, 0.0, 0.0))
    X, Y = backward_flow_map_xy(x.reshape(-1), y.reshape(-1), t=t)
    xi = np.empty((3, n, n, n), dtype=np.float64)
    xi[0] = X[None, :, :]
    xi[1] = Y[None, :, :]
    xi[2] = np.broadcast_to(z, (n, n, n))
    w = Workload("cavity256" if n == 256 else f"cavity{n}", (n, n, n), h, (0.0, 0.0, 0.0))
    w.solids.append(Solid(lo, ext, sphere_shape((0.6, 0.5, 0.5), 0.2), n_layers, xi))
    return w


# ------------------------------------------------------------------------------------------
# serving trace
# ------------------------------------------------------------------------------------------
@dataclass
class SimSpec:
    sim_id: int
    n: int
    n_solids_requested: int
    n_layers: int
    precision: int              # 0 = FP64, 1 = FP32-accumulate
    seed: int


@dataclass
class Request:
    arrival_s: float
    sim_id: int
    step: int


def serving_trace(seed: int = 5, n_sims: int = 100, steps: int = 20, rate: float = 200.0,
                  grid_sizes=(32, 64, 96, 128, 192)):
    rng = np.random.default_rng(seed)
    sims = []
    for s in range(n_sims):
        n = int(rng.choice(grid_sizes))
        ns = int(rng.integers(1, 65))
        L = int(rng.integers(4, 7))
        prec = int(rng.integers(0, 2))
        sims.append(SimSpec(s, n, ns, L, prec, int(rng.integers(0, 2**31 - 1))))
    order = []
    pending = [0] * n_sims
    total = n_sims * steps
    while len(order) < total:
        s = int(rng.integers(0, n_sims))
        if pending[s] < steps:
            order.append((s, pending[s]))
            pending[s] += 1
    gaps = rng.exponential(1.0 / rate, size=total)
    t = np.cumsum(gaps)
    reqs = [Request(float(t[i]), order[i][0], order[i][1]) for i in range(total)]
    return sims, reqs


def sim_layout(spec: SimSpec, semi_lo=0.05, semi_hi=0.2):
    """The solids of one served simulation (placed as in ``suspension``; the unit cube at
    n^3), without their fields."""
    return suspension_layout(seed=spec.seed, n_solids=spec.n_solids_requested,
                             grid_n=(spec.n, spec.n, spec.n), h=1.0 / spec.n,
                             n_layers=spec.n_layers, semi_lo=semi_lo, semi_hi=semi_hi)


def sim_workload(spec: SimSpec, semi_lo=0.05, semi_hi=0.2) -> Workload:
    """The resident fields of one served simulation (ellipsoids placed as in
    ``suspension``; the unit cube at n^3)."""
    w = suspension(seed=spec.seed, n_solids=spec.n_solids_requested,
                   grid_n=(spec.n, spec.n, spec.n), h=1.0 / spec.n, n_layers=spec.n_layers,
                   semi_lo=semi_lo, semi_hi=semi_hi)
    w.name = f"sim{spec.sim_id}"
    return w


def tiny_field_from_mask(mask: np.ndarray, inside_value=(0.0, 0.0, 0.0),
                         outside=np.nan) -> np.ndarray:
    """A field whose interior (for a sphere of radius 1 at the origin) is exactly `mask`
    ([ext2, ext1, ext0] bool): inside cells get `inside_value`, the rest `outside`."""
    xi = np.empty((3,) + mask.shape, dtype=np.float64)
    for a in range(3):
        xi[a] = np.where(mask, inside_value[a], outside)
    return xi


WORKLOADS = {
    "sphere32": sphere32,
    "ellipsoid128": ellipsoid128,
    "suspension": suspension,
    "cavity256": cavity256,
}


# ------------------------------------------------------------------------------------------
# time step: the advecting velocity
# ------------------------------------------------------------------------------------------
def flow_velocity(x, y, z, U=1.0, w0=0.3):
    """(sin pi x cos pi y, -cos pi x sin pi y) U, plus w0 along z."""
    ux = U * np.sin(math.pi * x) * np.cos(math.pi * y)
    uy = -U * np.cos(math.pi * x) * np.sin(math.pi * y)
    uz = np.full(np.broadcast(x, y, z).shape, float(w0))
    return np.stack(np.broadcast_arrays(ux, uy, uz)).astype(np.float64)


@dataclass
class StepVelocity:
    u: np.ndarray          # [3, e2, e1, e0] at cell centres
    uf: tuple              # x-faces [e2, e1, e0+1], y-faces [e2, e1+1, e0], z-faces [e2+1, e1, e0]


def step_velocity(w: "Workload", U=1.0, w0=0.3):
    """Per solid of `w`: the velocity at its cell centres and its face centres."""
    out = []
    (hx, hy, hz), o = w.deltas, w.origin
    for s in w.solids:
        lo, e = s.lo, s.ext
        x, y, z = cell_centres(lo, e, (hx, hy, hz), o)
        u = flow_velocity(x, y, z, U, w0)
        k, j, i = np.meshgrid(np.arange(e[2]), np.arange(e[1]), np.arange(e[0] + 1),
                              indexing="ij")
        ufx = flow_velocity(o[0] + (lo[0] + i) * hx, o[1] + (lo[1] + j + 0.5) * hy,
                            o[2] + (lo[2] + k + 0.5) * hz, U, w0)[0]
        k, j, i = np.meshgrid(np.arange(e[2]), np.arange(e[1] + 1), np.arange(e[0]),
                              indexing="ij")
        ufy = flow_velocity(o[0] + (lo[0] + i + 0.5) * hx, o[1] + (lo[1] + j) * hy,
                            o[2] + (lo[2] + k + 0.5) * hz, U, w0)[1]
        k, j, i = np.meshgrid(np.arange(e[2] + 1), np.arange(e[1]), np.arange(e[0]),
                              indexing="ij")
        ufz = flow_velocity(o[0] + (lo[0] + i + 0.5) * hx, o[1] + (lo[1] + j + 0.5) * hy,
                            o[2] + (lo[2] + k) * hz, U, w0)[2]
        out.append(StepVelocity(np.ascontiguousarray(u), (np.ascontiguousarray(ufx),
                                                          np.ascontiguousarray(ufy),
                                                          np.ascontiguousarray(ufz))))
    return out


def step_dt(w: "Workload", cfl=0.4, U=1.0, w0=0.3) -> float:
    """dt with max |u_a| dt / Delta_a <= cfl on every axis."""
    return cfl * min(w.deltas) / max(abs(U), abs(w0))


# ------------------------------------------------------------------------------------------
# periodic_box: unequal spacings, periodic axes, boxes across the periodic ends
# ------------------------------------------------------------------------------------------
def periodic_box(seed: int = 6, grid_n=(48, 40, 56), spacing=(1.0 / 48, 1.0 / 32, 1.0 / 64),
                 periodic=(1, 0, 1), n_solids: int = 6, n_layers: int = 5,
                 semi_lo: float = 0.07, semi_hi: float = 0.12) -> Workload:
    """Ellipsoids placed at random (overlaps allowed: every solid is independent); along a
    periodic axis the centre is anywhere and the box, lo taken mod n, may run past the
    grid's end with the field on its unwrapped coordinates; along a walled axis the box
    stays inside the grid."""
    rng = np.random.default_rng(seed)
    d = np.asarray(spacing, dtype=np.float64)
    n = np.asarray(grid_n)
    length = n * d
    w = Workload("periodic_box", tuple(int(v) for v in grid_n), float(d.min()),
                 (0.0, 0.0, 0.0), spacing=tuple(float(v) for v in d),
                 periodic=tuple(int(v) for v in periodic))
    for _ in range(n_solids):
        semi = rng.uniform(semi_lo, semi_hi, 3)
        rot = random_rotation(rng)
        # cells from the centre to the box face: the semi-axis bound, the band and a margin
        half = np.ceil(semi.max() * 1.05 / d).astype(int) + n_layers + 2
        ext = 2 * half + 1
        c = np.empty(3)
        lo = np.empty(3, dtype=int)
        for a in range(3):
            if periodic[a]:
                c[a] = rng.uniform(0.0, length[a])
            else:
                c[a] = rng.uniform((half[a] + 1) * d[a], length[a] - (half[a] + 1) * d[a])
            lo[a] = int(math.floor(c[a] / d[a])) - half[a]
        A = np.eye(3) + 0.04 * rng.standard_normal((3, 3))
        modes = _modes(rng, 3, 2)
        xi = affine_sine_field(tuple(int(v) for v in lo), tuple(int(v) for v in ext), d,
                               (0.0, 0.0, 0.0), c, A, 0.006, modes)
        lo_grid = tuple(int(lo[a] % n[a]) if periodic[a] else int(lo[a]) for a in range(3))
        w.solids.append(Solid(lo_grid, tuple(int(v) for v in ext),
                              ellipsoid_shape(c, semi, rot), n_layers, xi))
    return w
