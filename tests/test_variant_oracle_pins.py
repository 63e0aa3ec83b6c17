"""Pins of the oracle's method variants, anisotropic spacing and periodic domains, against
facts fixed outside it.

Spacing (SI "Variable arrangement": cells of Delta x, Delta y, Delta z):
  * equal spacings of any size change nothing (eq. (weight) is a cosine, scale-free);
  * relabelling the grid axes, spacings with them, relabels the result;
  * on a mirror-symmetric field the normal at a cell on a symmetry axis is that axis
    exactly, so eq. (weight) has a closed form in physical offsets there; the fit is
    then a library least-squares solve;
  * uniform transport of affine and bilinear fields is exact for any spacings (the
    advection equation's solution is xi0(x - u t));
  * the face stress of an affine map xi = A x + b is tau(A^{-1}) for any spacings
    (centred differences are exact on affine data).
Periodic domains (SI "Test cases": the pre-stretched sphere in a periodic box):
  * a box may run past the end of a periodic axis, and the extrapolation of its
    unwrapped map is that of the same box inside a walled grid;
  * no box face on a periodic axis is a wall, so a band reaching it is truncated;
  * moving every box by s cells along a periodic axis moves the blur fields by s cells
    (np.roll), and with no box at the grid's ends the periodic grid gives what the
    walled grid gives;
  * the difference stencil is taken in the box: a box spanning the whole periodic axis
    holds a jump of the unwrapped map between its ends, and no face takes it."""
import math

import numpy as np
import pytest

import oracle

EPS = 0.1


# ---- helpers -------------------------------------------------------------------------

def grid_coords(ext, spacing, lo=(0, 0, 0), origin=(0.0, 0.0, 0.0)):
    """Physical cell centres [3, e2, e1, e0] of the box at lo."""
    k, j, i = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]),
                          indexing="ij")
    return np.stack([origin[0] + (lo[0] + i + 0.5) * spacing[0],
                     origin[1] + (lo[1] + j + 0.5) * spacing[1],
                     origin[2] + (lo[2] + k + 0.5) * spacing[2]])


def deformed_ellipsoid_case(ext=(26, 24, 28), spacing=(0.04, 0.05, 0.035)):
    """A smooth non-affine map and an ellipsoid whose band fits the box."""
    X = grid_coords(ext, spacing)
    c = X.reshape(3, -1).mean(axis=1)
    d = X - c[:, None, None, None]
    xi = X + 0.06 * np.stack([np.sin(3.0 * d[1]) * d[2], np.cos(2.0 * d[2]) * d[0] * 0.8,
                              np.sin(2.5 * d[0]) * d[1]])
    t = 0.5
    rot = np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0],
                    [0.0, 0.0, 1.0]])
    shape = oracle.make_shape(2, c, (0.22, 0.28, 0.18), rot)
    return xi, shape


def run(ext, xi, shape, spacing, L=5, grid=None, lo=(0, 0, 0), periodic=(0, 0, 0)):
    grid = ext if grid is None else grid
    p = oracle.make_problem(grid, lo, ext, shape, L, periodic=periodic, spacing=spacing)
    return oracle.extrapolate(p, xi)


def band_close(a, b, mask, tol=1e-12):
    return np.max(np.abs(a[:, mask] - b[:, mask])) < tol


# ---- spacing: the extrapolation --------------------------------------------------------

def test_equal_spacings_of_any_size_change_nothing():
    xi, shape = deformed_ellipsoid_case()
    ext = xi.shape[1:][::-1]
    ref = run(ext, xi, shape, (1.0, 1.0, 1.0))
    assert ref[0] == oracle.OK
    band = (ref[2] >= 1)
    assert band.sum() > 1000
    for s in (0.37, 7.5):
        got = run(ext, xi, shape, (s, s, s))
        assert got[0] == oracle.OK
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
        assert band_close(got[1], ref[1], band, 1e-13)


def test_unequal_spacings_change_the_band():
    """The spacing reaches the result (else every pin below would hold vacuously)."""
    xi, shape = deformed_ellipsoid_case()
    ext = xi.shape[1:][::-1]
    iso = run(ext, xi, shape, (1.0, 1.0, 1.0))
    ani = run(ext, xi, shape, (1.0, 1.9, 0.6))
    assert np.array_equal(iso[2], ani[2]) and np.array_equal(iso[3], ani[3])
    near = (iso[2] >= 1) & (iso[2] <= 2)
    assert np.max(np.abs(iso[1][:, near] - ani[1][:, near])) > 1e-6


@pytest.mark.parametrize("perm", [(1, 2, 0), (2, 0, 1), (1, 0, 2)])
def test_relabelling_the_axes_relabels_the_result(perm):
    """New axis a is old axis perm[a]; the spacings follow their axes.  Values of xi are
    reference coordinates and do not move."""
    xi, shape = deformed_ellipsoid_case()
    sp = (0.04, 0.065, 0.03)
    ext = xi.shape[1:][::-1]
    ref = run(ext, xi, shape, sp)
    assert ref[0] == oracle.OK
    # numpy axes are (z, y, x) = grid axes (2, 1, 0); new grid axis a holds old perm[a]
    ax = [2 - perm[2 - q] for q in range(3)]          # old numpy axis of new numpy axis q
    xi2 = np.ascontiguousarray(np.transpose(xi, [0] + [1 + a for a in ax]))
    ext2 = tuple(ext[perm[a]] for a in range(3))
    sp2 = tuple(sp[perm[a]] for a in range(3))
    got = run(ext2, xi2, shape, sp2)
    assert got[0] == oracle.OK
    lab = np.transpose(ref[2], ax)
    dec = np.transpose(ref[3], ax)
    xo = np.transpose(ref[1], [0] + [1 + a for a in ax])
    assert np.array_equal(got[2], lab) and np.array_equal(got[3], dec)
    assert band_close(got[1], xo, lab >= 1, 1e-12)
    assert np.array_equal(got[4], ref[4])


@pytest.mark.parametrize("sp", [(1.0, 1.3, 0.8), (0.5, 0.5, 1.7)])
def test_normal_factor_on_a_symmetry_axis(sp):
    """xi - c = (x - c)(1 + kappa |x - c|^2) around a sphere centred on a cell: phi0(xi)
    is mirror-symmetric in every axis through that cell, bit for bit, so at a cell on
    the z axis the centred gradient is exactly (0, 0, g_z) and the physical normal is
    e_z.  There eq. (weight) reads w = max(0, -dz Delta_z / |delta . Delta|) 2^-|delta|_1
    with delta the data offset in cells; the extrapolated value is the intercept of the
    weighted least-squares affine fit, here by numpy's lstsq."""
    n, ic, kappa, R = 17, 8, 2.0, 0.25
    h = 0.05
    dsp = np.array(sp) * h
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.stack([(i - ic) * dsp[0], (j - ic) * dsp[1], (k - ic) * dsp[2]])
    r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    xi = d * (1.0 + kappa * r2)
    shape = oracle.make_shape(1, (0.0, 0.0, 0.0), (R,))
    st, xo, lab, dec, _ = run((n, n, n), xi, shape, tuple(dsp), L=3)
    assert st == oracle.OK
    checked = 0
    for side in (1, -1):
        for kk in range(n):
            le = int(lab[kk, ic, ic])
            if le not in (1, 2) or (kk - ic) * side <= 0:
                continue
            g = oracle.normal(oracle.make_problem((n, n, n), (0, 0, 0), (n, n, n), shape, 3,
                                                  spacing=tuple(dsp)), xi, ic, ic, kk)
            assert g[0] == 0.0 and g[1] == 0.0 and g[2] * side > 0.0
            assert dec[kk, ic, ic] == 2            # fitted at r_s = 2 with the normal
            rows, vals, rows_iso = [], [], []
            for dz in range(-2, 3):
                for dy in range(-2, 3):
                    for dx in range(-2, 3):
                        z, y, x = kk + dz, ic + dy, ic + dx
                        if not (0 <= x < n and 0 <= y < n and 0 <= z < n):
                            continue
                        if not (0 <= lab[z, y, x] < le):
                            continue
                        if dz * side >= 0:
                            continue               # x' . e_z <= 0: weight 0
                        plen = math.sqrt((dx * dsp[0]) ** 2 + (dy * dsp[1]) ** 2 +
                                         (dz * dsp[2]) ** 2)
                        base = 2.0 ** -(abs(dx) + abs(dy) + abs(dz))
                        w = (-dz * side * dsp[2] / plen) * base
                        w_iso = (-dz * side / math.sqrt(dx * dx + dy * dy + dz * dz)) * base
                        rows.append((math.sqrt(w), (1.0, dx, dy, dz)))
                        rows_iso.append((math.sqrt(w_iso), (1.0, dx, dy, dz)))
                        vals.append(xo[:, z, y, x])
            A = np.array([s * np.array(r) for s, r in rows])
            B = np.array([s * v for (s, _), v in zip(rows, vals)])
            want = np.linalg.lstsq(A, B, rcond=None)[0][0]
            assert np.max(np.abs(xo[:, kk, ic, ic] - want)) < 1e-12
            # the cell-unit cosine (spacing ignored) gives another value
            Ai = np.array([s * np.array(r) for s, r in rows_iso])
            Bi = np.array([s * v for (s, _), v in zip(rows_iso, vals)])
            wrong = np.linalg.lstsq(Ai, Bi, rcond=None)[0][0]
            if sp[0] != sp[2] or sp[1] != sp[2]:
                assert np.max(np.abs(wrong - want)) > 1e-9
            checked += 1
    assert checked >= 3


@pytest.mark.parametrize("sp", [(0.05, 0.025, 0.08), (0.07, 0.04, 0.03)])
def test_normal_factor_against_the_exact_normal(sp):
    """The normal comes from a field of its own (xi_normal = x) and a sphere so large
    (R = 1000) that centred differences of phi0 give its physical gradient
    (x - c) / |x - c| to about 1e-11: a tilted plane, every component non-zero.  The
    data field is nonlinear.  On every layer-1 and layer-2 cell off the walls fitted at
    r_s with the normal, the value is the weighted least-squares intercept with eq. (weight) written
    in physical offsets x' = -(dx Delta_x, dy Delta_y, dz Delta_z) and that normal."""
    n, R = 18, 1000.0
    ext = (n, n, n)
    X = grid_coords(ext, sp)
    p0 = X[:, n // 2, n // 2, n // 2]
    nh = np.array([0.45, -0.3, 0.84])
    nh /= np.linalg.norm(nh)
    c = p0 - R * nh
    d = X - p0[:, None, None, None]
    xi = X + 0.5 * np.stack([np.sin(9.0 * d[1]) * d[2], np.cos(7.0 * d[2]) * d[0],
                             np.sin(8.0 * d[0]) * d[1] + d[0] * d[0]])
    shape = oracle.make_shape(1, c, (R,))
    p = oracle.make_problem(ext, (0, 0, 0), ext, shape, 3, spacing=sp)
    st, xo, lab, dec, _ = oracle.extrapolate(p, xi, xi_normal=X)
    assert st == oracle.OK
    dsp = np.asarray(sp)
    checked = worst = sens = 0.0
    inner = np.zeros_like(lab, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True          # centred differences there (one-sided at walls)
    for (kk, jj, ii) in zip(*np.nonzero((lab >= 1) & (lab <= 2) & (dec == 2) & inner)):
        le = int(lab[kk, jj, ii])
        xe = X[:, kk, jj, ii]
        nrm = (xe - c) / np.linalg.norm(xe - c)     # the exact physical normal
        rows, rows_bad, vals = [], [], []
        for dz in range(-2, 3):
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    z, y, x = kk + dz, jj + dy, ii + dx
                    if not (0 <= x < n and 0 <= y < n and 0 <= z < n):
                        continue
                    if not (0 <= lab[z, y, x] < le):
                        continue
                    xp = -np.array([dx, dy, dz]) * dsp
                    cosv = float(xp @ nrm) / float(np.linalg.norm(xp))
                    if cosv <= 0.0:
                        continue
                    base = 2.0 ** -(abs(dx) + abs(dy) + abs(dz))
                    # a plausible mistake: the spacing multiplies the gradient
                    gb = nrm * dsp * dsp
                    cb = max(0.0, float(xp @ gb) / float(np.linalg.norm(xp) *
                                                          np.linalg.norm(gb)))
                    rows.append(math.sqrt(cosv * base) * np.array([1.0, dx, dy, dz]))
                    rows_bad.append(math.sqrt(cb * base) * np.array([1.0, dx, dy, dz]))
                    vals.append(xo[:, z, y, x])
        A, Ab, V = np.array(rows), np.array(rows_bad), np.array(vals)
        want = np.linalg.lstsq(A, np.sqrt((A[:, 0] ** 2))[:, None] * V, rcond=None)[0][0]
        bad = np.linalg.lstsq(Ab, np.sqrt((Ab[:, 0] ** 2))[:, None] * V, rcond=None)[0][0]
        worst = max(worst, float(np.max(np.abs(xo[:, kk, jj, ii] - want))))
        sens = max(sens, float(np.max(np.abs(bad - want))))
        checked += 1
    assert checked > 200
    assert worst < 1e-9, worst
    assert sens > 1e-5, sens


# ---- spacing: the time step ------------------------------------------------------------

def uniform_velocity(ext, vel):
    e0, e1, e2 = ext
    u = np.empty((3, e2, e1, e0))
    for a in range(3):
        u[a] = vel[a]
    uf = (np.full((e2, e1, e0 + 1), float(vel[0])), np.full((e2, e1 + 1, e0), float(vel[1])),
          np.full((e2 + 1, e1, e0), float(vel[2])))
    return u, uf


def predicted(ext, L=6):
    e0, e1, e2 = ext
    k, j, i = np.meshgrid(np.arange(e2), np.arange(e1), np.arange(e0), indexing="ij")
    return (i >= 3) & (i <= e0 - 4) & (j >= 3) & (j <= e1 - 4) & (k >= 3) & (k <= e2 - 4)


ANISO = [(0.1, 0.05, 0.16), (0.2, 0.09, 0.07)]


@pytest.mark.parametrize("sp", ANISO)
@pytest.mark.parametrize("vel", [(0.7, 0.3, -0.4), (-0.6, -0.2, 0.5)])
def test_affine_transport_is_exact_for_any_spacing(sp, vel):
    ext, dt = (16, 14, 15), 0.03
    X = grid_coords(ext, sp)
    A = np.array([[1.0, 0.2, -0.1], [0.05, 0.9, 0.3], [-0.2, 0.1, 1.1]])
    b0 = np.array([0.3, -0.2, 0.1])[:, None, None, None]
    xi = np.einsum("ab,bkji->akji", A, X) + b0
    labels = np.zeros(ext[::-1], dtype=np.int8)
    u, uf = uniform_velocity(ext, vel)
    out = np.full_like(xi, 7.25)
    oracle.predict(ext, 6, xi, labels, u, uf, dt, sp, out)
    P = predicted(ext)
    exact = np.einsum("ab,bkji->akji", A, X - dt * np.array(vel)[:, None, None, None]) + b0
    assert np.max(np.abs(out[:, P] - exact[:, P])) < 1e-13


@pytest.mark.parametrize("sp", ANISO)
@pytest.mark.parametrize("axes", [(0, 1), (0, 2), (1, 2)])
def test_bilinear_transport_is_exact_for_any_spacing(sp, axes):
    """The cross term a b dt^2 comes from the tangential terms along the other axis,
    each with its own dt / Delta_t."""
    ext, dt = (14, 13, 12), 0.03
    X = grid_coords(ext, sp)
    p, q = axes
    vel = [0.0, 0.0, 0.0]
    vel[p], vel[q] = 0.8, -0.55
    xi = np.stack([X[p] * X[q], X[1] + 0.5 * X[p], X[2] - 0.25 * X[q] * X[p]])
    labels = np.zeros(ext[::-1], dtype=np.int8)
    u, uf = uniform_velocity(ext, vel)
    out = np.full_like(xi, 7.25)
    oracle.predict(ext, 6, xi, labels, u, uf, dt, sp, out)
    P = predicted(ext)
    Xs = [X[a] - dt * vel[a] for a in range(3)]
    exact = np.stack([Xs[p] * Xs[q], Xs[1] + 0.5 * Xs[p], Xs[2] - 0.25 * Xs[q] * Xs[p]])
    assert np.max(np.abs(out[:, P] - exact[:, P])) < 1e-12


def smooth_xi(x, y, z):
    # monotone along every axis in [0, 1]^3 (no limiter active), nonlinear in every axis
    return np.stack([np.exp(0.7 * x + 0.2 * y) + 0.3 * z, np.exp(0.5 * y - 0.2 * z) + x,
                     z + 0.3 * np.exp(x + 0.4 * y - 0.3 * z)])


def swirl(x, y, z):
    return np.stack([0.6 + 0.2 * y + 0.1 * z, -(0.5 + 0.2 * x - 0.1 * z), 0.3 + 0.15 * x * y])


def sampled_velocity(ext, sp):
    """Cell-centred and face-normal samples of the swirl."""
    e0, e1, e2 = ext
    uc = swirl(*grid_coords(ext, sp))
    faces = []
    for a in range(3):
        shp = [e2, e1, e0]
        shp[2 - a] += 1
        k, j, i = np.meshgrid(*[np.arange(m) for m in shp], indexing="ij")
        pos = [(i + 0.5) * sp[0], (j + 0.5) * sp[1], (k + 0.5) * sp[2]]
        pos[a] = [i, j, k][a] * sp[a]
        faces.append(swirl(*pos)[a])
    return uc, tuple(faces)


def feet(x, y, z, dt, steps=64):
    """Foot of the characteristic of the swirl through (x, y, z) over dt (RK4)."""
    P = np.stack([x, y, z]).astype(np.float64)
    ds = -dt / steps
    for _ in range(steps):
        k1 = swirl(*P)
        k2 = swirl(*(P + 0.5 * ds * k1))
        k3 = swirl(*(P + 0.5 * ds * k2))
        k4 = swirl(*(P + ds * k3))
        P = P + ds / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return P


def test_one_step_error_is_third_order_for_unequal_spacings():
    """Spacings in the ratio 1 : 0.6 : 1.4, all halved twice with dt: the one-step error
    against the exact transport falls toward a factor 8."""
    errs = []
    for n in (16, 32, 64):
        sp = (1.0 / n, 0.6 / n, 1.4 / n)
        ext = tuple(int(round(1.0 / v)) for v in sp)
        dt = 0.4 * min(sp)
        X = grid_coords(ext, sp)
        xi = smooth_xi(*X)
        labels = np.zeros(ext[::-1], dtype=np.int8)
        uc, uf = sampled_velocity(ext, sp)
        out = np.full_like(xi, 7.25)
        oracle.predict(ext, 6, xi, labels, uc, uf, dt, sp, out)
        P = predicted(ext)
        exact = smooth_xi(*feet(*X, dt))
        errs.append(np.max(np.abs(out[:, P] - exact[:, P])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 5.0 and r2 > 6.3, (errs, r1, r2)


@pytest.mark.parametrize("perm", [(1, 2, 0), (2, 0, 1), (0, 2, 1)])
def test_step_relabelling_the_axes_relabels_the_result(perm):
    """New grid axis a is old axis perm[a]: fields are transposed, velocity components
    and face arrays follow their axes, the spacings too; xi's values do not move."""
    sp = (0.05, 0.03, 0.07)
    ext = (16, 19, 14)
    X = grid_coords(ext, sp)
    xi = smooth_xi(*X)
    labels = np.zeros(ext[::-1], dtype=np.int8)
    uc, uf = sampled_velocity(ext, sp)
    dt = 0.4 * min(sp)
    ref = np.full_like(xi, 7.25)
    oracle.predict(ext, 6, xi, labels, uc, uf, dt, sp, ref)
    ax = [2 - perm[2 - q] for q in range(3)]
    T3 = lambda f: np.ascontiguousarray(np.transpose(f, ax))
    T4 = lambda f: np.ascontiguousarray(np.transpose(f, [0] + [1 + a for a in ax]))
    ext2 = tuple(ext[perm[a]] for a in range(3))
    sp2 = tuple(sp[perm[a]] for a in range(3))
    uc2 = np.ascontiguousarray(T4(uc)[list(perm)])
    uf2 = tuple(T3(uf[perm[a]]) for a in range(3))
    got = np.full((3,) + ext2[::-1], 7.25)
    oracle.predict(ext2, 6, T4(xi), T3(labels), uc2, uf2, dt, sp2, got)
    want = T4(ref)
    P = predicted(ext2)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.max(np.abs(got[:, P] - want[:, P])) < 1e-13


# ---- spacing: the face stress ----------------------------------------------------------

def expected_tau(F, G):
    B = F @ F.T
    t = G * (B - np.trace(B) / 3.0 * np.eye(3))
    return np.array([t[0, 0], t[1, 1], t[2, 2], t[0, 1], t[0, 2], t[1, 2]])


def tau_init(grid, periodic=(0, 0, 0), fill=-7.0):
    out = []
    for a in range(3):
        n = [grid[2], grid[1], grid[0]]
        if not periodic[a]:
            n[2 - a] += 1
        out.append(np.full([6] + n, fill))
    return out


@pytest.mark.parametrize("sp", [(0.05, 0.03, 0.08), (0.02, 0.07, 0.045)])
def test_affine_stress_for_any_spacing(sp):
    G = 1.7
    A = np.array([[1.1, 0.2, -0.15], [0.05, 0.9, 0.3], [-0.2, 0.1, 1.05]])
    lo, ext, grid = (3, 2, 4), (10, 11, 9), (18, 17, 16)
    X = grid_coords(ext, sp, lo)
    xi = np.einsum("ab,bkji->akji", A, X) + np.array([0.1, -0.2, 0.3])[:, None, None, None]
    shape = oracle.make_shape(1, (0.0, 0.0, 0.0), (1e6,))
    sol = (lo, ext, shape, 6, xi, np.zeros(ext[::-1], np.int8))
    tau = oracle.solid_stress(grid, [sol], EPS, sp, [G], tau_init(grid))
    want = expected_tau(np.linalg.inv(A), G)
    for a in range(3):
        sl = []
        for b in (2, 1, 0):
            sl.append(slice(lo[b] + 1, lo[b] + ext[b]) if b == a else
                      slice(lo[b] + 1, lo[b] + ext[b] - 1))
        got = tau[a][(slice(None),) + tuple(sl)]
        assert got.size > 0
        assert np.max(np.abs(got - want[:, None, None, None])) < 1e-11
    # one isotropic spacing in place of the three gives another stress
    wrong = oracle.solid_stress(grid, [sol], EPS, sp[0], [G], tau_init(grid))
    assert np.max(np.abs(wrong[0] - tau[0])) > 1e-3


# ---- periodic: the extrapolation -------------------------------------------------------

def test_box_past_the_end_of_a_periodic_axis():
    xi, shape = deformed_ellipsoid_case()
    ext = xi.shape[1:][::-1]
    sp = (0.04, 0.05, 0.035)
    walled = run(ext, xi, shape, sp, grid=(40, 40, 40), lo=(5, 6, 4))
    crossing = run(ext, xi, shape, sp, grid=(30, 40, 32), lo=(20, 6, 17),
                   periodic=(1, 0, 1))
    assert walled[0] == oracle.OK and crossing[0] == oracle.OK
    for a, b in zip(walled[1:], crossing[1:]):
        assert np.array_equal(a, b, equal_nan=True)


def test_box_checks_on_a_periodic_axis():
    xi, shape = deformed_ellipsoid_case()
    ext = xi.shape[1:][::-1]
    sp = (1.0, 1.0, 1.0)
    # the box may not cover a cell twice, and starts inside the grid
    assert run(ext, xi, shape, sp, grid=(ext[0] - 1, 40, 40), periodic=(1, 0, 0))[0] == \
        oracle.E_BOX
    assert run(ext, xi, shape, sp, grid=(40, 40, 40), lo=(40, 0, 0),
               periodic=(1, 0, 0))[0] == oracle.E_BOX
    assert run(ext, xi, shape, sp, grid=(40, 40, 40), lo=(-1, 0, 0),
               periodic=(1, 0, 0))[0] == oracle.E_BOX
    # a box spanning the whole periodic axis is allowed
    assert run(ext, xi, shape, sp, grid=(ext[0], 40, 40), periodic=(1, 0, 0))[0] == oracle.OK


def test_a_periodic_axis_has_no_walls():
    """A sphere whose band reaches the box's low x face: at a wall the growth stops
    there (the paper's physical boundary); on a periodic axis the box face is no
    boundary, so the band would leave the box: truncated.  The labels agree."""
    n = 24
    X = grid_coords((n, n, n), (1.0, 1.0, 1.0))
    shape = oracle.make_shape(1, (4.0, 12.0, 12.0), (5.0,))
    pw = oracle.make_problem((n, n, n), (0, 0, 0), (n, n, n), shape, 4)
    pp = oracle.make_problem((n, n, n), (0, 0, 0), (n, n, n), shape, 4, periodic=(1, 0, 0))
    pz = oracle.make_problem((n, n, n), (0, 0, 0), (n, n, n), shape, 4, periodic=(0, 0, 1))
    nw, lw, tw = oracle.label(pw, X)
    npr, lp, tp = oracle.label(pp, X)
    nz, lz, tz = oracle.label(pz, X)
    assert nw == npr == nz > 0
    assert not tw and tp and not tz       # along z the interior is L cells clear
    assert np.array_equal(lw, lp) and np.array_equal(lw, lz)
    assert (lw[:, :, 0] >= 0).any()       # the band does reach x = 0
    assert run((n, n, n), X, shape, (1.0, 1.0, 1.0), L=4, periodic=(1, 0, 0))[0] == \
        oracle.E_TRUNCATED


# ---- periodic: the blur consumers ------------------------------------------------------

def sphere_solid(grid, lo, ext, c, R, sp, L=6, periodic=(0, 0, 0), warp=0.0):
    X = grid_coords(ext, sp, lo)
    xi = X + warp * np.stack([np.sin(7.0 * X[1]), np.cos(5.0 * X[2]), np.sin(6.0 * X[0])])
    shape = oracle.make_shape(1, c, (R,))
    prob = oracle.make_problem(grid, lo, ext, shape, L, periodic=periodic, spacing=sp)
    n, labels, tr = oracle.label(prob, xi)
    assert n > 0 and not tr
    return [lo, ext, shape, L, xi, labels]


BLUR_EPS = 0.05
BLUR_SP = (0.03, 0.025, 0.02)


def blur_all(grid, solids, sp, periodic, G=(1.0, 2.0, 0.5)):
    H, phis = oracle.blur(grid, solids, BLUR_EPS, np.full(grid[::-1], -3.0),
                          [np.full(s[4].shape[1:], -5.0) for s in solids], periodic=periodic)
    tau = oracle.solid_stress(grid, solids, BLUR_EPS, sp, list(G[:len(solids)]),
                              tau_init(grid, periodic), periodic=periodic)
    return H, phis, tau


def two_solids(grid, sp, periodic):
    """Two spheres of radius 0.07 centred in boxes of 16 x 17 x 18 cells (L = 4), away
    from the grid's ends; the boxes and the bands overlap."""
    out = []
    for lo, warp in (((3, 2, 4), 0.01), ((12, 6, 9), 0.008)):
        ext = (16, 17, 18)
        c = tuple((lo[a] + 0.5 * ext[a]) * sp[a] for a in range(3))
        out.append(sphere_solid(grid, lo, ext, c, 0.07, sp, L=4, periodic=periodic,
                                warp=warp))
    return out


def test_periodic_grid_without_a_box_at_its_ends_is_the_walled_grid():
    grid, sp = (32, 28, 30), BLUR_SP
    sols = two_solids(grid, sp, (1, 0, 1))
    Hp, php, tp = blur_all(grid, sols, sp, (1, 0, 1))
    Hw, phw, tw = blur_all(grid, sols, sp, (0, 0, 0))
    assert np.array_equal(Hp, Hw)
    for a, b in zip(php, phw):
        assert np.array_equal(a, b)
    # faces 0 .. n-1 along x and z are the same faces; the walled grid's face n is extra
    assert np.array_equal(tp[0], tw[0][:, :, :, :grid[0]])
    assert np.array_equal(tp[1], tw[1])
    assert np.array_equal(tp[2], tw[2][:, :grid[2]])
    assert (Hp < 1.0).sum() > 500 and np.abs(tp[0][tp[0] != -7.0]).max() > 1e-3


@pytest.mark.parametrize("shift", [(9, 0, 0), (0, 0, 21), (25, 0, 13)])
def test_moving_every_box_along_a_periodic_axis_rolls_the_fields(shift):
    grid, sp, per = (32, 28, 30), BLUR_SP, (1, 0, 1)
    sols = two_solids(grid, sp, per)
    H0, ph0, t0 = blur_all(grid, sols, sp, per)
    moved = []
    for s in sols:
        m = list(s)
        m[0] = tuple((s[0][a] + shift[a]) % grid[a] for a in range(3))
        moved.append(m)
    assert any(m[0][a] + m[1][a] > grid[a] for m in moved for a in range(3))   # wraps
    H1, ph1, t1 = blur_all(grid, moved, sp, per)
    roll = dict(shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2))
    assert np.array_equal(H1, np.roll(H0, **roll))
    for a, b in zip(ph0, ph1):
        assert np.array_equal(a, b)
    for a in range(3):
        want = np.roll(t0[a], shift=(shift[2], shift[1], shift[0]), axis=(1, 2, 3))
        assert np.array_equal(t1[a], want)


def test_box_spanning_a_periodic_axis_never_joins_its_ends():
    """xi = A x + b unwrapped over a box that covers the whole periodic x axis: the map
    jumps by A e_x n Delta_x between the box's two ends.  Faces whose stencil stays in the
    box carry the closed form; the face between the box's last and first cells, and the
    faces whose tangential differences would need both ends, get no contribution."""
    grid, sp, G = (12, 14, 13), (0.05, 0.04, 0.06), 1.3
    lo, ext = (7, 2, 3), (12, 10, 9)
    A = np.array([[1.1, 0.2, -0.15], [0.05, 0.9, 0.3], [-0.2, 0.1, 1.05]])
    X = grid_coords(ext, sp, lo)
    xi = np.einsum("ab,bkji->akji", A, X)
    shape = oracle.make_shape(1, (0.0, 0.0, 0.0), (1e6,))
    sol = (lo, ext, shape, 6, xi, np.zeros(ext[::-1], np.int8))
    per = (1, 0, 0)
    tau = oracle.solid_stress(grid, [sol], EPS, sp, [G], tau_init(grid, per), periodic=per)
    want = expected_tau(np.linalg.inv(A), G)
    tx = tau[0]                                     # faces along x: 12, face i at cells i-1, i
    ys, zs = slice(lo[1] + 1, lo[1] + ext[1] - 1), slice(lo[2] + 1, lo[2] + ext[2] - 1)
    for i in range(grid[0]):
        f = tx[:, zs, ys, i]
        if i == lo[0]:                              # P would be the box's last cell
            assert np.array_equal(f, np.zeros_like(f))
        else:
            assert np.max(np.abs(f - want[:, None, None])) < 1e-11
    ty = tau[1]                                     # faces along y: x-differences needed
    for i in range(grid[0]):
        f = ty[:, zs, lo[1] + 1:lo[1] + ext[1], i]
        if i in (lo[0], (lo[0] - 1) % grid[0]):     # the box's first and last x cells
            assert np.array_equal(f, np.zeros_like(f))
        else:
            assert np.max(np.abs(f - want[:, None, None])) < 1e-11
