"""Pins of the blur-zone oracle (smoothed Heaviside, multi-body modified Heaviside,
neo-Hookean solid stress at faces and its blend) against facts fixed outside it: the end
values, mirror symmetry and C^2 continuity of eq. (sm_heavi); bounds and limits of
eq. (mod_heaviside); closed forms of the stress for affine reference maps (centred
differences are exact there): zero for the identity and for rigid rotations (objectivity),
uniform stretch, simple shear, a general affine map through a library inverse; the
weights and the normalised blend of SI "Stress calculations".

Paper: main text "Blurred interface method and monolithic governing equations"
(eq. (blend), eq. (sm_heavi)); SI "Stress calculations" (F = (grad xi)^{-1}, B = F F^T,
tau_s = G (B - tr(B)/3 I), the blend over solids, eq. (mod_heaviside))."""
import math

import numpy as np
import pytest

import oracle

EPS = 0.1


def H(phi, eps=EPS):
    return oracle.heaviside_eps(phi, eps)


# ---- eq. (sm_heavi) ------------------------------------------------------------------

def test_heaviside_end_values_and_midpoint():
    assert H(-EPS) == 0.0 and H(-2 * EPS) == 0.0
    assert H(EPS) == 1.0 and H(3 * EPS) == 1.0
    assert H(0.0) == 0.5
    # at phi = eps/2: (1 + 1/2 + sin(pi/2)/pi) / 2
    assert H(0.5 * EPS) == pytest.approx(0.5 * (1.5 + 1.0 / math.pi), abs=1e-15)


def test_heaviside_mirror_symmetry_and_monotone():
    xs = np.linspace(-1.5 * EPS, 1.5 * EPS, 2001)
    v = np.array([H(x) for x in xs])
    w = np.array([H(-x) for x in xs])
    assert np.max(np.abs(v + w - 1.0)) < 1e-15
    assert np.all(np.diff(v) >= 0.0)
    assert v.min() == 0.0 and v.max() == 1.0


def test_heaviside_is_c2_at_the_ends():
    """The first and second derivatives vanish at +-eps from inside (one-sided
    differences), as they do outside: a continuous second derivative."""
    d = 1e-4 * EPS
    for e, s in ((EPS, -1), (-EPS, 1)):
        h0, h1, h2 = H(e), H(e + s * d), H(e + 2 * s * d)
        d1 = (h1 - h0) / d
        d2 = (h2 - 2 * h1 + h0) / (d * d)
        assert abs(d1) < 1e-6 and abs(d2) < 1e-2 / EPS


# ---- the blur field -----------------------------------------------------------------

def coords(lo, ext, h):
    k, j, i = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]),
                          indexing="ij")
    return np.stack([(lo[0] + i + 0.5) * h, (lo[1] + j + 0.5) * h, (lo[2] + k + 0.5) * h])


def sphere_solid(lo, ext, h, c, R, L=6, xi=None):
    X = coords(lo, ext, h)
    xi = X if xi is None else xi
    shape = oracle.make_shape(1, c, (R,))
    prob = oracle.make_problem((64, 64, 64), lo, ext, shape, L)
    n, labels, _ = oracle.label(prob, xi)
    assert n > 0
    return (lo, ext, shape, L, xi, labels)


def test_single_solid_blur_is_heaviside_of_distance():
    h = 1.0 / 32
    lo, ext = (2, 3, 1), (24, 22, 26)
    c, R = (0.45, 0.52, 0.44), 0.22
    s = sphere_solid(lo, ext, h, c, R)
    grid = (32, 32, 32)
    Hg, (phi,) = oracle.blur(grid, [s], EPS, np.full(grid[::-1], -3.0),
                             [np.full(ext[::-1], 9.0)])
    X = coords(lo, ext, h)
    dist = np.sqrt(((X - np.array(c)[:, None, None, None]) ** 2).sum(axis=0)) - R
    lab = s[5]
    band = lab >= 0
    assert np.max(np.abs(phi[band] - dist[band])) < 1e-14
    assert (phi[~band] == 9.0).all()
    box = Hg[lo[2]:lo[2] + ext[2], lo[1]:lo[1] + ext[1], lo[0]:lo[0] + ext[0]]
    expect = np.where(band, np.vectorize(H)(np.where(band, dist, 0.0)), 1.0)
    assert np.max(np.abs(box - expect)) < 1e-15
    # cells outside the box keep the caller's value
    mask = np.ones(grid[::-1], bool)
    mask[lo[2]:lo[2] + ext[2], lo[1]:lo[1] + ext[1], lo[0]:lo[0] + ext[0]] = False
    assert (Hg[mask] == -3.0).all()


def test_two_solid_modified_heaviside_bounds():
    h = 1.0 / 32
    s1 = sphere_solid((2, 4, 4), (20, 24, 24), h, (0.38, 0.5, 0.5), 0.16)
    s2 = sphere_solid((10, 4, 4), (20, 24, 24), h, (0.62, 0.5, 0.5), 0.16)
    grid = (32, 32, 32)
    init = np.full(grid[::-1], 1.0)
    Hb, _ = oracle.blur(grid, [s1, s2], 0.15, init)
    H1, _ = oracle.blur(grid, [s1], 0.15, init)
    H2, _ = oracle.blur(grid, [s2], 0.15, init)
    assert Hb.min() >= 0.0 and Hb.max() <= 1.0
    assert np.all(Hb <= np.minimum(H1, H2) + 1e-15)
    # max(1 - (1 - H1) - (1 - H2), 0), and order independence
    assert np.max(np.abs(Hb - np.maximum(H1 + H2 - 1.0, 0.0))) < 1e-15
    Hs, _ = oracle.blur(grid, [s2, s1], 0.15, init)
    assert np.max(np.abs(Hb - Hs)) < 1e-15
    # the overlap of the two blur zones is where the blend differs from either
    assert (np.abs(Hb - np.minimum(H1, H2)) > 1e-3).any()


# ---- solid stress at faces ------------------------------------------------------------

def affine_solid(A, b, lo=(3, 2, 4), ext=(10, 11, 9), h=0.05, L=6):
    """A box fully covered (labels 0) with xi = A x + b, inside a huge sphere (weight 1)."""
    X = coords(lo, ext, h)
    xi = np.einsum("ab,bkji->akji", A, X) + np.asarray(b)[:, None, None, None]
    shape = oracle.make_shape(1, (0.0, 0.0, 0.0), (1e6,))
    labels = np.zeros(ext[::-1], np.int8)
    return (lo, ext, shape, L, xi, labels), h


def stress_of(solids, h, G, grid=(20, 20, 20), eps=EPS):
    init = [np.full((6, grid[2] + (a == 2), grid[1] + (a == 1), grid[0] + (a == 0)), -7.0)
            for a in range(3)]
    return oracle.solid_stress(grid, solids, eps, h, G, init)


def inner_faces(sol, a):
    """Face indices (global) whose difference stencil lies inside the box."""
    lo, ext = sol[0], sol[1]
    sl = []
    for b in (2, 1, 0):
        if b == a:
            sl.append(slice(lo[b] + 1, lo[b] + ext[b]))
        else:
            sl.append(slice(lo[b] + 1, lo[b] + ext[b] - 1))
    return tuple(sl)


def expected_tau(F, G):
    B = F @ F.T
    t = G * (B - np.trace(B) / 3.0 * np.eye(3))
    return np.array([t[0, 0], t[1, 1], t[2, 2], t[0, 1], t[0, 2], t[1, 2]])


@pytest.mark.parametrize("case", ["identity", "stretch", "shear", "rotation", "affine"])
def test_stress_closed_forms(case):
    G = 2.5
    if case == "identity":
        A = np.eye(3)
    elif case == "stretch":
        lam = np.array([1.3, 0.8, 1 / (1.3 * 0.8)])
        A = np.diag(1.0 / lam)           # xi is the inverse of x = lam X
    elif case == "shear":
        g = 0.4
        A = np.array([[1.0, -g, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    elif case == "rotation":
        t = 0.7
        R = np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0],
                      [0.0, 0.0, 1.0]])
        A = R.T
    else:
        A = np.array([[1.1, 0.2, -0.15], [0.05, 0.9, 0.3], [-0.2, 0.1, 1.05]])
    sol, h = affine_solid(A, (0.1, -0.2, 0.3))
    tau = stress_of([sol], h, [G])
    F = np.linalg.inv(A)
    want = expected_tau(F, G)
    if case == "shear":
        g = 0.4
        assert np.allclose(want, [2 * G * g * g / 3, -G * g * g / 3, -G * g * g / 3, G * g, 0, 0])
    if case == "stretch":
        lam2 = np.array([1.3, 0.8, 1 / (1.3 * 0.8)]) ** 2
        assert np.allclose(want[:3], G * (lam2 - lam2.mean())) and np.allclose(want[3:], 0)
    if case in ("identity", "rotation"):
        assert np.allclose(want, 0.0, atol=1e-12)
    for a in range(3):
        got = tau[a][(slice(None),) + inner_faces(sol, a)]
        assert got.size > 0
        assert np.max(np.abs(got - want[:, None, None, None])) < 1e-11 * max(1.0, G)


def test_stress_written_where_a_box_cell_is_and_zero_without_stencil():
    sol, h = affine_solid(np.eye(3) * 1.2, (0, 0, 0))
    tau = stress_of([sol], h, [1.0])
    lo, ext = sol[0], sol[1]
    for a in range(3):
        t = tau[a]
        written = t[0] != -7.0
        # faces with a cell in the box: along a from lo[a] to lo[a] + ext[a], across the box
        want = np.zeros(written.shape, bool)
        sl = [slice(lo[b], lo[b] + ext[b]) for b in (2, 1, 0)]
        sl[2 - a] = slice(lo[a], lo[a] + ext[a] + 1)
        want[tuple(sl)] = True
        assert np.array_equal(written, want)
        inner = np.zeros(written.shape, bool)
        inner[inner_faces(sol, a)] = True
        # written faces without a full stencil carry zero
        assert (t[:, written & ~inner] == 0.0).all()


def test_weights_and_normalised_blend():
    G1, G2 = 1.0, 3.0
    A1 = np.diag([1.0 / 1.2, 1.0, 1.2])
    A2 = np.array([[1.0, -0.3, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    s1, h = affine_solid(A1, (0, 0, 0), lo=(3, 3, 3), ext=(10, 10, 10))
    s2, _ = affine_solid(A2, (0, 0, 0), lo=(5, 4, 3), ext=(10, 10, 10))
    tau = stress_of([s1, s2], h, [G1, G2])
    t1 = expected_tau(np.linalg.inv(A1), G1)
    t2 = expected_tau(np.linalg.inv(A2), G2)
    # deep in both: weights 1 + 1 = 2 > 1, so the mean
    f = (slice(None), slice(5, 12), slice(6, 12), slice(7, 12))   # x-faces [k, j, i]
    got = tau[0][f]
    assert np.max(np.abs(got - ((t1 + t2) / 2)[:, None, None, None])) < 1e-11
    # a solid whose weight is below one is scaled, not normalised: a sphere whose surface
    # crosses the box, identity map, one solid
    X = coords((3, 3, 3), (12, 12, 12), h)
    shape = oracle.make_shape(1, (0.45, 0.45, 0.45), (0.2,))
    labels = np.zeros((12, 12, 12), np.int8)
    A = np.diag([1.0 / 1.1, 1.1, 1.0])
    xi = np.einsum("ab,bkji->akji", A, X)
    sol = ((3, 3, 3), (12, 12, 12), shape, 6, xi, labels)
    tau = stress_of([sol], h, [2.0], eps=0.08)
    t = expected_tau(np.linalg.inv(A), 2.0)
    for a in range(3):
        sl = inner_faces(sol, a)
        # face xi: mean of the two cells' xi = A (face centre)
        k, j, i = np.meshgrid(np.arange(sl[0].start, sl[0].stop),
                              np.arange(sl[1].start, sl[1].stop),
                              np.arange(sl[2].start, sl[2].stop), indexing="ij")
        fc = np.stack([i + 0.5 * (a != 0), j + 0.5 * (a != 1), k + 0.5 * (a != 2)]) * h
        xf = np.einsum("ab,bkji->akji", A, fc)
        phi = np.sqrt(((xf - 0.45) ** 2).sum(axis=0)) - 0.2
        w = 1.0 - np.vectorize(lambda p: H(p, 0.08))(phi)
        got = tau[a][(slice(None),) + sl]
        assert np.max(np.abs(got - w[None] * t[:, None, None, None])) < 1e-11
        assert (w < 1.0).any() and (w > 0.0).any()


def test_stress_needs_every_stencil_cell_labelled():
    """An unlabelled plane inside the box: faces whose difference stencil touches it get no
    contribution (zero), all others keep the closed form."""
    A = np.diag([1.0 / 1.2, 1.0, 1.2])
    sol, h = affine_solid(A, (0, 0, 0), lo=(3, 3, 3), ext=(10, 10, 10))
    lab = sol[5].copy()
    zp = 5                                   # local z index of the unlabelled plane
    lab[zp] = -1
    sol = sol[:5] + (lab,)
    tau = stress_of([sol], h, [1.5])
    want = expected_tau(np.linalg.inv(A), 1.5)
    gz = 3 + zp                              # its global z index
    for a in range(3):
        t = tau[a]
        sl = inner_faces(sol, a)
        k = np.arange(sl[0].start, sl[0].stop)
        for kk in k:
            # z of the stencil cells: x/y faces reach kk-1..kk+1, z faces kk-1..kk
            zs = {kk - 1, kk} if a == 2 else {kk - 1, kk, kk + 1}
            got = t[:, kk, sl[1], sl[2]]
            if gz in zs:
                assert (got == 0.0).all(), (a, kk)
            else:
                assert np.max(np.abs(got - want[:, None, None])) < 1e-11, (a, kk)
