"""The layer count for a blur zone (rmx_layers_for_blur, host only): "Extrapolation of xi",
first paragraph -- L is chosen so that the band covers the whole blur zone.  Pinned by
brute force: around random resolved spheres and ellipsoids (xi = x), every cell with
phi0 < eps is labelled by the oracle's layers with the L the library returns, for both
adjacencies; and the count is the smallest of its closed form (a stated margin)."""
import math

import numpy as np
import pytest

import oracle
from paper_2104_00095_amd import rmx


def test_closed_form_values():
    # D = eps + sqrt(3) h; cube: ceil(D / h); faces: ceil(sqrt(3) D / h)
    h = 0.01
    assert rmx.layers_for_blur(2 * h, h, flags=rmx.FLAG_ADJ26) == math.ceil(2 + math.sqrt(3))
    assert rmx.layers_for_blur(2 * h, h) == math.ceil(math.sqrt(3) * (2 + math.sqrt(3)))
    assert rmx.layers_for_blur(2 * h, h, reach=2, flags=rmx.FLAG_ADJ26) == 4 + 2
    assert rmx.layers_for_blur(h, h, stretch=2.0, flags=rmx.FLAG_ADJ26) == \
        math.ceil(2 + math.sqrt(3))
    with pytest.raises(rmx.RmxError):
        rmx.layers_for_blur(20 * h, h)             # more than 16 layers
    for bad in ((0.0, h, 1.0, 0), (h, -1.0, 1.0, 0), (h, h, 0.5, 0), (h, h, 1.0, -1),
                (float("nan"), h, 1.0, 0)):
        with pytest.raises(rmx.RmxError):
            rmx.layers_for_blur(*bad)


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("adj", [6, 26])
def test_band_covers_the_blur_zone(seed, adj):
    rng = np.random.default_rng(300 + seed)
    n = 40
    h = 1.0 / n
    eps = float(rng.uniform(1.0, 2.5)) * h
    flags = rmx.FLAG_ADJ26 if adj == 26 else 0
    L = rmx.layers_for_blur(eps, h, flags=flags)
    c = rng.uniform(0.42, 0.58, 3)
    if seed % 2:
        shape = oracle.make_shape(1, c, (float(rng.uniform(0.08, 0.2)),))
    else:
        th = rng.uniform(0, 2 * math.pi, 3)
        Rz = np.array([[math.cos(th[0]), -math.sin(th[0]), 0], [math.sin(th[0]), math.cos(th[0]), 0], [0, 0, 1]])
        Rx = np.array([[1, 0, 0], [0, math.cos(th[1]), -math.sin(th[1])], [0, math.sin(th[1]), math.cos(th[1])]])
        shape = oracle.make_shape(2, c, tuple(rng.uniform(0.08, 0.2, 3)), Rz @ Rx)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h])
    prob = oracle.make_problem((n, n, n), (0, 0, 0), (n, n, n), shape, L, adjacency=adj)
    nint, lab, trunc = oracle.label(prob, X)
    assert nint > 0 and not trunc
    phi = np.vectorize(lambda x, y, z: oracle.phi0(shape, (x, y, z)))(X[0], X[1], X[2])
    blur = phi < eps
    assert np.all(lab[blur] >= 0), int((lab[blur] < 0).sum())


def test_grid_form_with_equal_spacings_is_the_plain_form():
    h = 0.02
    for eps, stretch, reach, flags in ((0.03, 1.0, 0, 0), (0.05, 1.5, 2, rmx.FLAG_ADJ26),
                                      (0.01, 1.0, 1, 0)):
        want = rmx.layers_for_blur(eps, h, stretch, reach, flags)
        assert rmx.layers_for_blur_grid(rmx.grid((10, 10, 10), h), eps, stretch, reach,
                                        flags) == want
        assert rmx.layers_for_blur_grid(rmx.grid((10, 10, 10), 1.0, spacing=(h, h, h)), eps,
                                        stretch, reach, flags) == want
    for bad in ((rmx.grid((10, 10, 10), h, spacing=(h, -h, h)), 0.03),
                (rmx.grid((10, 10, 10), h, spacing=(h, float("inf"), h)), 0.03),
                (rmx.grid((10, 10, 10), 0.0), 0.03), (rmx.grid((10, 10, 10), h), 0.0)):
        with pytest.raises(rmx.RmxError):
            rmx.layers_for_blur_grid(*bad)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("adj", [6, 26])
def test_band_covers_the_blur_zone_with_unequal_spacings(seed, adj):
    """Random spacings per axis (0.7..1.5 of h), random resolved spheres and rotated
    ellipsoids in physical coordinates (xi = x): every cell with phi0 < eps is labelled."""
    rng = np.random.default_rng(700 + seed)
    h = 1.0 / 40
    sp = tuple(float(v) for v in rng.uniform(0.7, 1.5, 3) * h)
    n = tuple(int(math.ceil(1.0 / d)) for d in sp)
    eps = float(rng.uniform(1.0, 2.5)) * max(sp)
    flags = rmx.FLAG_ADJ26 if adj == 26 else 0
    L = rmx.layers_for_blur_grid(rmx.grid(n, h, spacing=sp), eps, flags=flags)
    c = rng.uniform(0.42, 0.58, 3)
    if seed % 2:
        shape = oracle.make_shape(1, c, (float(rng.uniform(0.1, 0.2)),))
    else:
        th = rng.uniform(0, 2 * math.pi, 2)
        Rz = np.array([[math.cos(th[0]), -math.sin(th[0]), 0],
                       [math.sin(th[0]), math.cos(th[0]), 0], [0, 0, 1]])
        Rx = np.array([[1, 0, 0], [0, math.cos(th[1]), -math.sin(th[1])],
                       [0, math.sin(th[1]), math.cos(th[1])]])
        shape = oracle.make_shape(2, c, tuple(rng.uniform(0.1, 0.2, 3)), Rz @ Rx)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    X = np.stack([(i + 0.5) * sp[0], (j + 0.5) * sp[1], (k + 0.5) * sp[2]])
    prob = oracle.make_problem(n, (0, 0, 0), n, shape, L, adjacency=adj, spacing=sp)
    nint, lab, trunc = oracle.label(prob, X)
    assert nint > 0 and not trunc
    phi = np.vectorize(lambda x, y, z: oracle.phi0(shape, (x, y, z)))(X[0], X[1], X[2])
    blur = phi < eps
    assert np.all(lab[blur] >= 0), int((lab[blur] < 0).sum())
