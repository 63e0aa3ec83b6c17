"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU.

Labels, decision paths and per-solid counts must be identical; xi within 1e-12 relative
max-norm (FP64 path) or 1e-5 (FP32-accumulate path); interior and unmarked cells bitwise
unchanged.  Every workload is checked in full: the oracle finishes each in seconds.
"""
import numpy as np
import pytest

import oracle
from paper_2104_00095_amd import synth
from tests.helpers import (axis_plane_workload, edge_workloads, oracle_problem, rel_err,
                           run_oracle, wide_box_sphere, mixed_kinds_workload)

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}
# Launch forms: every solid of the call in one chain of launches (default), one chain per
# solid (the plain form), and the band work in one persistent launch.
MODES = {"batched": 0, "per_solid": 4, "persistent": 16}
MODE_PARAMS = sorted(MODES)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2104_00095_amd import rmx
    assert torch.cuda.is_available()
    c = rmx.Context(0)
    yield c
    c.close()


def run_gpu(ctx, w, precision=0, r_s=2, r_max=4, normal_layers=2, flags=0,
            xi_normal=None, decisions=True):
    import torch
    from paper_2104_00095_amd import fields, rmx
    dw = fields.upload(w, decisions=decisions, xi_normal=xi_normal)
    opt = rmx.options(r_s=r_s, r_max=r_max, normal_layers=normal_layers, precision=precision,
                      flags=flags)
    st, stats = ctx.extrapolate(dw.grid, dw.solids, opt, check=False)
    torch.cuda.synchronize()
    out = []
    for i in range(len(w.solids)):
        out.append((dw.xi[i].cpu().numpy(), dw.labels[i].cpu().numpy(),
                    dw.decisions[i].cpu().numpy() if decisions else None, stats[i]))
    return st, out


def compare(w, gpu, precision, r_s=2, r_max=4, normal_layers=2, xi_normal=None, tag="",
            adjacency=6):
    worst = 0.0
    for i, s in enumerate(w.solids):
        xg, lg, dg, stg = gpu[i]
        st, xo, lo, do, so = run_oracle(w, s, r_s=r_s, r_max=r_max,
                                        normal_layers=normal_layers,
                                        xi_normal=None if xi_normal is None else xi_normal[i],
                                        adjacency=adjacency)
        assert stg["status"] == st, (tag, i, stg["status"], st)
        assert np.array_equal(lg, lo), (tag, i, "labels", int((lg != lo).sum()))
        if dg is not None and st == 0:
            mism = np.argwhere(dg != do)
            assert mism.size == 0, (tag, i, "decisions", mism[:5], dg[tuple(mism[0])],
                                    do[tuple(mism[0])])
        assert stg["n_interior"] == so[0]
        assert stg["n_band"][1:17] == [int(v) for v in so[1:17]], (tag, i)
        if st == 0:
            assert [stg["n_r_grown"], stg["n_no_normal"], stg["n_f1"], stg["n_f2"]] == \
                [int(v) for v in so[17:21]], (tag, i)
        keep = lo <= 0
        assert np.array_equal(xg[:, keep].view(np.uint64), s.xi[:, keep].view(np.uint64)), \
            (tag, i, "known cells changed")
        band = lo > 0
        if st != 0:
            assert np.array_equal(xg.view(np.uint64), s.xi.view(np.uint64))
            continue
        e = rel_err(xg, xo, band)
        worst = max(worst, e)
        assert e <= TOL[precision], (tag, i, e)
    return worst


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_sphere32(ctx, precision, mode):
    w = synth.sphere32()
    st, gpu = run_gpu(ctx, w, precision, flags=MODES[mode])
    assert st == 0
    print("sphere32 rel err", compare(w, gpu, precision, tag="sphere32"))


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_ellipsoid_ragged(ctx, precision, mode):
    """40^3: ragged tiles along every axis (40 = 64 - 24 along x, 2.5 tiles in y, z)."""
    w = synth.ellipsoid128(n=40, n_layers=5)
    st, gpu = run_gpu(ctx, w, precision, flags=MODES[mode])
    assert st == 0
    compare(w, gpu, precision, tag="ell40")


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_ellipsoid128_full(ctx, precision, mode):
    w = synth.ellipsoid128()
    st, gpu = run_gpu(ctx, w, precision, flags=MODES[mode])
    assert st == 0
    print("ellipsoid128 rel err", compare(w, gpu, precision, tag="ell128"))


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_suspension_batched_full(ctx, precision, mode):
    w = synth.suspension()
    st, gpu = run_gpu(ctx, w, precision, flags=MODES[mode])
    assert st == 0
    print("suspension rel err", compare(w, gpu, precision, tag="susp"))


@pytest.mark.parametrize("n,L,tile_w", [(40, 16, 0), (48, 11, 0), (48, 11, 1), (40, 16, 2)])
def test_many_layers(ctx, n, L, tile_w):
    """Layer numbers up to 16 need all five bit planes of the label tiles (layers 8..16
    use the upper two); every label tile width that fits the LDS."""
    from paper_2104_00095_amd import fields, rmx
    w = synth.sphere32(n=n, n_layers=L)
    if tile_w:
        dw = fields.upload(w)
        ctx.set_tuning(dw.grid, dw.solids, tile_w, 256)
    st, gpu = run_gpu(ctx, w)
    assert st == 0 and int(gpu[0][1].max()) == L
    compare(w, gpu, 0, tag=f"sphere{n}_L{L}_tw{tile_w}")


@pytest.mark.parametrize("precision", [0, 1])
def test_sphere_and_ellipsoid_in_one_batch(ctx, precision):
    """A batch with both kinds runs the normal kernel's general form; each solid equals
    the oracle as when it is alone."""
    w = mixed_kinds_workload()
    st, gpu = run_gpu(ctx, w, precision)
    compare(w, gpu, precision, tag="mixed_kinds")


@pytest.mark.parametrize("L,tile_w", [(16, 0), (16, 1), (4, 1), (4, 2)])
def test_label_tiles_narrower_than_the_box(ctx, L, tile_w):
    """A box 130 cells wide (two words and a ragged third per row, no row 8-byte
    aligned): tiles narrower than the box write their rows in runs of one row."""
    from paper_2104_00095_amd import fields
    w = wide_box_sphere(n_layers=L)
    if tile_w:
        dw = fields.upload(w)
        ctx.set_tuning(dw.grid, dw.solids, tile_w, 256)
    st, gpu = run_gpu(ctx, w)
    assert st == 0 and int(gpu[0][1].max()) == L
    compare(w, gpu, 0, tag=f"wide_box_L{L}_tw{tile_w}")


@pytest.mark.parametrize("seed", range(31, 39))
def test_small_suspensions(ctx, seed):
    """Eight random batches of 8 small ellipsoids (semi-axes 2-5 cells, arbitrary
    rotations), L from 2 to 5, FP64 and FP32-accumulate in turn: strongly curved bands for
    the distance, the normals and the rank tests."""
    w = synth.suspension(seed=seed, n_solids=8, grid_n=(48, 48, 64), h=1 / 48,
                         n_layers=2 + seed % 4)
    precision = seed % 2
    st, gpu = run_gpu(ctx, w, precision)
    assert st == 0
    compare(w, gpu, precision, tag=f"small_susp{seed}")


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_cavity256_full(ctx, precision, mode):
    w = synth.cavity256()
    st, gpu = run_gpu(ctx, w, precision, decisions=True, flags=MODES[mode])
    assert st == 0
    print("cavity256 rel err", compare(w, gpu, precision, tag="cav256"))


def test_affine_reproduced_on_gpu(ctx):
    w = synth.sphere32(affine=True)
    s = w.solids[0]
    _, _, lab0, _, _ = run_oracle(w, s)
    band = lab0 > 0
    c = s.shape.centre
    d = s.xi[:, band] - c[:, None]
    s.xi[:, band] += 0.5 * w.h * d / np.linalg.norm(d, axis=0)
    A, b = w.affine
    x, y, z = synth.cell_centres(s.lo, s.ext, w.h, w.origin)
    X = np.broadcast_arrays(x, y, z)
    exact = np.stack([b[a] + A[a, 0] * X[0] + A[a, 1] * X[1] + A[a, 2] * X[2] for a in range(3)])
    for prec, tol in ((0, 1e-13), (1, 1e-6)):
        st, gpu = run_gpu(ctx, w, prec)
        xg, lg = gpu[0][0], gpu[0][1]
        assert np.array_equal(lg, lab0)
        assert rel_err(xg, exact, band) < tol


def _mask_workload(masks, L, grid_n=None, inside=(0.0, 0.0, 0.0)):
    w = synth.Workload("masks", grid_n or (masks[0].shape[2], masks[0].shape[1],
                                           masks[0].shape[0]), 1.0, (0.0, 0.0, 0.0))
    for m in masks:
        n2, n1, n0 = m.shape
        xi = synth.tiny_field_from_mask(m, inside_value=inside)
        w.solids.append(synth.Solid((0, 0, 0), (n0, n1, n2),
                                    synth.sphere_shape((0.0, 0.0, 0.0), 1.0), L, xi))
    return w


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("seed", range(6))
def test_random_masks_batched(ctx, seed, mode):
    """Many tiny solids of random shapes and layer counts in one batched call."""
    from tests.test_oracle_pins import _random_mask
    rng = np.random.default_rng(500 + seed)
    w = synth.Workload("masks", (20, 20, 20), 1.0, (0.0, 0.0, 0.0))
    for q in range(12):
        shp = tuple(int(v) for v in rng.integers(3, 21, size=3))
        m = _random_mask(rng, shp)
        L = int(rng.integers(0, 8))
        xi = synth.tiny_field_from_mask(m, inside_value=tuple(rng.uniform(-0.3, 0.3, 3)))
        # band cells get finite exterior values half of the time (normals from them)
        if q % 2:
            ext = ~m
            xi[:, ext] = 2.0 + rng.random((3, int(ext.sum())))
        w.solids.append(synth.Solid((0, 0, 0), (shp[2], shp[1], shp[0]),
                                    synth.sphere_shape((0.0, 0.0, 0.0), 1.0), L, xi))
    st, gpu = run_gpu(ctx, w, 0, flags=MODES[mode])
    compare(w, gpu, 0, tag=f"masks{seed}")


@pytest.mark.parametrize("mode", MODE_PARAMS)
def test_degenerate_paths(ctx, mode):
    """Single interior cell and one-cell-thin plate: radius growth, F1/F2 fallbacks."""
    m1 = np.zeros((9, 9, 9), dtype=bool)
    m1[4, 4, 4] = True
    m2 = np.zeros((15, 15, 15), dtype=bool)
    m2[7] = True
    w = _mask_workload([m1, m2], 3, grid_n=(15, 15, 15), inside=(0.1, 0.2, 0.3))
    w.solids[0].lo = (0, 0, 0)
    st, gpu = run_gpu(ctx, w, 0, flags=MODES[mode])
    compare(w, gpu, 0, tag="degenerate")
    assert gpu[0][3]["n_f2"] > 0 and gpu[1][3]["n_f2"] > 0


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_f1_and_grown_normal_fit(ctx, precision, mode):
    """Two one-cell plates with the normal fixed along +x (tests/helpers
    ``plates_workload``): whole planes of layer-1 cells whose positive-weight data stay
    coplanar up to r_max take F1 (kernel weights at radius 4), and the plane beyond the
    second plate is fitted with the normal factor at radius 4.  Both are the radius-4
    gathers from global memory, with and without the normal factor."""
    from tests.helpers import plates_workload
    w, xn = plates_workload()
    st, gpu = run_gpu(ctx, w, precision, flags=MODES[mode], xi_normal=[xn])
    assert st == 0
    compare(w, gpu, precision, xi_normal=[xn], tag="plates")
    dec, stats = gpu[0][2], gpu[0][3]
    assert stats["n_f1"] >= 3 * 81
    assert np.all(dec[:, :, [3, 5, 6]] == 32)
    assert dec[4, 4, 8] == 4


@pytest.mark.parametrize("mode", MODE_PARAMS)
def test_normal_factor_half_space(ctx, mode):
    """The half-space probe whose layer-1 value has a closed form under eq. (weight) (the
    oracle pin test_normal_factor_value_closed_form): interior k <= 3, xi = ((i-4)^2, 0, 0),
    normals along +z from a separate field."""
    n0, n1, n2 = 9, 9, 8
    xi = np.full((3, n2, n1, n0), np.nan)
    xi[0, :4] = ((np.arange(n0) - 4.0) ** 2)[None, None, :]
    xi[1, :4] = 0.0
    xi[2, :4] = 0.0
    xn = np.zeros_like(xi)
    xn[2] = (500.0 + 0.25 * np.arange(n2))[:, None, None]
    w = synth.Workload("half_space", (n0, n1, n2), 1.0, (0.0, 0.0, 0.0))
    w.solids.append(synth.Solid((0, 0, 0), (n0, n1, n2),
                                synth.sphere_shape((0.0, 0.0, 0.0), 1000.0), 3, xi))
    st, gpu = run_gpu(ctx, w, 0, flags=MODES[mode], xi_normal=[xn])
    assert st == 0
    compare(w, gpu, 0, xi_normal=[xn], tag="half_space")
    assert gpu[0][2][4, 4, 4] == 2


@pytest.mark.parametrize("mode", MODE_PARAMS)
@pytest.mark.parametrize("r_s,normal_layers", [(1, 2), (2, 0), (3, 4)])
def test_option_variants(ctx, r_s, normal_layers, mode):
    w = synth.sphere32(seed=7)
    st, gpu = run_gpu(ctx, w, 0, r_s=r_s, normal_layers=normal_layers, flags=MODES[mode])
    compare(w, gpu, 0, r_s=r_s, normal_layers=normal_layers, tag=f"opt{r_s}{normal_layers}")


def test_xi_normal_field(ctx):
    """Normals taken from a separate field (the previous step's xi)."""
    w = synth.sphere32(seed=3)
    prev = synth.sphere32(seed=4).solids[0].xi
    st, gpu = run_gpu(ctx, w, 0, xi_normal=[prev])
    compare(w, gpu, 0, xi_normal=[prev], tag="xi_normal")


@pytest.mark.parametrize("mode", MODE_PARAMS)
def test_statuses(ctx, mode):
    from paper_2104_00095_amd import rmx
    w = synth.sphere32()
    s = w.solids[0]
    sub = synth.Workload("trunc", w.grid_n, w.h, w.origin)
    sub.solids.append(synth.Solid((8, 4, 4), (12, 24, 24), s.shape, 4,
                                  s.xi[:, 4:28, 4:28, 8:20].copy()))
    sub.solids.append(synth.Solid(s.lo, s.ext, s.shape, 4, s.xi + 10.0))      # empty
    sub.solids.append(synth.Solid(s.lo, s.ext, s.shape, 0, s.xi.copy()))      # L = 0
    sub.solids.append(synth.Solid(s.lo, s.ext, s.shape, 4, s.xi.copy()))      # normal
    st, gpu = run_gpu(ctx, sub, 0, flags=MODES[mode])
    assert st == rmx.E_TRUNCATED
    assert [g[3]["status"] for g in gpu] == [rmx.E_TRUNCATED, rmx.W_EMPTY, 0, 0]
    compare(sub, gpu, 0, tag="statuses")


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_alone_and_per_solid(ctx, precision):
    """Object independence: each solid's result in the batched call is bitwise the result
    of its solo call and of the per-solid form (the per-cell arithmetic does not depend on
    the batch or the form)."""
    from paper_2104_00095_amd import rmx
    w = synth.suspension(n_solids=12, grid_n=(64, 64, 128), h=1.0 / 64)
    st, batched = run_gpu(ctx, w, precision)
    st2, per = run_gpu(ctx, w, precision, flags=rmx.FLAG_PER_SOLID)
    assert st == st2 == 0
    for i, s in enumerate(w.solids):
        one = synth.Workload("one", w.grid_n, w.h, w.origin)
        one.solids.append(s)
        _, alone = run_gpu(ctx, one, precision)
        assert np.array_equal(batched[i][0].view(np.uint64), alone[0][0].view(np.uint64))
        assert np.array_equal(batched[i][0].view(np.uint64), per[i][0].view(np.uint64))
        assert np.array_equal(batched[i][1], alone[0][1])
        assert np.array_equal(batched[i][2], per[i][2])


@pytest.mark.parametrize("mode", MODE_PARAMS)
def test_nonfinite_and_boundary(ctx, mode):
    """Classification edge cases (NaN / inf components, cells exactly on the sphere or on
    an axis) for a sphere and a rotated ellipsoid."""
    for w in edge_workloads():
        st, gpu = run_gpu(ctx, w, 0, flags=MODES[mode])
        compare(w, gpu, 0, tag="edge")


@pytest.mark.parametrize("mode", MODE_PARAMS)
def test_ellipsoid_axis_planes(ctx, mode):
    """Body coordinates exactly 0 and far below 2^-200 in the cells whose phi0 the normals
    need: the bisection's dropped terms and its plain-division path."""
    w = axis_plane_workload()
    st, gpu = run_gpu(ctx, w, 0, flags=MODES[mode])
    assert st == 0
    compare(w, gpu, 0, tag="axis_planes")


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_equals_chain(ctx, precision):
    """The persistent band launch runs the same per-brick arithmetic as the chain of
    launches: labels, decisions, statistics and xi are bitwise those of the chain, on a
    batch of ellipsoids, a sphere and a ragged ellipsoid box."""
    from paper_2104_00095_amd import rmx
    for w in (synth.suspension(n_solids=12, grid_n=(64, 64, 128), h=1.0 / 64),
              synth.sphere32(), synth.ellipsoid128(n=48, n_layers=5)):
        st, chain = run_gpu(ctx, w, precision)
        st2, pers = run_gpu(ctx, w, precision, flags=rmx.FLAG_PERSISTENT)
        assert st == st2 == 0
        for (xa, la, da, sa), (xb, lb, db, sb) in zip(chain, pers):
            assert np.array_equal(la, lb) and np.array_equal(da, db) and sa == sb
            assert np.array_equal(xa.view(np.uint64), xb.view(np.uint64))


@pytest.mark.parametrize("mode", MODE_PARAMS)
def test_graph_replay_matches_eager(ctx, mode):
    import torch
    from paper_2104_00095_amd import fields, rmx
    w = synth.suspension(n_solids=8, grid_n=(64, 64, 128), h=1.0 / 64)
    dw = fields.upload(w)
    ctx.extrapolate(dw.grid, dw.solids, rmx.options(flags=MODES[mode]))
    eager = [x.clone() for x in dw.xi]
    opt = rmx.options(flags=rmx.FLAG_GRAPH | MODES[mode])
    for rep in range(4):
        dw.reset()
        torch.cuda.synchronize()
        st, stats = ctx.extrapolate(dw.grid, dw.solids, opt)
        torch.cuda.synchronize()
        assert st == 0
        for a, b in zip(dw.xi, eager):
            assert torch.equal(a, b), rep
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between


def test_deterministic_repeats(ctx):
    import torch
    from paper_2104_00095_amd import fields, rmx
    w = synth.ellipsoid128(n=64)
    dw = fields.upload(w)
    outs = []
    for prec in (0, 1):
        for _ in range(3):
            dw.reset()
            ctx.extrapolate(dw.grid, dw.solids, rmx.options(precision=prec))
            torch.cuda.synchronize()
            outs.append(dw.xi[0].cpu().numpy().copy())
        assert np.array_equal(outs[-1].view(np.uint64), outs[-2].view(np.uint64))
        assert np.array_equal(outs[-1].view(np.uint64), outs[-3].view(np.uint64))


def test_autotune_keeps_inputs_and_results(ctx):
    """The autotuner restores xi, and a call with the tuned launch shapes gives, bit for
    bit, the result of a context that was never tuned."""
    import torch
    from paper_2104_00095_amd import fields, rmx
    w = synth.suspension(n_solids=6, grid_n=(64, 64, 128), h=1.0 / 64)
    dw = fields.upload(w)
    before = [x.clone() for x in dw.xi]
    best = ctx.autotune(dw.grid, dw.solids, rmx.options(), reps=2)
    torch.cuda.synchronize()
    assert best["tile_w"] in (1, 2, 4) and best["extrap_blocks"] > 0 and best["ms"] > 0
    for a, b in zip(dw.xi, before):
        assert torch.equal(a, b)
    st, tuned = run_gpu(ctx, w, 0)
    fresh = rmx.Context(0)
    try:
        st2, plain = run_gpu(fresh, w, 0)
    finally:
        fresh.close()
    assert st == st2 == 0
    for (xa, la, da, _), (xb, lb, db, _) in zip(tuned, plain):
        assert np.array_equal(xa.view(np.uint64), xb.view(np.uint64))
        assert np.array_equal(la, lb) and np.array_equal(da, db)
    print("autotune", best)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["sphere32", "ellipsoid48", "suspension12"])
def test_cube_adjacency_matches_oracle(ctx, name, precision):
    """Layers by the 26-neighbour adjacency (RMX_FLAG_ADJ26): labels equal the oracle's
    (Chebyshev distances), decisions and the band as for face layers."""
    from paper_2104_00095_amd import rmx
    w = {"sphere32": lambda: synth.sphere32(),
         "ellipsoid48": lambda: synth.ellipsoid128(n=48, n_layers=5),
         "suspension12": lambda: synth.suspension(n_solids=12, grid_n=(64, 64, 128),
                                                  h=1.0 / 64)}[name]()
    for fl in (0, rmx.FLAG_GRAPH):
        st, gpu = run_gpu(ctx, w, precision, flags=rmx.FLAG_ADJ26 | fl)
        assert st == 0
        compare(w, gpu, precision, tag=f"adj26/{name}/{fl}", adjacency=26)
    # the face-layer call after it is not affected (graph and tuning keys differ)
    st, gpu = run_gpu(ctx, w, precision)
    compare(w, gpu, precision, tag=f"adj6/{name}")
