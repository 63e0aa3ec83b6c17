"""The library's HIP kernels, host core included, built for the CPU over a host emulation
of the HIP subset they use (tests/cpu_hip) and run under AddressSanitizer and
UndefinedBehaviorSanitizer on tiny workloads.  Labels and decisions must equal the
oracle's and xi must meet the GPU tolerance.  The threads of a block are host threads
(blocks run in turn), and the workspace regions are separated by poisoned red zones, so an
access past any region is reported.  Test infrastructure only: the product library never
contains this build.  The emulated runs are separate processes; they run four at a time,
once per module, and each test checks its own.
"""
import os
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2104_00095_amd import synth
from tests.helpers import (axis_plane_workload, edge_workloads, plates_workload, rel_err,
                           run_oracle, wide_box_sphere, mixed_kinds_workload)

emu = pytest.importorskip("tests.cpu_hip.emu")
pytestmark = pytest.mark.skipif(not os.path.exists(emu.CLANG), reason="no host clang++")

TOL = {0: 1e-12, 1: 1e-5}
BATCHED, PER_SOLID, GRAPH, PERSISTENT, ADJ26 = 0, 4, 2, 16, 32
AUTOTUNE = 1024   # (run_case: run the autotuner on the fields first)
TILE_W = 8192     # (run_case: TILE_W + w fixes the label tile width w first)
NOALLOC = 4096    # (run_case: make the call through the allocation-free entry point)


def _truncation_batch():
    """Truncated band, no interior cell, L = 0 and an ordinary solid in one batch."""
    w0 = synth.sphere32(n=24, n_layers=3)
    s = w0.solids[0]
    w = synth.Workload("statuses", w0.grid_n, w0.h, w0.origin)
    w.solids.append(synth.Solid((8, 4, 4), (10, 16, 16), s.shape, 3,
                                s.xi[:, 4:20, 4:20, 8:18].copy()))
    w.solids.append(synth.Solid(s.lo, s.ext, s.shape, 3, s.xi + 10.0))
    w.solids.append(synth.Solid(s.lo, s.ext, s.shape, 0, s.xi.copy()))
    w.solids.append(synth.Solid(s.lo, s.ext, s.shape, 3, s.xi.copy()))
    return w


def _runs():
    sphere = synth.sphere32(n=16, n_layers=3)
    ell = synth.ellipsoid128(n=24, n_layers=3)
    susp = synth.suspension(n_solids=3, grid_n=(24, 24, 40), h=1 / 24)
    edges = edge_workloads()
    trunc = _truncation_batch()
    plates, plates_xn = plates_workload()
    # name: (workload, precision, flags, calls made first on the same context[, options:
    # "cus" = compute units of the emulated device, "xi_normal" = per-solid normal fields])
    return {
        "sphere16": (sphere, 0, BATCHED, ()),
        "ellipsoid24": (ell, 0, BATCHED, ()),
        "suspension3": (susp, 0, BATCHED, ()),
        "suspension3_per_solid": (susp, 0, PER_SOLID, ()),
        "suspension3_fp32_graph": (susp, 1, GRAPH, ()),
        # 5 CUs: 15 fit blocks over 8 XCDs, two blocks on some and one on others
        "suspension3_cus5": (susp, 0, BATCHED, (), {"cus": 5}),
        "repeated_calls": (susp, 0, BATCHED, (BATCHED, GRAPH, BATCHED)),
        "autotune_then_call": (sphere, 0, BATCHED, (AUTOTUNE,)),
        # the persistent band launch: every block of it runs at once (they wait on each
        # other's layers), after other forms on the same context, with graph replay
        "persistent": (sphere, 0, PERSISTENT, ()),
        "persistent_suspension_fp32": (susp, 1, PERSISTENT, ()),
        "persistent_graph_after_chain": (susp, 0, PERSISTENT | GRAPH, (BATCHED, PERSISTENT)),
        "persistent_statuses": (trunc, 0, PERSISTENT, ()),
        "persistent_plates": (plates, 0, PERSISTENT, (), {"xi_normal": [plates_xn]}),
        # 12 blocks: 8 queues, four of them with two blocks
        "persistent_cus12": (susp, 0, PERSISTENT, (), {"cus": 12}),
        "statuses_batched": (trunc, 0, BATCHED, ()),
        "statuses_per_solid": (trunc, 0, PER_SOLID, ()),
        "sphere64": (synth.sphere32(n=64, n_layers=3), 0, BATCHED, ()),
        # 16 layers: the label tiles' five bit planes all in use
        "sphere40_L16": (synth.sphere32(n=40, n_layers=16), 0, BATCHED, ()),
        # a sphere and an ellipsoid in one call: the general forms
        "mixed_kinds": (mixed_kinds_workload(n=24, n_layers=4), 0, BATCHED, ()),
        # label tiles narrower than a 130-cell box: rows written in runs of one row
        "wide_box_L16_tw1": (wide_box_sphere(n_layers=16), 0, BATCHED, (TILE_W + 1,)),
        "wide_box_L4_tw2": (wide_box_sphere(n_layers=4), 0, BATCHED, (TILE_W + 2,)),
        # 64 CUs: 125 fit blocks for a few dozen bricks per layer (most blocks find no
        # brick of their own)
        "ellipsoid40_cus64": (synth.ellipsoid128(n=40, n_layers=4), 0, BATCHED, (),
                              {"cus": 64}),
        "ellipsoid40_cus64_fp32": (synth.ellipsoid128(n=40, n_layers=4), 1, BATCHED, (),
                                   {"cus": 64}),
        "edge_sphere": (edges[0], 0, BATCHED, ()),
        "edge_ellipsoid": (edges[1], 0, BATCHED, ()),
        "axis_planes": (axis_plane_workload(), 0, BATCHED, ()),
        # F1 and a normal-weighted radius-4 fit (gathers from global memory)
        "plates": (plates, 0, BATCHED, (), {"xi_normal": [plates_xn]}),
        "plates_fp32_per_solid": (plates, 1, PER_SOLID, (), {"xi_normal": [plates_xn]}),
        # the allocation-free entry point (the static scratch array), after calls of both
        # entry points on a larger batch (the scratch keeps their contents)
        "noalloc": (sphere, 0, NOALLOC, (BATCHED, NOALLOC | PER_SOLID)),
        "noalloc_suspension_per_solid": (susp, 1, NOALLOC | PER_SOLID, (NOALLOC,)),
        # layers by the 26-neighbour adjacency, after a face-layer call on the context
        "adj26_sphere16": (sphere, 0, ADJ26, (BATCHED,)),
        "adj26_suspension3_fp32_graph": (susp, 1, ADJ26 | GRAPH, (GRAPH,)),
        "adj26_ellipsoid24_persistent": (ell, 0, ADJ26 | PERSISTENT, ()),
    }


@pytest.fixture(scope="module")
def emulated():
    emu.build()
    root = tempfile.mkdtemp(prefix="rmx_emu_")

    def one(item):
        name, (w, prec, flags, pre, *extra) = item
        o = extra[0] if extra else {}
        st, outs = emu.run(w, os.path.join(root, name), precision=prec, flags=flags,
                           pre_flags=pre, cus=o.get("cus"), xi_normal=o.get("xi_normal"))
        return name, (w, prec, st, outs, o.get("xi_normal"))

    with ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(one, _runs().items()))


def _check(w, outs, precision, xi_normal=None, adjacency=6):
    for i, ((xo, lab, dec, _), s) in enumerate(zip(outs, w.solids)):
        st, xr, lr, dr, _ = run_oracle(w, s, xi_normal=None if xi_normal is None
                                       else xi_normal[i], adjacency=adjacency)
        assert np.array_equal(lab, lr)
        if st == 0:
            assert np.array_equal(dec, dr)
            assert rel_err(xo, xr, lr > 0) <= TOL[precision]
        keep = lr <= 0 if st == 0 else np.ones(lr.shape, bool)
        assert np.array_equal(xo[:, keep].view(np.uint64), s.xi[:, keep].view(np.uint64))


@pytest.mark.parametrize("name", ["sphere16", "ellipsoid24", "suspension3",
                                  "suspension3_per_solid", "suspension3_fp32_graph",
                                  "suspension3_cus5", "sphere64", "sphere40_L16",
                                  "wide_box_L16_tw1", "wide_box_L4_tw2", "mixed_kinds",
                                  "ellipsoid40_cus64", "ellipsoid40_cus64_fp32"])
def test_emulated_kernels_match_oracle(emulated, name):
    w, prec, st, outs, xn = emulated[name]
    assert st == 0
    _check(w, outs, prec, xn)


def test_emulated_repeated_calls(emulated):
    """Calls of different forms on one context (shared workspace, descriptors cached
    between identical calls), each on a fresh copy of the field, before the checked call."""
    w, prec, st, outs, xn = emulated["repeated_calls"]
    assert st == 0
    _check(w, outs, prec, xn)


def test_emulated_autotune_then_call(emulated):
    """The autotuner (every candidate launch shape, xi saved and restored) followed by the
    checked call with the tuned shapes: the result must still be the oracle's."""
    w, prec, st, outs, xn = emulated["autotune_then_call"]
    assert st == 0
    _check(w, outs, prec, xn)


@pytest.mark.parametrize("name", ["persistent", "persistent_suspension_fp32",
                                  "persistent_graph_after_chain", "persistent_plates",
                                  "persistent_cus12"])
def test_emulated_persistent_band_launch(emulated, name):
    """The normals and every layer's fits in one persistent launch whose blocks take
    bricks by ticket and wait for the previous layer: the oracle's labels, decisions and
    xi."""
    w, prec, st, outs, xn = emulated[name]
    assert st == 0
    _check(w, outs, prec, xn)


def test_emulated_persistent_statuses(emulated):
    """A truncated solid, one with no interior cell and one with L = 0 beside an ordinary
    solid, through the persistent launch."""
    w, prec, st, outs, xn = emulated["persistent_statuses"]
    assert st == -7
    _check(w, outs, prec, xn)


@pytest.mark.parametrize("name", ["statuses_batched", "statuses_per_solid"])
def test_emulated_statuses(emulated, name):
    """Truncated band, no interior cell and L = 0 in one batch."""
    w, prec, st, outs, xn = emulated[name]
    assert st == -7
    _check(w, outs, prec, xn)


@pytest.mark.parametrize("name", ["edge_sphere", "edge_ellipsoid", "axis_planes"])
def test_emulated_nonfinite_and_boundary(emulated, name):
    """Edge cases against the oracle: NaN and infinite components, cells exactly on
    |xi - c|^2 = R^2 or on an axis (a sphere and a rotated ellipsoid); body coordinates
    exactly 0 or +-1e-230 in the cells whose distance the normals need."""
    w, prec, st, outs, xn = emulated[name]
    _check(w, outs, prec, xn)


@pytest.mark.parametrize("name", ["plates", "plates_fp32_per_solid"])
def test_emulated_f1_and_grown_normal_fit(emulated, name):
    """Two plates with the normal fixed along +x: F1 on whole planes of layer-1 cells and
    a normal-weighted fit at radius 4 (tests/helpers plates_workload)."""
    w, prec, st, outs, xn = emulated[name]
    assert st == 0
    _check(w, outs, prec, xn)
    dec = outs[0][2]
    assert np.all(dec[:, :, [3, 5, 6]] == 32) and dec[4, 4, 8] == 4


@pytest.mark.parametrize("name", ["noalloc", "noalloc_suspension_per_solid"])
def test_emulated_noalloc_entry(emulated, name):
    """rmx_extrapolate_noalloc on the static scratch array, after earlier calls on the same
    context left their contents there."""
    w, prec, st, outs, xn = emulated[name]
    assert st == 0
    _check(w, outs, prec, xn)


@pytest.mark.parametrize("name", ["adj26_sphere16", "adj26_suspension3_fp32_graph",
                                  "adj26_ellipsoid24_persistent"])
def test_emulated_cube_adjacency(emulated, name):
    w, prec, st, outs, xn = emulated[name]
    assert st == 0
    _check(w, outs, prec, xn, adjacency=26)
