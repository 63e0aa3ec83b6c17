"""The method variants (unequal spacings, periodic axes) through the library built for the
CPU over the host emulation of HIP, under AddressSanitizer and UndefinedBehaviorSanitizer,
against the oracle: the extrapolation in several launch forms, a time step and the
blur-zone consumers on a periodic box with unequal spacings whose boxes cross the periodic
ends, a normal-weighted radius-4 fit with unequal spacings (the gather from global memory),
and the truncation of a band that reaches a box face on a periodic axis.  Test
infrastructure only."""
import copy
import os
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2104_00095_amd import rmx, synth
from tests.helpers import (BlurCase, StepCase, compare_blur, compare_step, plates_workload,
                           rel_err, run_oracle, wall_sphere)

emu = pytest.importorskip("tests.cpu_hip.emu")
pytestmark = pytest.mark.skipif(not os.path.exists(emu.CLANG), reason="no host clang++")

TOL = {0: 1e-12, 1: 1e-5}
BATCHED, PER_SOLID, GRAPH, PERSISTENT, ADJ26 = 0, 4, 2, 16, 32


def _plates_aniso():
    w, xn = plates_workload()
    w.spacing = (1.0, 1.7, 0.6)
    return w, xn


def _wall_periodic():
    w = wall_sphere(24, n_layers=4)
    w.periodic = (0, 0, 1)
    return w


def _runs():
    box = synth.periodic_box()
    plates, xn = _plates_aniso()
    return {
        "box": (box, 0, BATCHED, {}),
        "box_fp32_graph": (box, 1, GRAPH, {}),
        "box_persistent": (box, 0, PERSISTENT, {}),
        "box_adj26_per_solid": (box, 0, ADJ26 | PER_SOLID, {"adjacency": 26}),
        "plates_aniso": (plates, 0, BATCHED, {"xi_normal": [xn]}),
        "wall_periodic": (_wall_periodic(), 0, BATCHED, {}),
    }


@pytest.fixture(scope="module")
def emulated():
    emu.build()
    root = tempfile.mkdtemp(prefix="rmx_emu_var_")

    def one(item):
        name, (w, prec, flags, o) = item
        st, outs = emu.run(w, os.path.join(root, name), precision=prec, flags=flags,
                           xi_normal=o.get("xi_normal"))
        return name, (w, prec, st, outs, o)

    with ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(one, _runs().items()))


def _check(w, outs, precision, o):
    xn = o.get("xi_normal")
    for i, ((xo, lab, dec, _), s) in enumerate(zip(outs, w.solids)):
        st, xr, lr, dr, _ = run_oracle(w, s, xi_normal=None if xn is None else xn[i],
                                       adjacency=o.get("adjacency", 6))
        assert np.array_equal(lab, lr)
        if st == 0:
            assert np.array_equal(dec, dr)
            assert rel_err(xo, xr, lr > 0) <= TOL[precision]
        keep = lr <= 0 if st == 0 else np.ones(lr.shape, bool)
        assert np.array_equal(xo[:, keep].view(np.uint64), s.xi[:, keep].view(np.uint64))


@pytest.mark.parametrize("name", ["box", "box_fp32_graph", "box_persistent",
                                  "box_adj26_per_solid", "plates_aniso"])
def test_emulated_variants_match_oracle(emulated, name):
    w, prec, st, outs, o = emulated[name]
    assert st == 0
    _check(w, outs, prec, o)


def test_emulated_grown_normal_fit_with_unequal_spacings(emulated):
    w, prec, st, outs, o = emulated["plates_aniso"]
    dec = outs[0][2]
    assert np.all(dec[:, :, [3, 5, 6]] == 32) and dec[4, 4, 8] == 4


def test_emulated_band_truncated_at_a_periodic_face(emulated):
    """The wall z = 0 that stops the band is gone on a periodic z axis: truncated."""
    w, prec, st, outs, o = emulated["wall_periodic"]
    assert st == rmx.E_TRUNCATED
    _check(w, outs, prec, o)


# ---- a time step and the blur-zone consumers ---------------------------------------------

@pytest.fixture(scope="module")
def stepped():
    emu.build()
    w = synth.periodic_box(n_solids=4)
    case = StepCase(w)
    d = tempfile.mkdtemp(prefix="rmx_emu_var_step_")
    st, outs = emu.run_step(w, d, case.xi_n, case.labels_n, [v.u for v in case.vel],
                            [v.uf for v in case.vel], case.dt, case.next_init, case.half_init)
    got = [(rmx.SolidStats.from_buffer_copy(raw).status, xo, lab, dec, half)
           for xo, lab, dec, raw, half in outs]
    return case, st, got


def test_emulated_step_on_the_periodic_box(stepped):
    case, st, got = stepped
    expect = [(o[0], o[1], o[2], o[3], o[5]) for o in case.oracle()]
    assert st == min([e[0] for e in expect] + [0]) == 0
    compare_step(case, got, expect, tag="periodic_box")


def test_emulated_blur_on_the_periodic_box():
    emu.build()
    case = BlurCase(synth.periodic_box())
    d = tempfile.mkdtemp(prefix="rmx_emu_var_blur_")
    st, H, phis, taus = emu.run_blur(case.w, d, case.xi, case.labels, case.eps, case.G,
                                     case.H_init, case.phi_init, case.tau_init)
    assert st == 0
    eH, ephi, etau = case.oracle()
    compare_blur(case, (H, phis, taus), (eH, ephi, etau), tag="periodic_box")
    # the fields do cross the periodic ends
    n0, n1, n2 = case.w.grid_n
    assert (eH[:, :, 0] != case.H_init[:, :, 0]).any() and \
        (eH[:, :, n0 - 1] != case.H_init[:, :, n0 - 1]).any()
    assert (etau[2][:, 0] != 7.0).any()
