"""The method variants on the GPU through the C ABI against the oracle: unequal spacings
(SI "Variable arrangement": the normal factor of eq. (weight) in physical offsets, the
predictor with dt / Delta per axis, the face stress with per-axis differences) and periodic
axes (SI "Test cases": boxes across the periodic ends, no walls there), in the launch
forms of the extrapolation, a time step and the blur-zone consumers.  Same bars as the
other parity tests: labels, decisions and counts equal, xi within the precision's
tolerance, predicted cells and phi bit for bit."""
import numpy as np
import pytest

from paper_2104_00095_amd import synth
from tests.helpers import BlurCase, StepCase, compare_blur, compare_step, plates_workload, \
    wall_sphere
from tests.test_gpu_blur import gpu_blur
from tests.test_gpu_parity import compare, run_gpu
from tests.test_gpu_step import gpu_step

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}
FORMS = {"batched": 0, "per_solid": 4, "graph": 2, "persistent": 16}


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_00095_amd import rmx
    c = rmx.Context(0)
    yield c
    c.close()


def big_box():
    """Twice the small box's cells per axis, twelve solids."""
    return synth.periodic_box(seed=8, grid_n=(96, 80, 112),
                              spacing=(1.0 / 96, 1.0 / 64, 1.0 / 128), n_solids=12,
                              semi_lo=0.05, semi_hi=0.09)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("form", sorted(FORMS))
def test_periodic_box_matches_oracle(ctx, form, precision):
    w = synth.periodic_box()
    st, gpu = run_gpu(ctx, w, precision=precision, flags=FORMS[form])
    assert st == 0
    compare(w, gpu, precision, tag=f"box/{form}/{precision}")


def test_big_periodic_box_matches_oracle(ctx):
    w = big_box()
    assert any(s.lo[a] + s.ext[a] > w.grid_n[a] for s in w.solids for a in (0, 2))
    st, gpu = run_gpu(ctx, w)
    assert st == 0
    compare(w, gpu, 0, tag="big_box")


def test_periodic_box_cube_layers(ctx):
    w = synth.periodic_box()
    st, gpu = run_gpu(ctx, w, flags=32)
    assert st == 0
    compare(w, gpu, 0, tag="box/adj26", adjacency=26)


@pytest.mark.parametrize("precision", [0, 1])
def test_grown_normal_fit_with_unequal_spacings(ctx, precision):
    """F1 and a normal-weighted radius-4 fit (the gather from global memory) with the
    spacings (1, 1.7, 0.6)."""
    w, xn = plates_workload()
    w.spacing = (1.0, 1.7, 0.6)
    st, gpu = run_gpu(ctx, w, precision=precision, xi_normal=[xn])
    assert st == 0
    compare(w, gpu, precision, xi_normal=[xn], tag="plates_aniso")
    dec = gpu[0][2]
    assert np.all(dec[:, :, [3, 5, 6]] == 32) and dec[4, 4, 8] == 4


def test_band_truncated_at_a_periodic_face(ctx):
    from paper_2104_00095_amd import rmx
    w = wall_sphere(32, n_layers=4)
    st, gpu = run_gpu(ctx, w)
    assert st == 0                   # z = 0 is a wall: the band stops there
    w.periodic = (0, 0, 1)
    st, gpu = run_gpu(ctx, w)
    assert st == rmx.E_TRUNCATED     # no wall on a periodic axis
    compare(w, gpu, 0, tag="wall_periodic")


@pytest.mark.parametrize("precision", [0, 1])
def test_step_on_the_periodic_box(ctx, precision):
    case = StepCase(synth.periodic_box())
    expect = [(o[0], o[1], o[2], o[3], o[5]) for o in case.oracle()]
    st, got = gpu_step(ctx, case, precision)
    assert st == 0 and all(e[0] == 0 for e in expect)
    compare_step(case, got, expect, tol=TOL[precision], tag=f"box/{precision}")


def test_step_on_the_big_periodic_box(ctx):
    case = StepCase(big_box())
    expect = [(o[0], o[1], o[2], o[3], o[5]) for o in case.oracle()]
    st, got = gpu_step(ctx, case)
    assert st == 0
    compare_step(case, got, expect, tag="big_box")


@pytest.mark.parametrize("name", ["box", "big_box"])
def test_blur_on_the_periodic_box(ctx, name):
    case = BlurCase(synth.periodic_box() if name == "box" else big_box())
    got = gpu_blur(ctx, case)
    compare_blur(case, got, case.oracle(), tag=name)
