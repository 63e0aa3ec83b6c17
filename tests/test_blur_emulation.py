"""The blur-zone consumers (rmx_blur, rmx_solid_stress) of the library built for the CPU
over the host emulation of HIP, under AddressSanitizer and UndefinedBehaviorSanitizer,
against the oracle: main text eq. (sm_heavi), SI "Stress calculations" and
eq. (mod_heaviside).  Test infrastructure only."""
import os
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2104_00095_amd import synth
from tests.helpers import BlurCase, blur_pair_workload, compare_blur

emu = pytest.importorskip("tests.cpu_hip.emu")
pytestmark = pytest.mark.skipif(not os.path.exists(emu.CLANG), reason="no host clang++")


def _cases():
    return {
        "sphere24": BlurCase(synth.sphere32(n=24, n_layers=6)),
        "pair": BlurCase(blur_pair_workload(n=32)),
        "suspension3": BlurCase(synth.suspension(n_solids=3, grid_n=(40, 40, 56), h=1.0 / 40,
                                                 n_layers=6)),
    }


@pytest.fixture(scope="module")
def blurred():
    emu.build()
    root = tempfile.mkdtemp(prefix="rmx_emu_blur_")

    def one(item):
        name, c = item
        d = os.path.join(root, name)
        st, H, phis, taus = emu.run_blur(c.w, d, c.xi, c.labels, c.eps, c.G, c.H_init,
                                         c.phi_init, c.tau_init)
        return name, (c, st, (H, phis, taus), emu.read_h_without_phi(d, H))

    with ThreadPoolExecutor(max_workers=3) as ex:
        return dict(ex.map(one, _cases().items()))


@pytest.mark.parametrize("name", ["sphere24", "pair", "suspension3"])
def test_emulated_blur_matches_oracle(blurred, name):
    c, st, got, _ = blurred[name]
    assert st == 0
    compare_blur(c, got, c.oracle(), tag=name)


@pytest.mark.parametrize("name", ["sphere24", "pair", "suspension3"])
def test_emulated_heaviside_without_phi_is_the_same(blurred, name):
    """Without phi outputs the kernel weighs ellipsoids through the certified distance
    bounds where they decide H_eps: H must not change by a bit."""
    c, st, got, h2 = blurred[name]
    assert np.array_equal(h2.view(np.uint64), got[0].view(np.uint64))
