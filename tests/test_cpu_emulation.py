"""The library's HIP kernels, host core included, built for the CPU over a host emulation
of the HIP subset they use (tests/cpu_hip) and run under AddressSanitizer and
UndefinedBehaviorSanitizer on tiny workloads.  Labels and decisions must equal the
oracle's and xi must meet the GPU tolerance.  Thread blocks are host threads; the
persistent launch runs several blocks concurrently, so its per-slab waits are exercised
in earnest.  Test infrastructure only: the product library never contains this build.
"""
import os

import numpy as np
import pytest

from paper_2104_00095_amd import synth
from tests.helpers import rel_err, run_oracle

emu = pytest.importorskip("tests.cpu_hip.emu")
pytestmark = pytest.mark.skipif(not os.path.exists(emu.CLANG), reason="no host clang++")

TOL = {0: 1e-12, 1: 1e-5}
CHAIN, PER_SOLID, PERSISTENT = 0, 4, 16


def _cases():
    return {
        "sphere16": synth.sphere32(n=16, n_layers=3),
        "ellipsoid24": synth.ellipsoid128(n=24, n_layers=3),
        "suspension3": synth.suspension(n_solids=3, grid_n=(24, 24, 40), h=1 / 24),
    }


@pytest.fixture(scope="module")
def built():
    return emu.build()


def _check(w, outs, precision, **kw):
    for (xo, lab, dec, _), s in zip(outs, w.solids):
        st, xr, lr, dr, _ = run_oracle(w, s, **kw)
        assert np.array_equal(lab, lr)
        if st == 0:
            assert np.array_equal(dec, dr)
            assert rel_err(xo, xr, lr > 0) <= TOL[precision]
        keep = lr <= 0 if st == 0 else np.ones(lr.shape, bool)
        assert np.array_equal(xo[:, keep].view(np.uint64), s.xi[:, keep].view(np.uint64))


@pytest.mark.parametrize("flags,blocks", [(CHAIN, 1), (PER_SOLID, 1), (PERSISTENT, 1),
                                          (PERSISTENT, 5)])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", ["sphere16", "ellipsoid24", "suspension3"])
def test_emulated_kernels_match_oracle(built, tmp_path, case, precision, flags, blocks):
    if precision == 1 and case != "suspension3":
        pytest.skip("FP32 accumulation: one multi-solid case suffices")
    w = _cases()[case]
    st, outs = emu.run(w, str(tmp_path), precision=precision, flags=flags, blocks=blocks)
    assert st == 0
    _check(w, outs, precision)


def test_emulated_persistent_after_chain_calls(built, tmp_path):
    """Persistent launches interleaved with chain calls on one context (shared workspace;
    each call on a fresh copy of the field): the counters must come back to zero after
    every persistent launch for the last one to be right."""
    w = _cases()["sphere16"]
    st, outs = emu.run(w, str(tmp_path), flags=PERSISTENT, blocks=4,
                       pre_flags=(CHAIN, PERSISTENT, CHAIN, PERSISTENT))
    assert st == 0
    _check(w, outs, 0)


def test_emulated_statuses(built, tmp_path):
    """Truncated band, no interior cell and L = 0 in one batch, both launch forms."""
    w0 = synth.sphere32(n=24, n_layers=3)
    s = w0.solids[0]
    w = synth.Workload("statuses", w0.grid_n, w0.h, w0.origin)
    w.solids.append(synth.Solid((8, 4, 4), (10, 16, 16), s.shape, 3,
                                s.xi[:, 4:20, 4:20, 8:18].copy()))
    w.solids.append(synth.Solid(s.lo, s.ext, s.shape, 3, s.xi + 10.0))
    w.solids.append(synth.Solid(s.lo, s.ext, s.shape, 0, s.xi.copy()))
    w.solids.append(synth.Solid(s.lo, s.ext, s.shape, 3, s.xi.copy()))
    for flags, blocks in ((CHAIN, 1), (PERSISTENT, 3)):
        st, outs = emu.run(w, str(tmp_path), flags=flags, blocks=blocks)
        assert st == -7
        _check(w, outs, 0)

