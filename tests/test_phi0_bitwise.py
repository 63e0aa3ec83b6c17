"""The library's ellipsoid phi0 (its device header, compiled for the host over the HIP
emulation in tests/cpu_hip) equals the oracle's bit for bit on random ellipsoids, rotations
and points: deep inside, near the surface, far out, with equal semi-axes and with body
coordinates exactly 0.  The normals' sign tests decide which data get weight, so the
distance must agree to the last bit; this covers the bisection's step skipping and its
written-out divisions (the emulated reciprocal is exact, so the skipping bounds differ from
the GPU's, but the result may not depend on them)."""
import os
import subprocess

import pytest

from tests.cpu_hip import emu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cpu_hip")
pytestmark = pytest.mark.skipif(not os.path.exists(emu.CLANG), reason="no host clang++")


def test_phi0_bitwise_equal_to_oracle(tmp_path):
    import oracle
    lib = oracle.build(force=False)
    exe = str(tmp_path / "phi0_check")
    subprocess.check_call([emu.CLANG, "-std=c++20", "-O2", "-Wno-unknown-attributes",
                           "-I", HERE, "-I", os.path.join(emu.ROOT, "include"), "-I", emu.CSRC,
                           "-x", "c++", os.path.join(HERE, "phi0_check.cpp"), "-x", "none",
                           lib, "-Wl,-rpath," + os.path.dirname(lib), "-o", exe])
    out = subprocess.run([exe, "400000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "400000 points, 0 mismatches" in out.stdout


def test_blur_weight_certificates_match_the_exact_distance(tmp_path):
    """The blur weight 1 - H_eps(phi0) skips the ellipsoid's bisection where certified
    bounds put the distance at eps or more; on points crowded within 3 eps of the surface
    (eps from 1e-3 to 0.5 of the shortest semi-axis) the weight must equal the one from the
    oracle's exact distance bit for bit."""
    import oracle
    lib = oracle.build(force=False)
    exe = str(tmp_path / "weight_check")
    subprocess.check_call([emu.CLANG, "-std=c++20", "-O2", "-ffp-contract=off",
                           "-Wno-unknown-attributes", "-I", HERE,
                           "-I", os.path.join(emu.ROOT, "include"), "-I", emu.CSRC,
                           "-x", "c++", os.path.join(HERE, "weight_check.cpp"), "-x", "none",
                           lib, "-Wl,-rpath," + os.path.dirname(lib), "-o", exe])
    out = subprocess.run([exe, "400000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "400000 points, 0 mismatches" in out.stdout
