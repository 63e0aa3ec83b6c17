"""MI355X-native reference-map extrapolation (layer-wise weighted least squares).

The compute path is the HIP library ``librmx.so`` built from ``csrc/``;
``paper_2104_00095_amd.rmx`` is its thin ctypes binding and
``paper_2104_00095_amd.synth`` holds the seeded input generators.  Import the submodule
you need; importing the package itself loads nothing.
"""
