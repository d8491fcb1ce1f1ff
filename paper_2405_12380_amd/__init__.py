"""MI355X-native DeepONet meta-solvers for Helmholtz scattering (arXiv 2405.12380).

The numerical path lives in ``libhelm.so`` (hand-written HIP for gfx950,
C ABI in ``include/helm.h``); :mod:`.helm` is its thin Python binding and
:mod:`.inputs` generates seeded synthetic workloads.  Import the binding
explicitly (``from paper_2405_12380_amd import helm``): it loads torch and
the compiled library and raises if the library has not been built.
"""
__all__ = ["helm", "inputs", "build"]
