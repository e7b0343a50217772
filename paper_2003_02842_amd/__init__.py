"""MI355X (gfx950) Malliavin-Mancino covariance estimation via type-1 NUFFT.

The computation lives in ``libmm.so`` (C ABI in ``include/mm.h``); the ``mm``
submodule is its thin PyTorch binding and ``synth`` the seeded workload generator.
"""
