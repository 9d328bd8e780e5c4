"""MI355X-native staggered-grid stencil kernels (advec_u, diff_uvw) with an
autotuner, wisdom files, a batched graph launch and a request server.

The GPU library is ``libkl.so`` (HIP, gfx950) behind the C-ABI declared in
``include/kl.h``; :mod:`paper_2303_12374_amd.kl` is its Python binding.
Importing this package loads nothing; import ``.kl`` for the binding and
``.inputs`` for the seeded input generators.
"""
__all__ = ["kl", "inputs"]
