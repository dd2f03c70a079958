"""MI355X (gfx950) implementation of the fluctuating lattice Boltzmann
method for Oldroyd-B viscoelastic flows (arXiv 2506.13072).

The hot path lives in ``libvflb.so`` (HIP kernels behind the C ABI of
``include/vflb.h``); :mod:`paper_2506_13072_amd.vflb` is its Python binding.
"""
