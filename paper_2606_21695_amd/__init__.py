"""MI355X (gfx950) block-level domain decomposition with WaveHoltz
subdomain solves for the 2D Helmholtz equation.

The compute path is the HIP library ``libwavedd.so`` (C ABI in
``include/wavedd.h``); ``wavedd`` is its ctypes binding.
"""
