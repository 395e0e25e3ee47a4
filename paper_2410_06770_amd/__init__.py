"""MI355X-native xGETT: binary tensor contraction on gfx950.

The compute path is the C-ABI library ``libgett.so`` (hand-written HIP
kernels); :mod:`paper_2410_06770_amd.gett` is its thin ctypes binding.
"""
