"""MI355X-native WCSPH hot path (neighbour search + pair sums) of the Nauticle
particle method, behind the C-ABI library ``libnauticle.so``.

Importing the package loads nothing; ``paper_1710_08259_amd.nauticle`` loads
the HIP library on first use and raises if it is missing.
"""
