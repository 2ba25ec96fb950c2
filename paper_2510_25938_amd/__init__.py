"""MI355X-native batched Lennard-Jones minimiser for adaptive, parallel Basin Hopping.

The compute path is the HIP library liblj_bh.so (C ABI declared in
include/lj_bh.h); `paper_2510_25938_amd.lj` is its thin ctypes binding.
"""
__all__ = ["lj", "inputs"]
