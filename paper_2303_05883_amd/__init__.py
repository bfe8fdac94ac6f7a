"""MI355X (gfx950) even-odd Wilson/clover operator and BiCGStab solvers.

The compute path is the HIP library ``liblqcd.so`` behind the C ABI in
``include/lqcd.h``; ``paper_2303_05883_amd.lqcd`` is its ctypes binding.
"""

__all__ = ["lqcd"]
