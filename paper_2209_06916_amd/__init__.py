"""MI355X-native MGRIT for method-of-lines discretizations of periodic linear
advection (arXiv 2209.06916).  The compute path is libmgrit.so (HIP, gfx950)
behind the C ABI in include/mgrit.h; ``mgrit`` is its ctypes binding and
``inputs`` draws the seeded synthetic workloads."""
