"""MI355X-native (HIP/gfx950) hot path of the synthetic iterative scheme for the
linearized Boltzmann equation (arXiv:1612.04488).

The compute path is libsis.so (C ABI in include/sis.h); `sis` is its ctypes
binding, `inputs` holds the seeded synthetic workloads, `build` compiles the
library in-tree.
"""
