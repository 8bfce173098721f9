"""MI355X-native hot path of the regularized colour-gradient lattice Boltzmann
model for direct-writing printing (arXiv:2102.02655).

The compute path is the HIP library ``liblbprint.so`` (built from ``csrc/``)
behind the C ABI of ``include/lbprint.h``; ``lbprint`` is its Python binding.
Importing this package loads nothing; ``workloads`` holds the seeded set-ups.
"""
