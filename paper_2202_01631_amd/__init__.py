"""MI355X-native lattice update of the multiphase-multicomponent lattice
Boltzmann model for self-diffusiophoretic Janus colloids at liquid-liquid
interfaces (Palacios, Scagliarini, Pagonabarraga, arXiv:2202.01631).

The solver is the HIP library ``csrc/liblbphoretic.so`` behind the C ABI in
``include/lb.h``; ``lb`` is its Python binding.  Importing this package does
not load the library; ``lb.load()`` does, and fails loudly when it is absent.
"""
__all__ = ["inputs", "lb", "serve", "tune"]
