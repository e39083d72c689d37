"""MI355X-native hot path of Nonequilibrium Monte Carlo (arXiv 2111.13628).

Replica-parallel Metropolis sweeps over k-SAT factor graphs and QAP
permutations with per-class inverse temperatures, cross-replica backbone
estimates and nonequilibrium re-anneals, as HIP kernels for gfx950 behind
the C ABI of include/nmc.h.  ``nmc`` is the ctypes binding (import it
explicitly: it needs the built libnmc.so), ``instances`` the seeded input
generators, ``build`` the gfx950 build of the library.
"""
from . import instances  # noqa: F401

__all__ = ["instances"]
