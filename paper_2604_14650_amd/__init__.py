"""MI355X-native batched IPv6 longest-prefix-match lookup (PlanB's linearized
B+-tree over elementary intervals).

The product is the C-ABI library ``libplanb.so`` (include/planb.h); the
``planb`` submodule is its ctypes binding.  Importing this package does not
load the library; ``from paper_2604_14650_amd import planb`` does, and fails
loudly if it has not been built.
"""
__all__ = ["planb"]
