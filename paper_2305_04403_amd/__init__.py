"""MI355X-native walk-on-boundary (WoB) Monte Carlo solver for Laplace boundary
value problems (Sugimoto et al., "A Practical Walk-on-Boundary Method for
Boundary Value Problems").

The compute path is a C-ABI HIP library (``libwob.so``, built for gfx950); the
Python side only marshals device pointers and streams.  Import
``paper_2305_04403_amd.wob`` for the binding; importing this package itself
loads nothing.
"""
__all__ = ["wob", "inputs"]
