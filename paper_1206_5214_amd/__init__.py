"""MI355X-native red/black Moebius domain-wall operator and CG solver.

The compute path is the HIP library ``libmobius.so`` (built from ``csrc/``)
behind a C ABI; ``mobius`` is its thin Python binding.  ``inputs`` draws the
seeded synthetic gauge fields and sources.
"""
__all__ = ["inputs"]
