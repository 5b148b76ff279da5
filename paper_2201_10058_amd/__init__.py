"""MI355X-native changeover-weighted N-body kick (GENGA II hot path).

The compute path is the HIP library libgenga.so (C ABI, include/genga.h);
`native` is its thin Python binding.  `workload` builds seeded synthetic
inputs.
"""
__all__ = ["workload", "native"]
