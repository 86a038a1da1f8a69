"""MI355X-native NSGA-III environmental selection.

The product is the C-ABI library ``libnsga3.so`` (hand-written HIP kernels for
gfx950, declared in ``include/nsga3.h``). ``nsga3`` is its thin Python binding
(argument marshalling only); ``workloads`` holds the seeded synthetic input
generators. Importing this package loads nothing; the binding loads the
library on first use and raises if it has not been built.
"""
__all__ = ["nsga3", "workloads"]
