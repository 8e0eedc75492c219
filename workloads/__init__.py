"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This package holds no arithmetic of the method (no t-products, transforms,
norms or sampling): it only draws the raw random arrays each workload is made
of, from NumPy's PCG64 seeded per workload. Where a workload is a t-product of
factors (the low-tubal-rank tensors), the factors are returned and each side
composes them with its own t-product.
"""
from .generators import *  # noqa: F401,F403
