"""MI355X-native Montgomery modular arithmetic and NTT polynomial products.

Submodules: ``mont`` (elementwise Montgomery operations), ``ntt`` (transforms
and polynomial products), ``workloads`` (seeded synthetic inputs), ``build``
(hipcc build of libmont.so).  Importing the package loads nothing; the HIP
library is loaded on first use and its absence is an error.
"""
__all__ = ["mont", "ntt", "workloads", "build"]
