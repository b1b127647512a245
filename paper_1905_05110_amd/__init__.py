"""MI355X-native volume-penalization lattice-Boltzmann hot path (Liberge & Beghein,
arXiv 1905.05110): HIP kernels behind the C ABI of include/vplbm.h.

Submodules: ``vplbm`` (ctypes binding, loads libvplbm.so), ``workloads`` (synthetic
workloads), ``build`` (hipcc build).  Importing the package loads nothing.
"""
