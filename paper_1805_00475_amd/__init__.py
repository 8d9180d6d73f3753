"""Exact #CSP counting by tensor-network contraction on MI355X (gfx950).

The library (``libtn.so``, C ABI in ``include/tn.h``) builds the network of
a formula, orders its pairwise contractions on the host and runs them in
HIP kernels; ``tn`` is its ctypes binding.
"""
