"""MI355X-native Monte Carlo Shiftable Filter (fast vector-valued bilateral
filter of Ghosh & Chaudhury, arXiv 1605.02164).

The product is the C-ABI library ``libbfvec.so`` (header ``include/bfvec.h``)
built from ``csrc/`` by ``build.py``; ``bfvec`` is its ctypes binding.
"""

from .bfvec import (  # noqa: F401
    bf_vec, bf_vec_ex, bf_vec_static, bf_vec_terms, bf_whiten, bf_sample_terms, bf_choose_N,
    bf_minmax, bf_direct, bf_autotune, bf_ubench, BfError, Server, Plan, lib, version, EXPORTS,
)
