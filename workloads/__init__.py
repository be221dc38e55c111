"""Seeded synthetic inputs for the RGDBEK solver (shared by tests, bench and
smoke).  Holds no part of the method's arithmetic: only matrices, planted
solutions and right-hand sides shaped like the paper's workloads."""
from .generators import (dense_consistent, dense_least_squares,
                         sparse_powerlaw, sparse_uniform, blur_operator,
                         blur_rhs, blur_tikhonov, smooth_fields,
                         fem_p1_unit_square,
                         laplacian_batch, Problem, to_csr_arrays)

__all__ = ["dense_consistent", "dense_least_squares", "sparse_powerlaw",
           "sparse_uniform", "blur_operator", "blur_rhs", "blur_tikhonov",
           "smooth_fields", "fem_p1_unit_square",
           "laplacian_batch", "Problem", "to_csr_arrays"]
