"""FP64 CPU oracle of the difference-free conservative phase-field LBM step.

TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and
this package imports nothing from it. The C source follows the paper
(Zhao, Patel & Lee, arXiv 2407.12263) step by step; see ``cpf_oracle.c``.
"""
from .oracle import (Oracle, OracleParams, build, lattice, node_equilibria, node_macro,
                     propagate, fd_gradient, num_threads, set_num_threads, DIAG_NAMES)

__all__ = ["Oracle", "OracleParams", "build", "lattice", "node_equilibria", "node_macro",
           "propagate", "fd_gradient", "num_threads", "set_num_threads", "DIAG_NAMES"]
