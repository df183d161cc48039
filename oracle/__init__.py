"""CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Importable only from tests/, the smoke check and the benchmark's CPU-baseline
leg.  The HIP product path never imports or calls anything here.
"""
from .amsp_oracle import (  # noqa: F401
    OracleError, validate, cores, grow, multiplicity, local_matrix, neumann_matrix,
    weighting, local_eigenpairs, prolongation, coarse_matrix, Setup, setup, apply,
    local_part, coarse_part, pcg, PCGResult, lanczos_condition, adjoint_gradients,
    gmres, GMRESResult, pseudo_inverse, apply_multiplicative, theta_gradient,
)
