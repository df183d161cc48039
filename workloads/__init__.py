"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds the Darcy matrix generator and the host graph partitioner only; none of
the preconditioner's arithmetic lives here.
"""
from .darcy import CSR, tpfa_matrix, rhs_from_source, gaussian_random_field  # noqa: F401
from .partition import partition, partition_hash  # noqa: F401
from .configs import Workload, get  # noqa: F401
