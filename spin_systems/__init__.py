"""Seeded synthetic inputs: crystal lattices, CSR neighbour lists, materials
and the workload recipes used by tests and benchmarks.  No spin dynamics."""
from .lattice import Lattice, simple_cubic, sc_long_range, bcc, fcc_sphere, fcc_ellipsoid, csr_from_padded  # noqa: F401
from .workloads import (  # noqa: F401
    MU_B, GAMMA, Workload, sc_reference, bcc_film, fcc_nanoparticle, bcc_block,
    serving_requests, sc_request_system, single_spin, dmi_matrix, with_tensor_exchange, with_demag, long_range_sc,
)
