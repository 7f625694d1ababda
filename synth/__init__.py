"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package draws random numbers and lays out arrays; it holds none of the
TensorNet arithmetic (no geometry, basis, cutoff, tensor algebra or network
evaluation).  Both the FP64 oracle and the HIP path consume what it produces,
and neither of them is imported here.
"""

from .generators import (  # noqa: F401
    DENSITY,
    DMIN,
    MASS_BY_Z,
    SPECIES,
    CONFIGS,
    make_config,
    make_weights,
    maxwell_boltzmann,
    periodic_box,
    random_cloud,
    molecule_batch,
    single_molecule,
)
from .blob import BLOB_MAGIC, BLOB_VERSION, tensor_layout, write_blob  # noqa: F401
