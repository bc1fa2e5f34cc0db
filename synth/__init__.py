"""Seeded synthetic inputs for the TU-fRG flow right-hand side.

This package is shared by the FP64 oracle, the tests and the benchmark.  It
holds only *inputs*: hopping tables of the model Hamiltonians, the initial
(onsite) interaction tensors, the plane-wave form-factor shells, chemical
potentials fixed by a target filling, and seeded random probe states.  None of
the flow arithmetic (loops, projections, bundle products, integration) lives
here, and nothing here imports the oracle or the HIP library.
"""

from .models import (  # noqa: F401
    PAULI,
    ff_shell,
    hubbard_hoppings,
    rashba_hoppings,
    t2g_soc_hoppings,
    onsite_V0,
    kanamori_V0,
    density_density_c0,
    chemical_potential,
    random_exchange_state,
    random_unitaries,
    mlp_shape,
    mlp_init,
    mlp_batch,
    probe_vector,
)
from .workloads import workload, WORKLOADS  # noqa: F401
