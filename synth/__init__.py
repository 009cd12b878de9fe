"""Seeded synthetic inputs for the rid Davidson solver.

This package is shared by the FP64 CPU oracle and by the GPU library's
tests and benchmark.  It draws random numbers and shapes them into the
inputs of a TDDFT response problem (orbital energies, RI three-index
tensors, a minimal-auxiliary ris tensor, dipole right-hand sides).  It holds
none of the solver's arithmetic: no operator products, no Krylov steps.
"""

from .generate import (  # noqa: F401
    HARTREE_PER_EV,
    TCUT_HA_DEFAULT,
    Problem,
    counter_normals,
    counter_uniforms,
    make_problem,
    make_dipoles,
    make_block,
    config_sizes,
    molecule_sizes,
    batch_member,
    serve_trace,
    related_problem,
)
from .molecule import Molecule, make_molecule  # noqa: F401,E402
