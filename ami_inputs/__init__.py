"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package draws random numbers and builds integer labels; it holds none of
the arithmetic of algorithmic Matsubara integration (no residues, no Fermi or
Bose functions, no dispersion).  Both the oracle and the device path receive
exactly the same arrays from here, so the two can be compared bit for bit.

* :mod:`ami_inputs.diagrams` -- self-energy topologies of a Hubbard-type model
  (local interaction lines) and their momentum/frequency labels
  ``alpha`` / ``epsilon`` (Sec. 2.2, Eq. (2) and the labelling of Sec. 2.5).
* :mod:`ami_inputs.samples` -- momentum samples, uniform energies and external
  frequency grids (Sec. 5.1.3 and Sec. 5.2).
"""
from .diagrams import (Diagram, order2_example, random_self_energy,  # noqa: F401
                       diagram_set, relabel)
from .samples import (k_samples, uniform_energies, complex_energies,  # noqa: F401
                      matsubara_freqs, real_freqs, DEFAULT_Q)
