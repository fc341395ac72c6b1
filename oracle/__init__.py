"""CPU FP64 oracle for the closed-shell (T) correction.

TEST INFRASTRUCTURE ONLY: this package is the yardstick the device library is
measured against. Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the library itself never imports, links or calls it,
and the two share no code. Inputs come from the seeded generators only.

closed_shell  -- the paper's Eqs. 1-6 written out plainly (numpy, FP64)
spin_orbital  -- the textbook spin-orbital (T) by brute force (tiny sizes)
"""
from . import closed_shell, spin_orbital  # noqa: F401
from .closed_shell import (DFIntegrals, ExplicitIntegrals, energy, energy_all_form,  # noqa: F401
                           energy_eq1_form, integrals_from_df, triple_energy, triples)
from .spin_orbital import mo_eri_from_df, so_energy  # noqa: F401
