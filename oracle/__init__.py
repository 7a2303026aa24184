"""FP64 CPU oracle for the docking hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, readable NumPy code that states what the GPU path must compute:
genotype -> pose, grid (intermolecular) energy, intramolecular pair energy, the
analytic genotype gradient, the ADADELTA and Solis-Wets local searches and the
Lamarckian genetic algorithm.  Only the test suite, the smoke check and the benchmark's CPU baseline
may import it.  The product library never calls it and shares no code with it.

Where the paper (Background, "Design and Structure of MiniMDock") only names a
part of the method, the functional form is the AutoDock4 lineage the paper builds
on (its references on AutoDock-GPU and on gradient-based local search in
AutoDock4); each such reading is listed with its constant values in `constants`.

Pins: every function here is checked by `tests/test_oracle_*.py` against closed
forms, library routines (scipy interpolation and rotations, torch's Adadelta),
invariances, finite differences or brute force; the LGA on 1-3-atom ligands against
exact lower bounds and a brute-force lattice minimum, its initial-population sampler
by distribution tests.  The GA operator choices beyond those and its invariants are
"parity unpinned" (see `lga`), and so are the Solis-Wets step parameters (the paper
gives none; `solis_wets` is pinned on hand-worked trajectories, its update rules, its
budget and closed-form minima).
"""
from . import constants, rng, ligand, pose, scoring, adadelta, solis_wets, lga  # noqa: F401
