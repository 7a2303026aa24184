"""Scoring and search constants of the oracle.

The paper names the terms of the score (a grid "reaction field" for the receptor,
and hydrogen bonding, van der Waals and desolvation among ligand atoms) but gives
no formula or constant.  The values below are the published AutoDock4 force-field
forms and weights that the paper's AutoDock-GPU lineage uses, taken as free
constants of this implementation:

  van der Waals 12-6, hydrogen bond 12-10, Coulomb with the Mehler-Solmajer
  distance-dependent dielectric, Gaussian desolvation, and the four term weights.
"""
import math

# term weights (AutoDock4 free-energy coefficients)
W_VDW = 0.1662
W_HB = 0.1209
W_EL = 0.1406
W_DS = 0.1322

COULOMB = 332.06363            # kcal*A/(mol*e^2)

# Mehler-Solmajer sigmoidal dielectric eps(r) = A + B / (1 + k exp(-lambda*B*r))
DIEL_A = -8.5525
DIEL_B = 78.4 - DIEL_A
DIEL_LAMBDA = 0.003627
DIEL_K = 7.7839

DESOLV_SIGMA = 3.6             # Angstrom
QASP = 0.01097                 # charge-dependent part of the solvation parameter

R_MIN = 0.5                    # distances are clamped below this (zero gradient there)
CUTOFF = 8.0                   # vdW / H-bond / desolvation cutoff (Angstrom)
CUTOFF_EL = 20.48              # electrostatics cutoff (Angstrom)

# energy of an atom outside the grid box: P_OUT + K_OUT * d^2
P_OUT = float(2 ** 14)
K_OUT = 100.0

HB_NONE, HB_DONOR, HB_ACCEPTOR = 0, 1, 2
N_TYPES = 7

TWO_PI = 2.0 * math.pi
