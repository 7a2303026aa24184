"""ADADELTA local search on the genotype (oracle).

The paper's docking search is memetic: a local optimisation is applied to a
sample of each generation and its gains are written back (Background, "Design and
Structure of MiniMDock").  The local optimiser here is the gradient-based one of
the AutoDock4 GPU line the paper cites ("Accelerating AutoDock4 with GPUs and
gradient-based local search"): ADADELTA (Zeiler 2012, Algorithm 1) with learning
rate 1, decay rho and conditioning constant eps:

  E[g^2]  <- rho E[g^2]  + (1 - rho) g^2
  dx      =  - sqrt(E[dx^2] + eps) / sqrt(E[g^2] + eps) * g
  E[dx^2] <- rho E[dx^2] + (1 - rho) dx^2
  x       <- x + dx

Readings taken here: both running averages start at zero and are never reset;
after every step the quaternion genes are renormalised to unit length and the
torsion genes wrapped to (-pi, pi]; the search evaluates energy and gradient once
per step, keeps the best pose seen (strictly lower energy wins, so the earliest of
equal energies is kept) and returns it.  S steps cost S evaluations.
"""
from __future__ import annotations

import numpy as np

from .pose import wrap_angle
from .scoring import energy_and_gradient


def adadelta_step(x, g, eg2, edx2, rho, eps):
    """One ADADELTA update of the parameter vector (no renormalisation)."""
    eg2 = rho * eg2 + (1.0 - rho) * g * g
    dx = -np.sqrt(edx2 + eps) / np.sqrt(eg2 + eps) * g
    edx2 = rho * edx2 + (1.0 - rho) * dx * dx
    return x + dx, eg2, edx2


def project_genes(x, n_torsions):
    """Unit quaternion and wrapped torsions after a step."""
    x = x.copy()
    x[3:7] /= np.linalg.norm(x[3:7])
    for k in range(n_torsions):
        x[7 + k] = wrap_angle(x[7 + k])
    return x


def local_search(grid, lig, genes0, iters=300, rho=0.8, eps=1e-2, trace=False):
    """Returns (best_genes, best_energy[, trajectory of (energy, genes) per step])."""
    x = np.asarray(genes0, dtype=np.float64).copy()
    eg2 = np.zeros_like(x)
    edx2 = np.zeros_like(x)
    best_x, best_e = x.copy(), np.inf
    traj = []
    for _ in range(iters):
        res = energy_and_gradient(grid, lig, x, want_margin=False)
        if trace:
            traj.append((res.energy, x.copy()))
        if res.energy < best_e:
            best_e, best_x = res.energy, x.copy()
        x, eg2, edx2 = adadelta_step(x, res.grad, eg2, edx2, rho, eps)
        x = project_genes(x, lig.n_torsions)
    if trace:
        return best_x, best_e, traj
    return best_x, best_e
