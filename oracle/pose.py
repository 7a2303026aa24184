"""Genotype -> atom coordinates (oracle).

Degrees of freedom (Background, "Design and Structure of MiniMDock"): translation,
orientation and the rotatable bonds.  The energy kernel applies the bond rotations
in a fixed order before the per-atom energies are taken (Section "Approach 1",
listing of decomposed target functions, and the paragraph that follows it).

Genotype layout (a reading; the paper fixes none): genes[0:3] translation t in
Angstrom, genes[3:7] orientation quaternion q = (w, x, y, z) used after
normalisation, genes[7:] torsion angles theta_k in radians, relative to the input
conformation, right-handed about the bond direction a_k -> b_k.

Construction used here: root-to-leaf.  Torsions are applied in order of increasing
depth of their root-side atom, each about its bond axis as it stands at that
moment (after the rotations of the torsions nearer the root); then the whole
ligand is rotated by R(q/|q|) about the origin (the reference centroid) and
translated by t.
"""
from __future__ import annotations

import math

import numpy as np


def quat_normalise(q):
    q = np.asarray(q, dtype=np.float64)
    return q / np.linalg.norm(q)


def quat_to_matrix(q):
    """Rotation matrix of the unit quaternion q/|q| = (w, x, y, z) (Hamilton convention)."""
    w, x, y, z = quat_normalise(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def quat_mul(a, b):
    """Hamilton product a (x) b for (w, x, y, z) quaternions."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def rodrigues(u, theta, v):
    """Rotate vector(s) v by angle theta about the unit axis u (right-handed):
    v cos(theta) + (u x v) sin(theta) + u (u . v)(1 - cos(theta))."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    c, s = math.cos(theta), math.sin(theta)
    return v * c + np.cross(u, v) * s + np.outer(v @ u, u).reshape(v.shape) * (1.0 - c)


def torsion_order(lig):
    """Torsion indices sorted by the depth of their root-side atom (stable)."""
    return sorted(range(lig.n_torsions), key=lambda k: (lig.depth[lig.tors_a[k]], k))


def internal_coords(lig, genes):
    """Ligand-frame coordinates after the torsion rotations only (root-to-leaf)."""
    genes = np.asarray(genes, dtype=np.float64)
    p = lig.p0.copy()
    for k in torsion_order(lig):
        a, b = lig.tors_a[k], lig.tors_b[k]
        axis = p[b] - p[a]
        axis = axis / np.linalg.norm(axis)
        m = lig.moving[k]
        p[m] = p[a] + rodrigues(axis, genes[7 + k], p[m] - p[a])
    return p


def pose(lig, genes):
    """Atom coordinates [N][3] in the receptor frame for one genotype."""
    genes = np.asarray(genes, dtype=np.float64)
    p = internal_coords(lig, genes)
    R = quat_to_matrix(genes[3:7])
    return p @ R.T + genes[0:3]


def wrap_angle(theta):
    """Map an angle to (-pi, pi]."""
    return theta - 2.0 * math.pi * math.ceil((theta - math.pi) / (2.0 * math.pi))
