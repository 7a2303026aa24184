"""Ligand preprocessing for the oracle: bond graph (rings allowed inside rigid fragments),
rotatable bonds, moving sets, and the intramolecular pair list.

The paper describes the ligand as point atoms whose degrees of freedom are the
rigid-body translation (and orientation) plus the rotatable bonds (Background,
"Design and Structure of MiniMDock"), and the energy kernel as a sequence of
per-atom position set-up, rotations applied in a fixed order, and a per-atom
energy sum (Section "Approach 1", listing of decomposed target functions).

Readings taken here (the paper gives none of them):
  * reference coordinates are moved so that their centroid is the origin, which is
    the centre of the orientation and the point the translation genes place;
  * atom `root` (default 0) anchors the torsion tree; torsion k turns the atoms on the far
    side of its bond (a_k, b_k), a_k being the end nearer the root; a rotatable bond lies in
    no ring (cutting it splits the molecule), so its far side is well defined;
  * intramolecular pairs are the atom pairs at least three bonds apart (1-4 and
    beyond) whose connecting path crosses at least one rotatable bond; pairs inside
    one rigid fragment keep a constant distance and are left out.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np


class LigandError(ValueError):
    pass


@dataclass
class OracleLigand:
    n_atoms: int
    n_torsions: int
    p0: np.ndarray            # float64 [N][3], centroid at the origin
    types: np.ndarray         # int [N]
    charges: np.ndarray       # float64 [N]
    type_params: np.ndarray   # float64 [7][7]
    neighbours: list          # adjacency lists
    depth: np.ndarray         # graph distance from the root
    tors_a: np.ndarray        # int [T], root-side atom of torsion k (gene order)
    tors_b: np.ndarray        # int [T], far-side atom
    moving: np.ndarray        # bool [T][N], atoms turned by torsion k
    pairs: np.ndarray         # int [P][2], i < j

    @property
    def n_genes(self):
        return 7 + self.n_torsions


def _bfs(neighbours, start):
    n = len(neighbours)
    dist = -np.ones(n, dtype=np.int64)
    parent = -np.ones(n, dtype=np.int64)
    dist[start] = 0
    dq = deque([start])
    while dq:
        a = dq.popleft()
        for b in neighbours[a]:
            if dist[b] < 0:
                dist[b] = dist[a] + 1
                parent[b] = a
                dq.append(b)
    return dist, parent


def prepare(xyz, types, charges, bonds, torsions, type_params, root=0) -> OracleLigand:
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = xyz.shape[0]
    types = np.asarray(types, dtype=np.int64).reshape(n)
    charges = np.asarray(charges, dtype=np.float64).reshape(n)
    bonds = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
    torsions = np.asarray(torsions, dtype=np.int64).reshape(-1)
    tp = np.asarray(type_params, dtype=np.float64).reshape(-1, 7)
    if n < 1:
        raise LigandError("a ligand needs at least one atom")
    if bonds.shape[0] < n - 1:
        raise LigandError("a connected bond graph needs at least n_atoms - 1 bonds")
    if len({frozenset((int(a), int(b))) for a, b in bonds}) != bonds.shape[0]:
        raise LigandError("bond listed twice")
    if np.any(bonds < 0) or np.any(bonds >= n) or np.any(bonds[:, 0] == bonds[:, 1]):
        raise LigandError("bond atom index out of range")
    if np.any(types < 0) or np.any(types >= tp.shape[0]):
        raise LigandError("atom type out of range")
    if not (0 <= root < n):
        raise LigandError("root atom out of range")
    neighbours = [[] for _ in range(n)]
    for a, b in bonds:
        neighbours[a].append(int(b))
        neighbours[b].append(int(a))
    depth, parent = _bfs(neighbours, root)
    if np.any(depth < 0):
        raise LigandError("bonds do not connect every atom")

    T = torsions.shape[0]
    if len(set(torsions.tolist())) != T or np.any(torsions < 0) or np.any(torsions >= bonds.shape[0]):
        raise LigandError("torsion bond index invalid or repeated")
    tors_a = np.zeros(T, dtype=np.int64)
    tors_b = np.zeros(T, dtype=np.int64)
    moving = np.zeros((T, n), dtype=bool)
    for k, bi in enumerate(torsions):
        a, b = bonds[bi]
        if depth[a] > depth[b]:
            a, b = b, a
        if len(neighbours[a]) < 2 or len(neighbours[b]) < 2:
            raise LigandError("a terminal bond cannot be a torsion")
        tors_a[k], tors_b[k] = a, b
        # far side of the bond: everything reachable from b without crossing (a, b); in a ring
        # the other way round reaches a, and the bond has no far side
        seen = {int(b)}
        dq = deque([int(b)])
        while dq:
            x = dq.popleft()
            for y in neighbours[x]:
                if (x, y) != (b, a) and y not in seen:
                    seen.add(y)
                    dq.append(y)
        if int(a) in seen:
            raise LigandError("a rotatable bond cannot lie in a ring")
        moving[k, list(seen)] = True

    # pair list: graph distance >= 3 and a rotatable bond on the path (every path between two
    # atoms crosses the same rotatable bonds, since none lies in a ring)
    rot_bonds = {frozenset((int(tors_a[k]), int(tors_b[k]))) for k in range(T)}
    pairs = []
    for i in range(n):
        dist, par = _bfs(neighbours, i)
        for j in range(i + 1, n):
            if dist[j] < 3:
                continue
            x, crosses = j, False
            while x != i:
                if frozenset((int(x), int(par[x]))) in rot_bonds:
                    crosses = True
                    break
                x = par[x]
            if crosses:
                pairs.append((i, j))
    pairs = np.array(pairs, dtype=np.int64).reshape(-1, 2)

    p0 = xyz - xyz.mean(axis=0)
    return OracleLigand(n_atoms=n, n_torsions=T, p0=p0, types=types, charges=charges,
                        type_params=tp, neighbours=neighbours, depth=depth,
                        tors_a=tors_a, tors_b=tors_b, moving=moving, pairs=pairs)


def from_synth(lig) -> OracleLigand:
    """Convenience: prepare from an object with xyz/types/charges/bonds/torsions/type_params."""
    return prepare(lig.xyz, lig.types, lig.charges, lig.bonds, lig.torsions,
                   lig.type_params, getattr(lig, "root", 0))
