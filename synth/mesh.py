"""Voxel tet meshes with the Freudenthal (Kuhn) six-tet split of every cell.

Vertex numbering: the vertices of the occupied cells are the grid corners
``(i, j, k)``; they are numbered in increasing order of the global grid key
``i + (NX+1) * (j + (NY+1) * k)``.  For a full box this is exactly
``i + (nx+1) * (j + (ny+1) * k)``.

Tet order: occupied cells in increasing cell key ``i + NX*(j + NY*k)``, and
inside a cell the six axis permutations in lexicographic order.  The tet of
permutation ``p`` walks the cell diagonal from corner (0,0,0) to (1,1,1),
stepping along axis ``p[0]``, then ``p[1]``, then ``p[2]``.  For odd
permutations the last two vertices are swapped so that every tet has positive
orientation (the rest-shape edge matrix has positive determinant).  All cells
use the same split, so the mesh is conforming.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np

_PERMS = list(itertools.permutations((0, 1, 2)))  # lexicographic order


def _perm_is_odd(p) -> bool:
    inv = sum(1 for a in range(3) for b in range(a + 1, 3) if p[a] > p[b])
    return inv % 2 == 1


@dataclasses.dataclass
class VoxelMesh:
    rest: np.ndarray  # (n_verts, 3) float64, metres
    tets: np.ndarray  # (n_tets, 4) int32
    grid_index: np.ndarray  # (n_verts, 3) int64 integer corner coordinates
    cell: float

    @property
    def n_verts(self) -> int:
        return int(self.rest.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def voxel_mesh(occupied: np.ndarray, cell: float, origin=(0.0, 0.0, 0.0)) -> VoxelMesh:
    """Tet mesh of the occupied cells of a boolean grid ``occupied[i, j, k]``."""
    occ = np.asarray(occupied, dtype=bool)
    NX, NY, NZ = occ.shape
    # occupied cells in increasing key i + NX*(j + NY*k)
    ks, js, is_ = np.nonzero(np.transpose(occ, (2, 1, 0)))
    cells = np.stack([is_, js, ks], axis=1)  # already sorted by key (k, j, i)

    def vkey(i, j, k):
        return i + (NX + 1) * (j + (NY + 1) * k)

    # corner keys used by each tet
    raw = []
    for p in _PERMS:
        path = [np.zeros(3, dtype=np.int64)]
        for ax in p:
            step = path[-1].copy()
            step[ax] += 1
            path.append(step)
        if _perm_is_odd(p):
            path = [path[0], path[1], path[3], path[2]]
        raw.append(path)
    tet_keys = np.empty((cells.shape[0], 6, 4), dtype=np.int64)
    for t, path in enumerate(raw):
        for a, off in enumerate(path):
            c = cells + off[None, :]
            tet_keys[:, t, a] = vkey(c[:, 0], c[:, 1], c[:, 2])
    tet_keys = tet_keys.reshape(-1, 4)
    used = np.unique(tet_keys)
    remap = {int(k): n for n, k in enumerate(used)}
    tets = np.vectorize(remap.__getitem__, otypes=[np.int64])(tet_keys).astype(np.int32)
    gi = np.stack(
        [used % (NX + 1), (used // (NX + 1)) % (NY + 1), used // ((NX + 1) * (NY + 1))], axis=1
    )
    rest = np.asarray(origin, dtype=np.float64)[None, :] + cell * gi.astype(np.float64)
    return VoxelMesh(rest=rest, tets=tets, grid_index=gi, cell=float(cell))


def box_mesh(nx: int, ny: int, nz: int, cell: float, origin=(0.0, 0.0, 0.0)) -> VoxelMesh:
    return voxel_mesh(np.ones((nx, ny, nz), dtype=bool), cell, origin)


def quadruped_mesh(cell: float, origin=(0.0, 0.0, 0.0)) -> VoxelMesh:
    """Torso of 32x16x8 cells on four 4x4x16-cell legs under its corners."""
    NX, NY, NZ = 32, 16, 16 + 8
    occ = np.zeros((NX, NY, NZ), dtype=bool)
    occ[:, :, 16:] = True  # torso
    for x0 in (0, NX - 4):
        for y0 in (0, NY - 4):
            occ[x0:x0 + 4, y0:y0 + 4, :16] = True  # legs
    return voxel_mesh(occ, cell, origin)
