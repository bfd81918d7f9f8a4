"""Structured tetrahedral meshes of the unit cube (input data only).

The cube [0,1]^3 is cut into n^3 sub-cubes and every sub-cube into six
tetrahedra by the Kuhn (Freudenthal) split: each tetrahedron follows one
monotone lattice path from the sub-cube's lowest corner to its highest corner,
one per ordering of the three axis steps. Neighbouring sub-cubes then agree on
their shared face diagonals, so the mesh is conforming and every interior node
has 14 neighbours.

Numbering: node (i, j, k) -> i + (n+1) * (j + (n+1) * k), x fastest; tets are
ordered by sub-cube (x fastest) and then by the axis ordering below.

Second-order (10-node) tets add the midpoint of every edge. On the Kuhn split
every point of the half-step lattice is the midpoint of exactly one edge (an
axis edge, the one diagonal of a face, or the body diagonal of a sub-cube), so
the nodes are the (2n+1)^3 lattice points with spacing 1/(2n), numbered the
same way; a tet lists its 4 vertices and then the midpoints of its edges
(0,1), (0,2), (0,3), (1,2), (1,3), (2,3).
"""

from __future__ import annotations

import itertools

import numpy as np

# Orderings of the three axis steps, fixed once so that tet numbering is stable.
AXIS_ORDERS = tuple(itertools.permutations((0, 1, 2)))


def _kuhn_offsets() -> np.ndarray:
    """Vertex offsets (6 tets x 4 vertices x 3 axes) of the Kuhn split of a unit cube."""
    offs = np.zeros((6, 4, 3), dtype=np.int64)
    for t, order in enumerate(AXIS_ORDERS):
        cur = np.zeros(3, dtype=np.int64)
        offs[t, 0] = cur
        for v, axis in enumerate(order, start=1):
            cur = cur.copy()
            cur[axis] = 1
            offs[t, v] = cur
    return offs


def kuhn_cube_mesh(n: int):
    """Return (xyz [N,3] float64, tets [6 n^3, 4] int32) for the n^3 Kuhn cube mesh."""
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    g = np.arange(m, dtype=np.float64) / n
    # lexicographic nodes, x fastest
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)

    c = np.arange(n, dtype=np.int64)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    base = (ci + m * (cj + m * ck)).ravel()  # lowest corner of each sub-cube
    offs = _kuhn_offsets()  # (6, 4, 3)
    off_id = offs[..., 0] + m * (offs[..., 1] + m * offs[..., 2])  # (6, 4)
    tets = base[:, None, None] + off_id[None, :, :]  # (n^3, 6, 4)
    if m ** 3 >= 2 ** 31:
        raise ValueError("mesh too large for int32 node ids")
    return xyz, tets.reshape(-1, 4).astype(np.int32)


def permute_nodes(xyz, tets, dir_nodes, seed: int):
    """Relabel nodes by a seeded random permutation.

    Returns (xyz', tets', dir_nodes', perm) with xyz'[perm[i]] = xyz[i]; a
    consumer that relies on connectivity rather than on the structured
    numbering must give the same physics on the relabelled mesh.
    """
    rng = np.random.default_rng(seed)
    n = xyz.shape[0]
    perm = rng.permutation(n)
    xyz2 = np.empty_like(xyz)
    xyz2[perm] = xyz
    tets2 = perm[tets].astype(np.int32)
    dn2 = perm[dir_nodes].astype(np.int32)
    return xyz2, tets2, dn2, perm


def shuffle_tets(tets, tet_mat, seed: int, flip_orientation: bool = True):
    """Reorder tets and (optionally) their vertices by a seeded permutation.

    Swapping two vertices flips a tet's orientation; consumers use |det J|, so
    the physics must not change.
    """
    rng = np.random.default_rng(seed)
    order = rng.permutation(tets.shape[0])
    t2 = tets[order].copy()
    m2 = tet_mat[order].copy()
    if flip_orientation:
        flip = rng.random(t2.shape[0]) < 0.5
        t2[flip, 0], t2[flip, 1] = t2[flip, 1].copy(), t2[flip, 0].copy()
        rot = rng.integers(0, 4, size=t2.shape[0])
        for r in range(1, 4):
            sel = rot == r
            t2[sel] = np.roll(t2[sel], r, axis=1)
    return t2, m2, order


P2_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def kuhn_cube_mesh_p2(n: int):
    """Return (xyz [(2n+1)^3, 3], tets [6 n^3, 10] int32) for the n^3 Kuhn cube
    mesh with second-order (10-node) tets."""
    if n < 1:
        raise ValueError("n must be >= 1")
    m = 2 * n + 1
    if m ** 3 >= 2 ** 31:
        raise ValueError("mesh too large for int32 node ids")
    g = np.arange(m, dtype=np.float64) / (2 * n)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    c = np.arange(n, dtype=np.int64)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    corner = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)  # (n^3, 3) lowest corner
    offs = _kuhn_offsets()  # (6, 4, 3) vertex offsets in sub-cube units
    # lattice coordinates (spacing 1/(2n)) of the 4 vertices and 6 midpoints
    pts = [2 * offs[:, a, :] for a in range(4)] + [offs[:, a, :] + offs[:, b, :] for a, b in P2_EDGES]
    loc = np.stack(pts, axis=1)  # (6, 10, 3)
    lat = 2 * corner[:, None, None, :] + loc[None, :, :, :]  # (n^3, 6, 10, 3)
    ids = lat[..., 0] + m * (lat[..., 1] + m * lat[..., 2])
    return xyz, ids.reshape(-1, 10).astype(np.int32)
