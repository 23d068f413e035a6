"""Linear-simplex heat-transfer subdomains: P1 triangles on the unit square
and P1 tetrahedra on the unit cube (the element types of the paper's own
experiments, Sec. 4: heat transfer on 2D triangle and 3D tetrahedron meshes).

Node (ix, iy[, iz]) of a grid with e elements per side has id
ix + (e+1) * (iy + (e+1) * iz), as for the box meshes.  Each square is cut
into two triangles along its (0,0)-(1,1) diagonal; each cube into the six
tetrahedra of its Kuhn (Freudenthal) subdivision, one per ordering of the
axes, all sharing the (0,0,0)-(1,1,1) diagonal.  These are conforming
triangulations of the grid, and the tetrahedra of the Kuhn subdivision are
congruent.

This module produces INPUTS only (element matrices, assembled K, K_reg,
kernel basis and B), like the rest of the package.
"""
from functools import lru_cache
from itertools import permutations
from typing import Tuple

import numpy as np
import scipy.sparse as sp

from .mesh import Subdomain, _grid_nodes, _regularise, _boundary_nodes
from .rng import signs_from_seed


def p1_stiffness(verts: np.ndarray) -> np.ndarray:
    """Stiffness of the Laplace operator on one linear simplex (d + 1
    vertices in R^d): K = |T| G G^T, G[a] = gradient of the barycentric
    coordinate of vertex a, |T| = |det J| / d!, J = [x_1 - x_0, ..., x_d - x_0]."""
    verts = np.asarray(verts, dtype=np.float64)
    d = verts.shape[1]
    J = (verts[1:] - verts[0]).T                  # d x d, columns are edge vectors
    Jinv = np.linalg.inv(J)
    G = np.zeros((d + 1, d))
    G[1:] = Jinv                                  # grad lambda_a = row a-1 of J^{-1}
    G[0] = -G[1:].sum(axis=0)
    vol = abs(np.linalg.det(J)) / float(np.prod(np.arange(1, d + 1)))
    return vol * (G @ G.T)


def _local_simplices(dim: int):
    """Local vertex offsets of the simplices of one grid cell."""
    if dim == 2:
        a, b, c, dd = (0, 0), (1, 0), (0, 1), (1, 1)
        return [np.array([a, b, dd]), np.array([a, dd, c])]
    out = []
    for perm in permutations(range(3)):
        v = [np.zeros(3, dtype=int)]
        for ax in perm:
            nxt = v[-1].copy()
            nxt[ax] += 1
            v.append(nxt)
        out.append(np.array(v))
    return out


@lru_cache(maxsize=32)
def _simplex_operator(dim: int, e: int):
    h = 1.0 / e
    elems = (e,) * dim
    npx = e + 1
    nodes = _grid_nodes(elems)
    nn = nodes.shape[0]
    cells = np.stack(np.meshgrid(*([np.arange(e)] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    rows, cols, data = [], [], []
    for loc in _local_simplices(dim):
        ke = p1_stiffness(loc.astype(np.float64) * h)
        corner = cells[:, None, :] + loc[None, :, :]                # cells x (d+1) x d
        if dim == 2:
            ids = corner[..., 0] + npx * corner[..., 1]
        else:
            ids = corner[..., 0] + npx * (corner[..., 1] + npx * corner[..., 2])
        nl = dim + 1
        rows.append(np.repeat(ids, nl, axis=1).ravel())
        cols.append(np.tile(ids, (1, nl)).ravel())
        data.append(np.tile(ke.ravel(), ids.shape[0]))
    K = sp.coo_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))), shape=(nn, nn)).tocsr()
    K.sum_duplicates()
    # couplings that cancel exactly in exact arithmetic (the face and body
    # diagonals of the Kuhn cells, the off-diagonal of the squares) are left
    # with round-off residue; they are zero entries of the P1 stiffness
    K.data[np.abs(K.data) <= 1e-12 * np.abs(K.diagonal()).max()] = 0.0
    K.eliminate_zeros()
    K.sort_indices()
    coords = nodes.astype(np.float64) * h
    R = np.ones((nn, 1))
    mid = [e // 2] * dim
    centre = mid[0] + npx * mid[1] if dim == 2 else mid[0] + npx * (mid[1] + npx * mid[2])
    fix = np.array([centre])
    Kreg, Q, rho = _regularise(K, R, fix)
    for arr in (K.indptr, K.indices, K.data, Kreg.indptr, Kreg.indices, Kreg.data, coords):
        arr.setflags(write=False)
    return K, Kreg, coords, R, fix, Q, rho


def simplex_subdomain(dim: int, e: int, seed: int) -> Subdomain:
    """P1 heat subdomain on the unit square (dim 2, triangles) or cube (dim 3,
    tetrahedra) with e elements per side ((e+1)^dim DOFs); multipliers on
    every boundary node (node-id order), signs from the SplitMix64 stream
    `seed`; regularised at the centre node (rho = mean(diag K))."""
    K, Kreg, coords, R, fix, Q, rho = _simplex_operator(int(dim), int(e))
    dof = _boundary_nodes((e,) * dim).astype(np.int32)
    sign = signs_from_seed(seed, dof.shape[0])
    kind = "heat_p1_tri" if dim == 2 else "heat_p1_tet"
    return Subdomain(kind=kind, dim=dim, elems=(e,) * dim, h=1.0 / e, dofs_per_node=1, n=K.shape[0],
                     k_rowptr=K.indptr.astype(np.int64), k_col=K.indices.astype(np.int32), k_val=K.data,
                     rowptr=Kreg.indptr.astype(np.int64), col=Kreg.indices.astype(np.int32), val=Kreg.data,
                     coords=coords, R=R, fix_dofs=fix, Q=Q, rho=rho, dof=dof, sign=sign, seed=seed)


def grid_shape(sd: Subdomain) -> Tuple[int, ...]:
    return tuple(e + 1 for e in sd.elems)
