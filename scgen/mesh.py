"""Structured-box FEM subdomains (heat transfer and linear elasticity).

Node (ix, iy, iz) of a box with (nx, ny, nz) elements has id
ix + (nx+1) * (iy + (ny+1) * iz); DOF c of node v is v * dofs_per_node + c.
"""
from dataclasses import dataclass, field
from functools import lru_cache
from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp

from .rng import signs_from_seed

# 1D linear-element stiffness (times 1/h) and mass (times h) on a unit segment.
_K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
_M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


@dataclass
class Subdomain:
    kind: str                      # "heat" | "elasticity" | "laplace1d"
    dim: int
    elems: Tuple[int, ...]         # elements per axis
    h: float
    dofs_per_node: int
    n: int
    # K (SPSD) and K_reg (SPD), full symmetric CSR with sorted columns
    k_rowptr: np.ndarray
    k_col: np.ndarray
    k_val: np.ndarray
    rowptr: np.ndarray             # K_reg
    col: np.ndarray
    val: np.ndarray
    coords: np.ndarray             # [n_nodes, dim]
    R: np.ndarray                  # [n, nker] kernel basis of K
    fix_dofs: np.ndarray           # DOFs carrying the regularisation
    Q: np.ndarray                  # [len(fix_dofs), nker], orthonormal columns
    rho: float
    dof: np.ndarray                # [m] int32, DOF of column j of B^T
    sign: np.ndarray               # [m] int8, +1/-1
    seed: int = 0
    gluing: str = "unique"
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.dof.shape[0])

    @property
    def node_grid(self) -> Tuple[int, ...]:
        return tuple(e + 1 for e in self.elems)

    def K_csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.k_val, self.k_col, self.k_rowptr), shape=(self.n, self.n))

    def Kreg_csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def Bt_dense(self) -> np.ndarray:
        """B^T as a dense n x m array (tests only)."""
        bt = np.zeros((self.n, self.m))
        bt[self.dof, np.arange(self.m)] = self.sign
        return bt

    def with_signs(self, sign: np.ndarray) -> "Subdomain":
        import copy
        s = copy.copy(self)
        s.sign = np.asarray(sign, dtype=np.int8)
        return s

    def with_columns(self, dof: np.ndarray, sign: np.ndarray) -> "Subdomain":
        import copy
        s = copy.copy(self)
        s.dof = np.asarray(dof, dtype=np.int32)
        s.sign = np.asarray(sign, dtype=np.int8)
        return s


# ----------------------------------------------------------------------------
# element matrices
# ----------------------------------------------------------------------------

def q1_heat_element() -> np.ndarray:
    """Bilinear square element, Laplace stiffness (independent of h in 2D).
    Local node a = ix + 2*iy."""
    return np.kron(_M1, _K1) + np.kron(_K1, _M1)


def hex8_heat_element(h: float) -> np.ndarray:
    """Trilinear cube element of side h, Laplace stiffness.
    Local node a = ix + 2*iy + 4*iz (kron order z, y, x)."""
    return h * (np.kron(np.kron(_M1, _M1), _K1) + np.kron(np.kron(_M1, _K1), _M1)
                + np.kron(np.kron(_K1, _M1), _M1))


def hex8_elasticity_element(h: float, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """Trilinear cube element of side h, isotropic elasticity, 2x2x2 Gauss.
    Local DOF 3*a + c with local node a = ix + 2*iy + 4*iz."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    corners = np.array([[ix, iy, iz] for iz in (0, 1) for iy in (0, 1) for ix in (0, 1)], dtype=float)
    ke = np.zeros((24, 24))
    for gz in g:
        for gy in g:
            for gx in g:
                xi = np.array([gx, gy, gz])
                dN = np.zeros((8, 3))  # derivatives w.r.t. physical x = h * xi
                for a in range(8):
                    f = [(xi[d] if corners[a, d] else 1 - xi[d]) for d in range(3)]
                    df = [(1.0 if corners[a, d] else -1.0) for d in range(3)]
                    dN[a, 0] = df[0] * f[1] * f[2] / h
                    dN[a, 1] = f[0] * df[1] * f[2] / h
                    dN[a, 2] = f[0] * f[1] * df[2] / h
                Bm = np.zeros((6, 24))
                for a in range(8):
                    dx, dy, dz = dN[a]
                    c = 3 * a
                    Bm[0, c] = dx
                    Bm[1, c + 1] = dy
                    Bm[2, c + 2] = dz
                    Bm[3, c] = dy
                    Bm[3, c + 1] = dx
                    Bm[4, c + 1] = dz
                    Bm[4, c + 2] = dy
                    Bm[5, c] = dz
                    Bm[5, c + 2] = dx
                ke += Bm.T @ D @ Bm * (h ** 3) / 8.0
    return 0.5 * (ke + ke.T)


# ----------------------------------------------------------------------------
# assembly helpers
# ----------------------------------------------------------------------------

def _grid_nodes(elems):
    npx = [e + 1 for e in elems]
    if len(elems) == 2:
        iy, ix = np.meshgrid(np.arange(npx[1]), np.arange(npx[0]), indexing="ij")
        return np.stack([ix.ravel(), iy.ravel()], axis=1)
    iz, iy, ix = np.meshgrid(np.arange(npx[2]), np.arange(npx[1]), np.arange(npx[0]), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)


def _connectivity(elems):
    npx = [e + 1 for e in elems]
    if len(elems) == 2:
        ey, ex = np.meshgrid(np.arange(elems[1]), np.arange(elems[0]), indexing="ij")
        base = (ex + npx[0] * ey).ravel()
        offs = [dx + npx[0] * dy for dy in (0, 1) for dx in (0, 1)]
    else:
        ez, ey, ex = np.meshgrid(np.arange(elems[2]), np.arange(elems[1]), np.arange(elems[0]), indexing="ij")
        base = (ex + npx[0] * (ey + npx[1] * ez)).ravel()
        offs = [dx + npx[0] * (dy + npx[1] * dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
    return base[:, None] + np.array(offs)[None, :]


def _assemble(elems, ke, dpn):
    conn = _connectivity(elems)
    nn = int(np.prod([e + 1 for e in elems]))
    n = nn * dpn
    if dpn == 1:
        edofs = conn
    else:
        edofs = (conn[:, :, None] * dpn + np.arange(dpn)[None, None, :]).reshape(conn.shape[0], -1)
    nl = edofs.shape[1]
    rows = np.repeat(edofs, nl, axis=1).ravel()
    cols = np.tile(edofs, (1, nl)).ravel()
    data = np.tile(ke.ravel(), conn.shape[0])
    K = sp.coo_matrix((data, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def _boundary_nodes(elems):
    nodes = _grid_nodes(elems)
    on = np.zeros(nodes.shape[0], dtype=bool)
    for d, e in enumerate(elems):
        on |= (nodes[:, d] == 0) | (nodes[:, d] == e)
    return np.nonzero(on)[0]


def _face_nodes(elems):
    """Faces x-, x+, y-, y+, (z-, z+), each in node-id order."""
    nodes = _grid_nodes(elems)
    out = []
    for d, e in enumerate(elems):
        out.append(np.nonzero(nodes[:, d] == 0)[0])
        out.append(np.nonzero(nodes[:, d] == e)[0])
    return out


def central_axis(elems) -> int:
    """Axis with the most elements (first one on ties)."""
    return int(np.argmax(np.asarray(elems)))


def fixing_nodes(elems, kind):
    """Nodes that carry the regularisation: the box centre for heat; three
    non-collinear nodes of the central plane for elasticity."""
    a = central_axis(elems)
    others = [d for d in range(len(elems)) if d != a]
    npx = [e + 1 for e in elems]

    def nid(p):
        if len(elems) == 2:
            return p[0] + npx[0] * p[1]
        return p[0] + npx[0] * (p[1] + npx[1] * p[2])

    mid = [e // 2 for e in elems]
    if kind == "heat":
        return np.array([nid(mid)])
    pts = []
    lo = [elems[d] // 4 for d in range(len(elems))]
    hi = [elems[d] - elems[d] // 4 for d in range(len(elems))]
    b, c = others
    for (pb, pc) in ((lo[b], lo[c]), (hi[b], lo[c]), (lo[b], hi[c])):
        p = list(mid)
        p[b] = pb
        p[c] = pc
        pts.append(nid(p))
    return np.array(pts)


def rigid_body_modes(coords: np.ndarray, dpn: int) -> np.ndarray:
    nn = coords.shape[0]
    if dpn == 1:
        return np.ones((nn, 1))
    c = coords - coords.mean(axis=0)
    R = np.zeros((nn * 3, 6))
    for k in range(3):
        R[k::3, k] = 1.0
    x, y, z = c[:, 0], c[:, 1], c[:, 2]
    R[1::3, 3] = -z
    R[2::3, 3] = y
    R[0::3, 4] = z
    R[2::3, 4] = -x
    R[0::3, 5] = -y
    R[1::3, 5] = x
    return R


def _regularise(K: sp.csr_matrix, R: np.ndarray, fix_dofs: np.ndarray):
    rho = float(K.diagonal().mean())
    Rf = R[fix_dofs, :]
    Q, _ = np.linalg.qr(Rf)
    add = rho * (Q @ Q.T)
    rr, cc = np.meshgrid(fix_dofs, fix_dofs, indexing="ij")
    Kreg = (K + sp.csr_matrix((add.ravel(), (rr.ravel(), cc.ravel())), shape=K.shape)).tocsr()
    Kreg.sum_duplicates()
    Kreg.sort_indices()
    return Kreg, Q, rho


@lru_cache(maxsize=64)
def _box_operator(kind: str, elems: Tuple[int, ...], h: float):
    dim = len(elems)
    if kind == "heat":
        dpn = 1
        ke = q1_heat_element() if dim == 2 else hex8_heat_element(h)
    elif kind == "elasticity":
        assert dim == 3
        dpn = 3
        ke = hex8_elasticity_element(h)
    else:
        raise ValueError(kind)
    K = _assemble(elems, ke, dpn)
    coords = _grid_nodes(elems).astype(np.float64) * h
    R = rigid_body_modes(coords, dpn)
    fn = fixing_nodes(elems, kind)
    fix_dofs = (fn[:, None] * dpn + np.arange(dpn)[None, :]).ravel()
    Kreg, Q, rho = _regularise(K, R, fix_dofs)
    for arr in (K.indptr, K.indices, K.data, Kreg.indptr, Kreg.indices, Kreg.data, coords, R):
        arr.setflags(write=False)
    return dpn, K, Kreg, coords, R, fix_dofs, Q, rho


def gluing_columns(elems, dpn, mode="unique"):
    """DOF of each column of B^T in generation order."""
    if mode == "unique":
        nodes = _boundary_nodes(elems)
    elif mode == "per_face":
        nodes = np.concatenate(_face_nodes(elems))
    else:
        raise ValueError(mode)
    return (nodes[:, None] * dpn + np.arange(dpn)[None, :]).ravel().astype(np.int32)


def box_subdomain(kind: str, elems, h: float, seed: int, gluing: str = "unique") -> Subdomain:
    elems = tuple(int(e) for e in elems)
    dpn, K, Kreg, coords, R, fix_dofs, Q, rho = _box_operator(kind, elems, float(h))
    dof = gluing_columns(elems, dpn, gluing)
    sign = signs_from_seed(seed, dof.shape[0])
    return Subdomain(kind=kind, dim=len(elems), elems=elems, h=float(h), dofs_per_node=dpn,
                     n=K.shape[0], k_rowptr=K.indptr.astype(np.int64), k_col=K.indices.astype(np.int32),
                     k_val=K.data, rowptr=Kreg.indptr.astype(np.int64), col=Kreg.indices.astype(np.int32),
                     val=Kreg.data, coords=coords, R=R, fix_dofs=fix_dofs, Q=Q, rho=rho,
                     dof=dof, sign=sign, seed=seed, gluing=gluing)


def heat_q1_2d(nx: int, ny: int, h: float, seed: int) -> Subdomain:
    return box_subdomain("heat", (nx, ny), h, seed)


def heat_hex8(nx: int, ny: int, nz: int, h: float, seed: int, gluing="unique") -> Subdomain:
    return box_subdomain("heat", (nx, ny, nz), h, seed, gluing)


def elasticity_hex8(nx: int, ny: int, nz: int, h: float, seed: int, gluing="unique") -> Subdomain:
    return box_subdomain("elasticity", (nx, ny, nz), h, seed, gluing)


def laplace_1d(N: int, dof: Optional[np.ndarray] = None, seed: int = 1,
               fix_node: int = 0) -> Subdomain:
    """N linear elements on [0, 1] (h = 1/N), nodes 0..N, fixing node `fix_node`,
    rho = mean(diag K).  Default multipliers: both end nodes."""
    h = 1.0 / N
    n = N + 1
    main = np.full(n, 2.0 / h)
    main[0] = main[-1] = 1.0 / h
    K = sp.diags([np.full(n - 1, -1.0 / h), main, np.full(n - 1, -1.0 / h)], [-1, 0, 1], format="csr")
    K.sort_indices()
    R = np.ones((n, 1))
    fix = np.array([fix_node])
    Kreg, Q, rho = _regularise(K, R, fix)
    if dof is None:
        dof = np.array([0, N])
    dof = np.asarray(dof, dtype=np.int32)
    sign = signs_from_seed(seed, dof.shape[0])
    coords = (np.arange(n, dtype=float) * h)[:, None]
    return Subdomain(kind="laplace1d", dim=1, elems=(N,), h=h, dofs_per_node=1, n=n,
                     k_rowptr=K.indptr.astype(np.int64), k_col=K.indices.astype(np.int32), k_val=K.data,
                     rowptr=Kreg.indptr.astype(np.int64), col=Kreg.indices.astype(np.int32), val=Kreg.data,
                     coords=coords, R=R, fix_dofs=fix, Q=Q, rho=rho, dof=dof, sign=sign, seed=seed)
