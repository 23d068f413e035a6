"""ORACLE -- test infrastructure only.

Plain, slow CPU references for the dual Schur complement assembly and the
iteration phase.  Only tests, the smoke check and the benchmark's CPU-baseline
leg import this package; the product library never does, and this package
imports nothing from it.  Inputs come from `scgen` (seeded generator).

  schur(sd, sel)      F[S,S] = (B K_reg^{-1} B^T)[S,S] by the plain C routine
                      in oracle.c (natural-order Cholesky, full forward
                      substitution, Y^T Y), long double by default
  brute_F(sd)         F by a dense LU solve (numpy), the plain definition
  saddle_F(sd)        F from the inverse of the saddle-point matrix of eq. (13)
  pinv_F(sd)          F with the Moore-Penrose inverse of K (another valid K^+)
  projector(G)        I - G (G^T G)^{-1} G^T
  pcpg(F, G, d, it)   projected CG on one subdomain's dual problem
  dual_direct(F,G,d)  the same problem by one dense saddle-point solve (pins pcpg)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MUTATIONS = {
    "none": 0, "chol_skip_first_term": 1, "chol_plus": 2, "chol_no_sqrt": 3,
    "fwd_no_div": 4, "fwd_transposed": 5, "ignore_sign": 6, "syrk_index": 7,
    "dof_off_by_one": 8,
}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_schur.restype = ctypes.c_int
        lib.orc_schur.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_int32]
        lib.orc_last_phase_seconds.restype = None
        lib.orc_last_phase_seconds.argtypes = [ctypes.c_void_p]
        lib.orc_cholesky_dense.restype = ctypes.c_int
        lib.orc_cholesky_dense.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    pass


def schur_csr(n, rowptr, col, val, dof, sign, sel=None, prec="ld", nthreads=None,
              mutation="none", want_Y=False):
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    dof = np.ascontiguousarray(dof, dtype=np.int32)
    sign = np.ascontiguousarray(sign, dtype=np.int8)
    m = dof.shape[0]
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        nsel = sel.shape[0]
    else:
        nsel = m
    F = np.zeros((nsel, nsel), dtype=np.float64, order="F")
    Y = np.zeros((n, nsel), dtype=np.float64, order="F") if want_Y else None
    if nthreads is None:
        nthreads = max(1, min(16, os.cpu_count() or 1))
    rc = lib.orc_schur(n, _ptr(rowptr), _ptr(col), _ptr(val), m, _ptr(dof), _ptr(sign), nsel,
                       _ptr(sel), 1 if prec == "ld" else 0, _ptr(F), _ptr(Y), int(nthreads),
                       MUTATIONS[mutation])
    if rc != 0:
        raise OracleError(f"orc_schur returned {rc}")
    return (F, Y) if want_Y else F


def schur(sd, sel=None, prec="ld", nthreads=None, mutation="none", want_Y=False):
    """F[S,S] for a scgen.Subdomain (all columns when sel is None)."""
    return schur_csr(sd.n, sd.rowptr, sd.col, sd.val, sd.dof, sd.sign, sel=sel, prec=prec,
                     nthreads=nthreads, mutation=mutation, want_Y=want_Y)


def last_phase_seconds():
    """(Cholesky, forward substitution, Y^T Y) wall seconds of the last
    schur() call in this process."""
    out = np.zeros(3)
    _load().orc_last_phase_seconds(_ptr(out))
    return tuple(float(x) for x in out)


def cholesky_dense(sd):
    lib = _load()
    L = np.zeros((sd.n, sd.n))
    rc = lib.orc_cholesky_dense(sd.n, _ptr(np.ascontiguousarray(sd.rowptr, dtype=np.int64)),
                                _ptr(np.ascontiguousarray(sd.col, dtype=np.int32)),
                                _ptr(np.ascontiguousarray(sd.val)), _ptr(L))
    if rc != 0:
        raise OracleError(f"orc_cholesky_dense returned {rc}")
    return L


# --------------------------------------------------------------------------
# independent routes used to pin the oracle (dense numpy, small sizes only)
# --------------------------------------------------------------------------

def brute_F(sd):
    """F = B K_reg^{-1} B^T by numpy's LU solve (paper eq. (9)-(10))."""
    K = sd.Kreg_csr().toarray()
    Bt = sd.Bt_dense()
    return Bt.T @ np.linalg.solve(K, Bt)


def saddle_F(sd):
    """F from the saddle-point matrix [[K_reg, B^T], [B, 0]] (paper eq. (13)):
    the multiplier block of its inverse equals -F^{-1} when F is nonsingular."""
    K = sd.Kreg_csr().toarray()
    Bt = sd.Bt_dense()
    n, m = Bt.shape
    S = np.zeros((n + m, n + m))
    S[:n, :n] = K
    S[:n, n:] = Bt
    S[n:, :n] = Bt.T
    inv = np.linalg.inv(S)
    return -np.linalg.inv(inv[n:, n:])


def pinv_F(sd, rcond=1e-10):
    """B K^+ B^T with the Moore-Penrose inverse of the unregularised K."""
    K = sd.K_csr().toarray()
    Bt = sd.Bt_dense()
    return Bt.T @ np.linalg.pinv(K, rcond=rcond, hermitian=True) @ Bt


def gluing_G(sd):
    """G = B R (paper, Sec. 2.1), m x nker."""
    return sd.sign[:, None].astype(np.float64) * sd.R[sd.dof, :]


def projector(G):
    """P_G = I - G (G^T G)^{-1} G^T."""
    GtG = G.T @ G
    return np.eye(G.shape[0]) - G @ np.linalg.solve(GtG, G.T)


def relF(A, B):
    """||A - B||_F / ||B||_F."""
    return float(np.linalg.norm(A - B) / np.linalg.norm(B))


# --------------------------------------------------------------------------
# iteration phase
# --------------------------------------------------------------------------

PCPG_MUTATIONS = ("none", "no_projection", "beta_unprojected", "alpha_inverted", "lambda_minus")


def pcpg(F, G, d, iters, mutation="none"):
    """Projected conjugate gradients on one subdomain's dual problem
    [F -G; -G^T 0][lambda; alpha] = [d; -e] with e = 0 (paper eq. (7); the
    paper cites PCPG without listing it), identity preconditioner, FP64:
        lambda_0 = 0, r_0 = d, w_0 = P r_0, p_0 = w_0
        q = F p;  alpha = (w.w)/(p.q);  lambda += alpha p;  r -= alpha q
        w' = P r;  beta = (w'.w')/(w.w);  p = w' + beta p
    Returns lambda and the history of ||w_k||.  `mutation` plants one
    deliberate mistake (PCPG_MUTATIONS; tests show that the direct solve of
    the dual system catches each); "none" = the correct iteration."""
    assert mutation in PCPG_MUTATIONS, mutation
    P = projector(G)
    proj = (lambda v: v.copy()) if mutation == "no_projection" else (lambda v: P @ v)
    lam = np.zeros_like(d)
    r = d.copy()
    w = proj(r)
    p = w.copy()
    ww = float(w @ w)
    hist = [np.sqrt(ww)]
    for _ in range(iters):
        q = F @ p
        pq = float(p @ q)
        if pq == 0.0 or ww == 0.0:
            break
        alpha = pq / ww if mutation == "alpha_inverted" else ww / pq
        lam = lam - alpha * p if mutation == "lambda_minus" else lam + alpha * p
        r -= alpha * q
        w = proj(r)
        ww_new = float(w @ w)
        beta = (float(r @ r) if mutation == "beta_unprojected" else ww_new) / ww
        p = w + beta * p
        ww = ww_new
        hist.append(np.sqrt(ww))
    return lam, np.array(hist)


def dual_direct(F, G, d):
    """lambda of the dual problem (paper eq. (7)) with e = 0 by one dense
    solve of the saddle-point system [F -G; -G^T 0][lambda; alpha] = [d; 0]
    (numpy LU; F SPD on ker G^T, G of full column rank).  Returns (lambda,
    alpha)."""
    m, k = G.shape
    A = np.zeros((m + k, m + k))
    A[:m, :m] = F
    A[:m, m:] = -G
    A[m:, :m] = -G.T
    rhs = np.concatenate([d, np.zeros(k)])
    x = np.linalg.solve(A, rhs)
    return x[:m], x[m:]
