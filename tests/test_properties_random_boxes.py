"""Property tests over randomly drawn small boxes (hypothesis; CPU only).

The boxes are heat (2D / 3D) and elasticity (3D) subdomains of 1-6 elements
per side with random sign seeds and both gluings.  On each one:

* the oracle's F = B K_reg^{-1} B^T (Sec. 2.2 eq. (10)) equals the dense LU
  route and is exactly symmetric, positive definite with distinct gluing DOFs
  and positive semi-definite with the per-face gluing;
* the host planner of the library (no GPU) returns a permutation, a factor
  with L L^T = P K_reg P^T, pivots p_j = iperm[dof_j] sorted stably by
  (p_j, j) (Sec. 3, the stepped shape of P B^T), and the forward substitution
  Y = L^{-1} P B^T keeps every entry above a column's pivot exactly zero
  (Sec. 3) and every entry off the elimination-tree path of the pivot exactly
  zero (the reach the TRSM's visit lists rely on).
"""
import numpy as np
import pytest
import scipy.linalg
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import scgen

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def boxes(draw):
    kind = draw(st.sampled_from(["heat2", "heat3", "elasticity"]))
    if kind == "heat2":
        elems = tuple(draw(st.integers(1, 6)) for _ in range(2))
    elif kind == "heat3":
        elems = tuple(draw(st.integers(1, 5)) for _ in range(3))
    else:
        elems = tuple(draw(st.integers(1, 4)) for _ in range(3))
    gluing = draw(st.sampled_from(["unique", "per_face"]))
    seed = draw(st.integers(0, 2**32 - 1))
    return scgen.box_subdomain("heat" if kind != "elasticity" else "elasticity", elems,
                               1.0 / max(elems), seed=seed, gluing=gluing), gluing


@SETTINGS
@given(boxes())
def test_oracle_matches_dense_lu_and_is_symmetric(case):
    s, gluing = case
    F = oracle.schur(s)
    assert np.array_equal(F, F.T)
    assert oracle.relF(F, oracle.brute_F(s)) < 1e-12
    w = np.linalg.eigvalsh(F)
    if gluing == "unique":
        assert w.min() > 0
    else:
        # repeated DOFs (edges and corners shared by faces) give equal columns of B^T
        assert w.min() > -1e-12 * w.max()


def _etree_paths(L):
    """Parent of each column: the first row below the diagonal holding a nonzero."""
    n = L.shape[0]
    parent = np.full(n, -1)
    for j in range(n):
        nz = np.nonzero(L[j + 1:, j])[0]
        if nz.size:
            parent[j] = j + 1 + nz[0]
    return parent


@SETTINGS
@given(boxes())
def test_host_planner_factor_pivots_staircase_and_reach(case):
    P = pytest.importorskip("paper_2509_21037_amd.scasm")
    s, _ = case
    h = P.host_analyze(s, values=True, want_L=True)
    n, m = s.n, s.m
    perm = h["perm"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)

    L = h["L"]
    assert np.abs(np.triu(L, 1)).max() == 0
    K = s.Kreg_csr().toarray()[np.ix_(perm, perm)]
    assert np.linalg.norm(L @ L.T - K) / np.linalg.norm(K) < 1e-13

    # pivots of the columns of P B^T, sorted stably by (pivot, column)
    p = iperm[s.dof]
    order = np.lexsort((np.arange(m), p))
    assert np.array_equal(h["pi"], order)
    assert np.array_equal(h["piv"], p[order])

    # Y = L^{-1} P B^T: exact zeros above each pivot and off its path
    Bt = np.zeros((n, m))
    Bt[iperm[s.dof], np.arange(m)] = s.sign
    Y = scipy.linalg.solve_triangular(L, Bt, lower=True)
    parent = _etree_paths(L)
    for j in range(m):
        r = p[j]
        assert not Y[:r, j].any()
        on = np.zeros(n, dtype=bool)
        while r >= 0:
            on[r] = True
            r = parent[r]
        assert not Y[~on, j].any()
