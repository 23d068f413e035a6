"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, independent routes (dense LU, saddle-point inverse, Moore-Penrose
and spectral generalised inverses), residuals and invariants.  The mutation
test at the end plants each plausible mistake in the oracle and checks that
at least one pin catches it."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import scgen
from scgen.rng import signs_from_seed


def _small_cases():
    return [
        scgen.config_subdomains(1)[0],
        scgen.box_subdomain("heat", (4, 5, 3), 0.25, seed=11),
        scgen.box_subdomain("elasticity", (3, 4, 3), 0.25, seed=12),
        scgen.box_subdomain("elasticity", (2, 2, 5), 0.5, seed=13, gluing="unique"),
        scgen.simplex_subdomain(2, 9, seed=14),
        scgen.simplex_subdomain(3, 5, seed=15),
    ]


# ---------------------------------------------------------------- closed form

def _laplace_inverse_closed_form(N, rho):
    """K_reg^{-1}[i, j] = 1/rho + h min(i, j) for 1D Laplace fixed at node 0."""
    h = 1.0 / N
    i = np.arange(N + 1)
    return 1.0 / rho + h * np.minimum.outer(i, i)


@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 50, 200])
def test_1d_laplace_closed_form(N):
    rng = np.random.default_rng(N)
    mm = min(N + 1, 12)
    dof = np.sort(rng.choice(N + 1, size=mm, replace=False)).astype(np.int32)
    rng.shuffle(dof)
    s = scgen.laplace_1d(N, dof=dof, seed=N)
    G = _laplace_inverse_closed_form(N, s.rho)
    want = s.sign[:, None] * s.sign[None, :] * G[np.ix_(dof, dof)]
    got = oracle.schur(s)
    assert oracle.relF(got, want) < 1e-15


# ---------------------------------------------------------------- independent routes

@pytest.mark.parametrize("case", range(6))
def test_matches_dense_lu(case):
    s = _small_cases()[case]
    assert oracle.relF(oracle.schur(s), oracle.brute_F(s)) < 1e-13


@pytest.mark.parametrize("case", range(6))
def test_matches_saddle_point_route(case):
    # -F is the Schur complement of [[K_reg, B^T], [B, 0]] (paper eq. (13))
    s = _small_cases()[case]
    assert oracle.relF(oracle.schur(s), oracle.saddle_F(s)) < 1e-11


@pytest.mark.parametrize("case", range(6))
def test_projected_invariance_moore_penrose(case):
    # any two generalised inverses give the same P_G F P_G, G = B R
    s = _small_cases()[case]
    P = oracle.projector(oracle.gluing_G(s))
    F = oracle.schur(s)
    Fp = oracle.pinv_F(s)
    assert oracle.relF(P @ F @ P, P @ Fp @ P) < 1e-11


def _heat3d_spectral_F(s):
    """B G B^T with the generalised inverse G = V3 Lambda^+ V3^T of the Kronecker-sum
    grid operator K = Kz(x)My(x)Mx + ..., built from the 1D generalised eigenproblem
    K1 V = M1 V D (scipy), without any factorisation of K."""
    N = s.elems[0]
    assert s.elems == (N, N, N)
    h = s.h
    n1 = N + 1
    K1 = np.zeros((n1, n1))
    M1 = np.zeros((n1, n1))
    for e in range(N):
        K1[e:e + 2, e:e + 2] += np.array([[1, -1], [-1, 1]]) / h
        M1[e:e + 2, e:e + 2] += np.array([[2, 1], [1, 2]]) * h / 6
    D, V = scipy.linalg.eigh(K1, M1)
    D[0] = 0.0                                   # constant mode
    lam = (D[:, None, None] + D[None, :, None] + D[None, None, :]).ravel()   # (z, y, x)
    inv = np.where(lam > 1e-9 * lam.max(), 1.0 / np.where(lam == 0, 1, lam), 0.0)
    node = s.dof
    ix = node % n1
    iy = (node // n1) % n1
    iz = node // (n1 * n1)
    W = (V[iz][:, :, None, None] * V[iy][:, None, :, None] * V[ix][:, None, None, :]).reshape(len(node), -1)
    W *= s.sign[:, None]
    return (W * inv[None, :]) @ W.T


def test_projected_invariance_spectral_full_heat_workload():
    s = scgen.config_subdomains(2, count=1)[0]          # 12^3 heat, n = 2197, m = 866
    P = oracle.projector(oracle.gluing_G(s))
    F = oracle.schur(s)
    Fs = _heat3d_spectral_F(s)
    assert oracle.relF(P @ F @ P, P @ Fs @ P) < 1e-12


# ---------------------------------------------------------------- residuals / invariants

@pytest.mark.parametrize("case", range(6))
def test_factor_and_forward_residuals(case):
    s = _small_cases()[case]
    L = oracle.cholesky_dense(s)
    K = s.Kreg_csr().toarray()
    assert np.abs(np.triu(L, 1)).max() == 0
    assert np.linalg.norm(L @ L.T - K) / np.linalg.norm(K) < 1e-15
    F, Y = oracle.schur(s, want_Y=True)
    Bt = s.Bt_dense()
    assert np.linalg.norm(L @ Y - Bt) / np.linalg.norm(Bt) < 1e-14
    # K_reg Z = B^T with Z = L^{-T} Y
    Z = scipy.linalg.solve_triangular(L.T, Y, lower=False)
    assert np.linalg.norm(K @ Z - Bt) / np.linalg.norm(Bt) < 1e-11


@pytest.mark.parametrize("case", range(6))
def test_symmetric_positive_definite(case):
    s = _small_cases()[case]
    F = oracle.schur(s)
    assert np.array_equal(F, F.T)
    w = np.linalg.eigvalsh(F)
    assert w.min() > 0                     # distinct DOFs -> F is SPD


def test_per_face_gluing_is_psd_singular():
    s = scgen.box_subdomain("elasticity", (2, 2, 2), 0.5, seed=5, gluing="per_face")
    F = oracle.schur(s)
    w = np.linalg.eigvalsh(F)
    assert w.min() > -1e-12 * w.max()
    assert w.min() < 1e-10 * w.max()       # repeated DOFs -> dependent columns


def test_sign_flip_is_exact():
    s = scgen.box_subdomain("heat", (4, 4, 4), 0.25, seed=21)
    F = oracle.schur(s)
    flip = signs_from_seed(99, s.m)
    F2 = oracle.schur(s.with_signs(s.sign * flip))
    S = flip.astype(float)
    assert np.array_equal(F2, S[:, None] * F * S[None, :])


def test_column_permutation_is_exact():
    s = scgen.box_subdomain("elasticity", (2, 3, 2), 0.5, seed=22)
    F = oracle.schur(s)
    perm = np.random.default_rng(0).permutation(s.m)
    F2 = oracle.schur(s.with_columns(s.dof[perm], s.sign[perm]))
    assert np.array_equal(F2, F[np.ix_(perm, perm)])


def test_column_subset_matches_full():
    s = scgen.box_subdomain("heat", (5, 4, 4), 0.25, seed=23)
    F = oracle.schur(s)
    sel = np.array([7, 3, 50, 0, s.m - 1])
    assert np.array_equal(oracle.schur(s, sel=sel), F[np.ix_(sel, sel)])


def test_double_close_to_long_double():
    s = scgen.config_subdomains(1)[0]
    assert oracle.relF(oracle.schur(s, prec="d"), oracle.schur(s)) < 1e-14


def test_not_spd_reported():
    s = scgen.box_subdomain("heat", (3, 3), 0.3, seed=1)
    with pytest.raises(oracle.OracleError):
        oracle.schur_csr(s.n, s.k_rowptr, s.k_col, s.k_val, s.dof, s.sign)   # singular K


# ---------------------------------------------------------------- mutation coverage

def _pins_pass(mutation):
    """True when every cheap pin still passes with the planted mistake."""
    cases = [scgen.laplace_1d(20, dof=np.array([0, 5, 20, 11], dtype=np.int32), seed=3),
             scgen.box_subdomain("heat", (3, 4, 3), 0.25, seed=31),
             scgen.box_subdomain("elasticity", (2, 2, 3), 0.5, seed=32)]
    try:
        for s in cases:
            F = oracle.schur(s, mutation=mutation)
            if s.kind == "laplace1d":
                G = _laplace_inverse_closed_form(20, s.rho)
                want = s.sign[:, None] * s.sign[None, :] * G[np.ix_(s.dof, s.dof)]
                if oracle.relF(F, want) > 1e-13:
                    return False
            if oracle.relF(F, oracle.brute_F(s)) > 1e-12:
                return False
    except oracle.OracleError:
        return False
    return True


@pytest.mark.parametrize("mutation", [m for m in oracle.MUTATIONS if m != "none"])
def test_each_planted_mistake_is_caught(mutation):
    assert _pins_pass("none")
    assert not _pins_pass(mutation)


def test_large_golden_sample_reproduces():
    """The stored F[S, S] sample of the 20^3 elasticity subdomain (written by
    tests/golden/make_golden.py) is what the oracle computes, and it is
    symmetric with a positive diagonal."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "elast3d_hex8_20cube_F_sample.txt")
    with open(path) as f:
        f.readline()
        sel = np.array([int(v) for v in f.readline().split()], dtype=np.int64)
    F = np.loadtxt(path, comments="#", skiprows=2).reshape(len(sel), len(sel), order="F")
    assert np.array_equal(F, F.T) and np.all(np.diag(F) > 0)
    s = scgen.config_subdomains(5, count=1)[0]
    assert oracle.relF(oracle.schur(s, sel=sel), F) < 1e-16


def test_golden_fixture_reproduces():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "heat2d_q1_16x16_F.txt")
    vals = np.loadtxt(path, comments="#")
    s = scgen.config_subdomains(1)[0]
    F = vals.reshape(s.m, s.m, order="F")
    assert oracle.relF(oracle.schur(s), F) < 1e-16
    assert oracle.relF(oracle.brute_F(s), F) < 1e-13
