"""Pins of the oracle's PCPG (paper, Sec. 2.1 eq. (7): the dual problem
[F -G; -G^T 0][lambda; alpha] = [d; -e], solved by projected conjugate
gradients; e = 0 here).  The paper cites PCPG without listing it, so the
iteration is checked against what the dual problem itself fixes:

  * lambda after enough iterations equals the solution of one dense LU solve
    of the saddle-point system (a route that shares nothing with the
    iteration but F, G and d);
  * the converged lambda satisfies the constraint G^T lambda = e = 0 and the
    projected equation P (d - F lambda) = 0;
  * the first recorded ||w_0|| is ||P d||.

Each planted mistake (projector skipped, beta from the unprojected residual,
alpha inverted, update with the wrong sign) fails the direct-solve pin.
"""
import numpy as np
import pytest

import oracle
import scgen


def _cases():
    """(name, F, G, d): a 16 x 16 Q1 heat square (k = 1) and the two smallest
    of the first 32 uneven elasticity boxes (subdomains 27 and 0: n = 1323 and
    1920, k = 6); F from the long-double oracle, d uniform in [-1, 1)."""
    out = []
    s1 = scgen.config_subdomains(1)[0]
    subs = [("heat2d_q1_16x16", s1)]
    for i in (27, 0):
        subs.append((f"elast_uneven_{i}", scgen.config_subdomains(3, count=1, start=i)[0]))
    for k, (name, s) in enumerate(subs):
        F = oracle.schur(s)
        G = oracle.gluing_G(s)
        d = scgen.splitmix64_uniform(scgen.BASE_SEED + 40 + k, s.m)
        out.append((name, F, G, d))
    return out


_CACHE = {}


def cases():
    if "c" not in _CACHE:
        _CACHE["c"] = _cases()
    return _CACHE["c"]


ITERS = 100


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("idx", range(3))
def test_pcpg_matches_direct_dual_solve(idx):
    name, F, G, d = cases()[idx]
    lam, hist = oracle.pcpg(F, G, d, ITERS)
    ref, alpha = oracle.dual_direct(F, G, d)
    assert _rel(lam, ref) <= 1e-10, name
    # constraint and projected equation of eq. (7)
    assert np.linalg.norm(G.T @ lam) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(lam), name
    P = oracle.projector(G)
    assert np.linalg.norm(P @ (d - F @ lam)) <= 1e-10 * np.linalg.norm(d), name
    # the multiplier of the constraint: F lambda - G alpha = d
    assert np.linalg.norm(F @ ref - G @ alpha - d) <= 1e-10 * np.linalg.norm(d), name
    assert abs(hist[0] - np.linalg.norm(P @ d)) <= 1e-13 * hist[0]


def test_direct_dual_solve_on_a_closed_form_case():
    # F = I (m x m), G = constant column: lambda = P d, alpha = -mean(d).
    m = 10
    F = np.eye(m)
    G = np.ones((m, 1))
    d = np.arange(m, dtype=np.float64) - 3.0
    lam, alpha = oracle.dual_direct(F, G, d)
    assert np.allclose(lam, d - d.mean(), rtol=0, atol=1e-14)
    assert np.allclose(alpha, [-d.mean()], rtol=0, atol=1e-14)
    # CG on the identity converges in one step
    lp, _ = oracle.pcpg(F, G, d, 1)
    assert np.allclose(lp, lam, rtol=0, atol=1e-14)


@pytest.mark.parametrize("mutation", [m for m in oracle.PCPG_MUTATIONS if m != "none"])
def test_each_planted_pcpg_mistake_is_caught(mutation):
    caught = False
    for name, F, G, d in cases():
        with np.errstate(all="ignore"):
            lam, _ = oracle.pcpg(F, G, d, ITERS, mutation=mutation)
        ref, _ = oracle.dual_direct(F, G, d)
        if not np.all(np.isfinite(lam)) or _rel(lam, ref) > 1e-6:
            caught = True
            break
    assert caught, mutation
