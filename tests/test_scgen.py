"""Pins of the seeded input generator: element closed forms, kernels, counts."""
import numpy as np
import pytest

import scgen
from scgen import mesh
from scgen.rng import MASK64, splitmix64


def _splitmix64_reference(seed, count):
    """Scalar SplitMix64, one output per call of next() (Vigna's definition)."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


@pytest.mark.parametrize("seed", [0, 1, 250921038, MASK64])
def test_splitmix_counter_form_matches_sequential(seed):
    assert [int(v) for v in splitmix64(seed, 37)] == _splitmix64_reference(seed, 37)
    assert [int(v) for v in splitmix64(seed, 5, start=30)] == _splitmix64_reference(seed, 35)[30:]


def test_q1_heat_element_textbook():
    # bilinear square, Laplace: diag 2/3, edge neighbours -1/6, opposite corner -1/3
    expect = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.allclose(mesh.q1_heat_element(), expect, rtol=0, atol=1e-15)


def test_hex8_heat_element_closed_form():
    h = 0.25
    ke = mesh.hex8_heat_element(h)
    corners = [(x, y, z) for z in (0, 1) for y in (0, 1) for x in (0, 1)]
    for a, ca in enumerate(corners):
        for b, cb in enumerate(corners):
            d = sum(int(u != v) for u, v in zip(ca, cb))
            want = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[d] * h
            assert abs(ke[a, b] - want) < 1e-15


def test_hex8_elasticity_element_entries():
    # u_x-u_x at one node: h (lambda + 4 mu) / 9; u_x-u_y at one node: h (lambda + mu) / 12
    E, nu, h = 1.0, 0.3, 0.5
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    ke = mesh.hex8_elasticity_element(h, E, nu)
    assert abs(ke[0, 0] - h * (lam + 4 * mu) / 9) < 1e-14
    assert abs(ke[0, 1] - h * (lam + mu) / 12) < 1e-14
    w = np.linalg.eigvalsh(ke)
    assert np.sum(np.abs(w) < 1e-12) == 6 and w.min() > -1e-12


def test_kernels_and_symmetry():
    s = scgen.box_subdomain("heat", (3, 4, 5), 0.2, seed=1)
    K = s.K_csr()
    assert abs(K - K.T).max() == 0
    assert np.abs(K @ np.ones(s.n)).max() < 1e-14
    e = scgen.box_subdomain("elasticity", (3, 2, 4), 0.25, seed=2)
    Ke = e.K_csr()
    assert abs(Ke - Ke.T).max() < 1e-16
    assert np.abs(Ke @ e.R).max() < 1e-13 * abs(Ke).max()


@pytest.mark.parametrize("kind,elems", [("heat", (4, 3)), ("heat", (3, 3, 4)), ("elasticity", (2, 3, 2))])
def test_regularised_inverse_is_generalised_inverse(kind, elems):
    # paper Sec. 2.1: K K^+ K = K with K^+ = K_reg^{-1} (Sec. 2.2, eq. (10))
    s = scgen.box_subdomain(kind, elems, 0.5, seed=3)
    K = s.K_csr().toarray()
    Kr = s.Kreg_csr().toarray()
    assert np.linalg.eigvalsh(Kr).min() > 0
    G = np.linalg.inv(Kr)
    assert np.abs(K @ G @ K - K).max() < 1e-11 * np.abs(K).max()


def test_multiplier_counts():
    assert scgen.config_subdomains(1)[0].m == 64
    assert scgen.config_subdomains(1)[0].n == 289
    s2 = scgen.config_subdomains(2, count=1)[0]
    assert (s2.n, s2.m) == (2197, 866)
    assert scgen.box_subdomain("elasticity", (6, 6, 6), 1 / 16, 0).m == 654
    assert scgen.box_subdomain("elasticity", (16, 16, 16), 1 / 16, 0).m == 4614
    s5 = scgen.box_subdomain("elasticity", (20, 20, 20), 1 / 20, 0, gluing="per_face")
    assert (s5.n, s5.m) == (27783, 7938)


def test_uneven_sizes_range_and_determinism():
    a = scgen.uneven_sizes(scgen.BASE_SEED + 3, 512)
    assert a.min() == 6 and a.max() == 16
    b = scgen.uneven_sizes(scgen.BASE_SEED + 3, 10, start=100)
    assert np.array_equal(a[100:110], b)
    # all eleven values appear on every axis
    for ax in range(3):
        assert set(a[:, ax].tolist()) == set(range(6, 17))


def test_signs_per_subdomain_differ_and_are_pm1():
    ss = scgen.config_subdomains(2, count=3)
    for s in ss:
        assert set(np.unique(s.sign).tolist()) == {-1, 1}
    assert not np.array_equal(ss[0].sign, ss[1].sign)


# ------------------------------------------------ P1 triangles / tetrahedra

def test_p1_triangle_closed_form():
    # right isosceles triangle, right angle at vertex 0: K = 1/2 [[2,-1,-1],[-1,1,0],[-1,0,1]]
    # for any leg length (the 2D Laplace stiffness is scale-free)
    for h in (1.0, 0.125):
        K = scgen.p1_stiffness(np.array([[0, 0], [h, 0], [0, h]]))
        assert np.allclose(K, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), rtol=0, atol=1e-15)


def test_p1_tetrahedron_closed_form():
    # corner tetrahedron of the unit cube: K = (1/6) [[3,-1,-1,-1],[-1,1,0,0],[-1,0,1,0],[-1,0,0,1]],
    # scaling like h in 3D
    for h in (1.0, 0.25):
        K = scgen.p1_stiffness(h * np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]))
        ref = h / 6 * np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]])
        assert np.allclose(K, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim,e", [(2, 6), (2, 9), (3, 4), (3, 5)])
def test_simplex_grids_give_the_finite_difference_stencils(dim, e):
    # P1 on the diagonal-split square grid is the 5-point Laplacian; on the
    # Kuhn subdivision of the cube grid it is h times the 7-point Laplacian
    # (the face- and body-diagonal couplings of the six tetrahedra cancel)
    s = scgen.simplex_subdomain(dim, e, seed=3)
    K = s.K_csr()
    npx = e + 1
    h = 1.0 / e
    scale = 1.0 if dim == 2 else h
    for c in range(s.n):
        idx = np.unravel_index(c, (npx,) * dim, order="F")
        if min(idx) == 0 or max(idx) == e:
            continue
        row = K.getrow(c)
        nb = sorted(row.indices.tolist())
        strides = [1, npx, npx * npx][:dim]
        expect = sorted([c] + [c + st for st in strides] + [c - st for st in strides])
        assert nb == expect
        assert np.isclose(row[0, c], 2 * dim * scale, rtol=1e-14)
        for st in strides:
            assert np.isclose(row[0, c + st], -scale, rtol=1e-14)
    assert np.abs(K @ np.ones(s.n)).max() <= 1e-13
    assert abs(K - K.T).max() == 0.0
    assert np.linalg.eigvalsh(K.toarray()).min() > -1e-12
    assert s.m == npx ** dim - (npx - 2) ** dim


def test_kuhn_tetrahedra_fill_the_cube():
    from scgen.simplex import _local_simplices
    vols = [abs(np.linalg.det((t[1:] - t[0]).astype(float))) / 6 for t in _local_simplices(3)]
    assert np.allclose(vols, 1 / 6) and abs(sum(vols) - 1.0) < 1e-15


@pytest.mark.parametrize("dim,e", [(2, 5), (3, 3)])
def test_simplex_regularised_inverse_is_generalised_inverse(dim, e):
    s = scgen.simplex_subdomain(dim, e, seed=1)
    K = s.K_csr().toarray()
    Kr = s.Kreg_csr().toarray()
    X = np.linalg.solve(Kr, K)
    assert np.abs(K @ X - K).max() <= 1e-10 * np.abs(K).max()


def test_paper_batches_are_seeded_and_distinct():
    a = scgen.paper_subdomains(3, 9, count=3)
    b = scgen.paper_subdomains(3, 9, count=2, start=1)
    assert np.array_equal(a[1].sign, b[0].sign)
    assert not np.array_equal(a[0].sign, a[1].sign)
    assert a[0].n == 729 and a[0].m == 729 - 343
    assert scgen.paper_batch_size(3, 41) == 16 and scgen.paper_batch_size(2, 7) == 512
