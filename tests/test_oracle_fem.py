"""Pins for the oracle's mesh, coefficient and P1 matrices (section 2.3).

Each check compares against something other than the oracle's own formula:
closed-form integrals, the textbook five-point stencil, and an independent
quadrature of piecewise-linear functions.
"""

import math

import numpy as np
import pytest

from oracle import coeff, fem, mesh
from synth import coeff_family, problem1_family


def _nodal(n, f):
    x, y = mesh.node_coords(n)
    return f(x, y)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_constant_coefficient_is_five_point_laplacian(n):
    # textbook: P1 on right-isosceles "/" triangles reproduces the 5-point stencil
    A = fem.stiffness(n, np.ones(2 * n * n)).toarray()
    m = n - 1
    T = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    L5 = np.kron(np.eye(m), T) + np.kron(T, np.eye(m))
    assert np.array_equal(A, L5)


def test_single_element_stiffness_is_right_triangle_matrix():
    # one element with a = 1, all others a = 0: the right-triangle element
    # matrix with the right angle at the middle vertex of the lower triangle
    n = 3
    aK = np.zeros(2 * n * n)
    e = 2 * (1 * n + 1)                      # lower triangle of square (1,1)
    aK[e] = 1.0
    A = fem.stiffness(n, aK, full=True).toarray()
    v = mesh.elements(n)[e]                  # (1,1), (2,1), (2,2); right angle at (2,1)
    K = A[np.ix_(v, v)]
    expect = np.array([[0.5, -0.5, 0.0], [-0.5, 1.0, -0.5], [0.0, -0.5, 0.5]])
    assert np.allclose(K, expect, atol=1e-15)
    assert abs(A.sum()) < 1e-14 and np.count_nonzero(np.abs(A) > 0) == 7


@pytest.mark.parametrize("n", [4, 8, 16])
def test_mass_integrates_quadratics_exactly(n):
    M = fem.mass(n, full=True)
    one = np.ones(M.shape[0])
    x = _nodal(n, lambda x, y: x)
    y = _nodal(n, lambda x, y: y)
    assert abs(one @ M @ one - 1.0) < 1e-14          # area of the unit square
    assert abs(one @ M @ x - 0.5) < 1e-14            # int x
    assert abs(x @ M @ x - 1.0 / 3.0) < 1e-14        # int x^2
    assert abs(x @ M @ y - 0.25) < 1e-14             # int x y


@pytest.mark.parametrize("n", [4, 8])
def test_forms_match_independent_quadrature(n):
    # f^T M g and f^T A(a) g against edge-midpoint quadrature of the piecewise
    # linear interpolants and their leg-difference gradients
    rng = np.random.default_rng(5)
    N = (n + 1) ** 2
    f, g = rng.standard_normal(N), rng.standard_normal(N)
    aK = 0.5 + rng.random(2 * n * n)
    el = mesh.elements(n)
    h = 1.0 / n
    mm, aa = 0.0, 0.0
    for e, (p0, p1, p2) in enumerate(el):
        area = 0.5 * h * h
        fm = [(f[p0] + f[p1]) / 2, (f[p1] + f[p2]) / 2, (f[p2] + f[p0]) / 2]
        gm = [(g[p0] + g[p1]) / 2, (g[p1] + g[p2]) / 2, (g[p2] + g[p0]) / 2]
        mm += area * sum(a * b for a, b in zip(fm, gm)) / 3.0
        if e % 2 == 0:   # lower: (i,j),(i+1,j),(i+1,j+1): x-leg p0->p1, y-leg p1->p2
            gf = ((f[p1] - f[p0]) / h, (f[p2] - f[p1]) / h)
            gg = ((g[p1] - g[p0]) / h, (g[p2] - g[p1]) / h)
        else:            # upper: (i,j),(i+1,j+1),(i,j+1): y-leg p0->p2, x-leg p2->p1
            gf = ((f[p1] - f[p2]) / h, (f[p2] - f[p0]) / h)
            gg = ((g[p1] - g[p2]) / h, (g[p2] - g[p0]) / h)
        aa += aK[e] * area * (gf[0] * gg[0] + gf[1] * gg[1])
    M = fem.mass(n, full=True)
    A = fem.stiffness(n, aK, full=True)
    assert abs(f @ M @ g - mm) < 1e-12 * max(1.0, abs(mm))
    assert abs(f @ A @ g - aa) < 1e-12 * max(1.0, abs(aa))


def test_stiffness_energy_of_linear_function():
    n = 8
    A = fem.stiffness(n, np.full(2 * n * n, 2.5), full=True)
    f = _nodal(n, lambda x, y: 3.0 * x - 2.0 * y + 1.0)
    assert abs(f @ A @ f - 2.5 * (9.0 + 4.0)) < 1e-12     # int a |grad f|^2
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) < 1e-13  # constants in the kernel


def test_interior_mass_stencil_and_restriction():
    n = 6
    M = fem.mass(n).toarray()
    h2 = 1.0 / n ** 2
    m = n - 1
    c = (3 - 1) * m + (3 - 1)   # interior node (3,3)
    row = M[c]
    assert abs(row[c] - h2 / 2) < 1e-16
    for d in (1, -1, m, -m, m + 1, -(m + 1)):
        assert abs(row[c + d] - h2 / 12) < 1e-16
    assert np.count_nonzero(row) == 7


@pytest.mark.parametrize("k1,k2", [(1, 2), (3, 1), (2, 2)])
def test_centroid_coefficient_moments(k1, k2):
    # centroid rule vs closed-form integrals of sin(k1 pi x) sin(k2 pi y) and of
    # x * sin(k1 pi x) sin(k2 pi y): pins the centroid positions and the x/y roles
    n = 64
    fam = {"a0": 0.0, "c": np.array([1.0]), "k1": np.array([k1]), "k2": np.array([k2])}
    a = coeff.coefficient(n, [1.0], fam)
    xc, _ = mesh.centroids(n)
    area = 0.5 / n ** 2
    Ix = (1 - (-1) ** k1) / (k1 * math.pi)
    Iy = (1 - (-1) ** k2) / (k2 * math.pi)
    Jx = (-1) ** (k1 + 1) / (k1 * math.pi)          # int_0^1 x sin(k pi x) dx
    assert abs(area * a.sum() - Ix * Iy) < 5e-3 * max(abs(Ix * Iy), 1e-3) + 1e-4
    assert abs(area * (xc * a).sum() - Jx * Iy) < 5e-3 * max(abs(Jx * Iy), 1e-3) + 1e-4


def test_centroids_are_triangle_centroids():
    n = 4
    xc, yc = mesh.centroids(n)
    h = 1.0 / n
    # square (1,2): lower centroid ((i+2/3)h, (j+1/3)h), upper ((i+1/3)h, (j+2/3)h)
    e = 2 * (2 * n + 1)
    assert np.allclose([xc[e], yc[e]], [(1 + 2 / 3) * h, (2 + 1 / 3) * h])
    assert np.allclose([xc[e + 1], yc[e + 1]], [(1 + 1 / 3) * h, (2 + 2 / 3) * h])


def test_family_tables():
    fam = coeff_family(16)
    pairs = list(zip(fam["k1"].tolist(), fam["k2"].tolist()))
    assert pairs[:6] == [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1)]
    norms = [a * a + b * b for a, b in pairs]
    assert norms == sorted(norms)
    assert len(set(pairs)) == 16
    assert abs(fam["c"][3] - 4 ** -2.5) < 1e-16
    p1 = problem1_family(4, 4.0 / 3.0)
    assert abs(p1["a0"] - math.pi / math.sqrt(2)) < 1e-15
    assert p1["k1"].tolist() == [1, 2, 3, 4] and p1["k2"].tolist() == [2, 3, 4, 5]


def test_coefficient_bounds_hold():
    fam = coeff_family(16)
    lo, hi = coeff.bounds(fam, 16)
    rng = np.random.default_rng(1)
    for _ in range(5):
        a = coeff.coefficient(16, rng.random(16) - 0.5, fam)
        assert lo <= a.min() and a.max() <= hi
    assert lo > 0.3   # 1 - zeta(2.5)/2 = 0.3293...
