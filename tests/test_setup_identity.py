"""The identity behind the coarse-side set-up products of the batched path
(k_sep_setup_dots): for v = P u_H on nested P1 meshes with the "/" diagonal,

    v^T A_h v = sum over coarse triangles T of |grad u_H|_T^2 (h^2/2) sum_{K in T} a_K,
    v^T M_h v = u_H^T M_H u_H,

with a_K the coefficient at the centroid of fine element K, and the sums over T
formed, as the kernel forms them, from the separable row sums U and interval
sums of the sine table S.  Host-side check in numpy of the formula and its
index bookkeeping (grid of thirds, lower / upper elements, the diagonal
squares), against the edge-weight form of the stiffness (mean of the two
element values per edge; section 2.3, eq. fe-evp) and the element form."""

import numpy as np
import pytest


def _case(n, nH, kx, ky, seed):
    rng = np.random.default_rng(seed)
    a0 = 1.3
    r = n // nH
    M = 3 * n + 2
    C = rng.standard_normal((kx, ky)) * 0.2
    m = np.arange(M)
    S = np.sin(np.pi * np.outer(np.arange(1, max(kx, ky) + 1), m) / (3 * n))  # [k x M]
    U = (C @ S[:ky]).T                                                          # [M x kx]
    uH = np.zeros((nH + 1, nH + 1))
    uH[1:nH, 1:nH] = rng.standard_normal((nH - 1, nH - 1))
    return a0, r, M, S[:kx], U, uH


def _prolong(uH, n, r):
    nH = uH.shape[0] - 1
    V = np.zeros((n + 1, n + 1))
    for i in range(n + 1):
        for j in range(n + 1):
            A, B, li, lj = min(i // r, nH - 1), min(j // r, nH - 1), 0, 0
            li, lj = i - r * A, j - r * B
            xi, eta = li / r, lj / r
            u00, u11 = uH[A, B], uH[A + 1, B + 1]
            if lj <= li:
                V[i, j] = u00 + xi * (uH[A + 1, B] - u00) + eta * (u11 - uH[A + 1, B])
            else:
                V[i, j] = u00 + eta * (uH[A, B + 1] - u00) + xi * (u11 - uH[A, B + 1])
    return V


@pytest.mark.parametrize("n,nH,kx,ky", [(32, 8, 4, 3), (64, 16, 5, 4), (64, 8, 3, 5)])
def test_coarse_setup_products(n, nH, kx, ky):
    a0, r, M, S, U, uH = _case(n, nH, kx, ky, seed=n + nH + kx)
    V = _prolong(uH, n, r)
    acent = lambda mx, my: a0 + S[:, mx] @ U[my]
    # edge form: horizontal edge (i-1, j)-(i, j), vertical (i, j-1)-(i, j), each
    # weighted by the mean of its two elements (grid-of-thirds centroids)
    fine = 0.0
    for j in range(1, n):
        for i in range(1, n + 1):
            w = a0 + 0.5 * (S[:, 3 * i - 2] @ U[3 * j - 1] + S[:, 3 * i - 1] @ U[3 * j + 1])
            fine += w * (V[i, j] - V[i - 1, j]) ** 2
    for j in range(1, n + 1):
        for i in range(1, n):
            w = a0 + 0.5 * (S[:, 3 * i - 1] @ U[3 * j - 2] + S[:, 3 * i + 1] @ U[3 * j - 1])
            fine += w * (V[i, j] - V[i, j - 1]) ** 2
    # element form: lower (a,b),(a+1,b),(a+1,b+1), upper (a,b),(a+1,b+1),(a,b+1)
    elem = 0.0
    for a in range(n):
        for b in range(n):
            gl = (V[a + 1, b] - V[a, b]) ** 2 + (V[a + 1, b + 1] - V[a + 1, b]) ** 2
            gu = (V[a + 1, b + 1] - V[a, b + 1]) ** 2 + (V[a, b + 1] - V[a, b]) ** 2
            elem += 0.5 * (acent(3 * a + 2, 3 * b + 1) * gl + acent(3 * a + 1, 3 * b + 2) * gu)
    # coarse form: interval sums Tp [3 r kx x 2 nH] against the U rows of each coarse row
    K, NC = 3 * r * kx, 2 * nH
    Tp = np.zeros((K, NC))
    for k in range(K):
        beta, e, p = k // (3 * kx), (k // kx) % 3, k % kx
        for col in range(NC):
            A, upper = col % nH, col // nH
            if e == 1:
                off, lo, hi = 2, (0 if upper else beta), (beta if upper else r)
            elif e == 2:
                off, lo, hi = 1, (0 if upper else beta + 1), (beta + 1 if upper else r)
            else:
                continue
            Tp[k, col] = sum(S[p, 3 * (r * A + al) + off] for al in range(lo, hi))
    coarse = 0.0
    for Bc in range(nH):
        Csum = U[3 * r * Bc: 3 * r * (Bc + 1)].reshape(-1) @ Tp
        for A in range(nH):
            dl = (uH[A + 1, Bc] - uH[A, Bc]) ** 2 + (uH[A + 1, Bc + 1] - uH[A + 1, Bc]) ** 2
            du = (uH[A + 1, Bc + 1] - uH[A, Bc + 1]) ** 2 + (uH[A, Bc + 1] - uH[A, Bc]) ** 2
            coarse += dl * (r * r * a0 + Csum[A]) + du * (r * r * a0 + Csum[nH + A])
    coarse /= 2.0 * r * r
    assert abs(elem - fine) <= 1e-12 * fine
    assert abs(coarse - fine) <= 1e-12 * fine

    def m12(X, N):
        x = X[1:N, 1:N]
        return float(np.sum(x * (6 * x + X[0:N - 1, 1:N] + X[2:N + 1, 1:N] + X[1:N, 0:N - 1] +
                                 X[1:N, 2:N + 1] + X[2:N + 1, 2:N + 1] + X[0:N - 1, 0:N - 1])))
    # the mass stencil on the fine mesh against r^2 times the coarse one (the
    # scale h^2 / 12 against H^2 / 12)
    assert abs(m12(V, n) - r * r * m12(uH, nH)) <= 1e-12 * m12(V, n)


def test_identity_fails_with_a_swapped_element():
    # a plausible slip (the upper element's centroid taken for the lower one)
    # must break the identity, so the test above can tell
    n, nH, kx, ky = 32, 8, 4, 3
    a0, r, M, S, U, uH = _case(n, nH, kx, ky, seed=5)
    V = _prolong(uH, n, r)
    good = bad = 0.0
    for a in range(n):
        for b in range(n):
            gl = (V[a + 1, b] - V[a, b]) ** 2 + (V[a + 1, b + 1] - V[a + 1, b]) ** 2
            lo = a0 + S[:, 3 * a + 2] @ U[3 * b + 1]
            up = a0 + S[:, 3 * a + 1] @ U[3 * b + 2]
            good += 0.5 * lo * gl
            bad += 0.5 * up * gl
    assert abs(good - bad) > 1e-6 * abs(good)
