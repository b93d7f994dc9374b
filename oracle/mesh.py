"""Uniform triangulation of D = (0,1)^2 with mesh width h = 1/n.

Section 2.3 asks for a shape-regular triangulation; the numerical section uses
uniform meshes with h_l = 2^-(l+3).  Reading fixed here: every square
[i h, (i+1) h] x [j h, (j+1) h] is cut by its "/" diagonal (south-west to
north-east) into

    lower triangle  (i,j), (i+1,j),   (i+1,j+1)   element 2*(j*n+i)
    upper triangle  (i,j), (i+1,j+1), (i,j+1)     element 2*(j*n+i)+1

so meshes are nested under halving.  Nodes of the full mesh are numbered
g = j*(n+1) + i, 0 <= i, j <= n; interior nodes (1 <= i, j <= n-1) are
numbered (j-1)*(n-1) + (i-1), x fastest.
"""

from __future__ import annotations

import numpy as np


def n_interior(n: int) -> int:
    return (n - 1) * (n - 1)


def node_coords(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Coordinates of all (n+1)^2 nodes, global numbering."""
    i = np.arange(n + 1)
    I, J = np.meshgrid(i, i, indexing="xy")
    return (I.ravel() / n).astype(np.float64), (J.ravel() / n).astype(np.float64)


def elements(n: int) -> np.ndarray:
    """Vertex triples (global node numbers) of the 2 n^2 elements, int64[2n^2, 3]."""
    out = np.empty((2 * n * n, 3), dtype=np.int64)
    for j in range(n):
        for i in range(n):
            g00 = j * (n + 1) + i
            g10 = g00 + 1
            g01 = g00 + (n + 1)
            g11 = g01 + 1
            e = 2 * (j * n + i)
            out[e] = (g00, g10, g11)
            out[e + 1] = (g00, g11, g01)
    return out


def centroids(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Element centroids, ordered as ``elements``."""
    x, y = node_coords(n)
    el = elements(n)
    return x[el].mean(axis=1), y[el].mean(axis=1)


def interior_map(n: int) -> np.ndarray:
    """For each global node, its interior number or -1 on the boundary."""
    m = np.full((n + 1) * (n + 1), -1, dtype=np.int64)
    for j in range(1, n):
        for i in range(1, n):
            m[j * (n + 1) + i] = (j - 1) * (n - 1) + (i - 1)
    return m
