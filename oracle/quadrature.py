"""Triangle quadrature exact for polynomials (oracle; test infrastructure only).

The column basis of the interpolation H2 matrix (Section 4) integrates a hat
function times the normal derivative of a tensor Lagrange polynomial over flat
triangles.  The integrand is a polynomial, so an exact rule gives the exact
integral.  Here: the Duffy collapse of the unit square onto the reference
triangle {u, v >= 0, u + v <= 1}, v = (1 - u) w, with Gauss-Legendre nodes in
u and w (numpy's leggauss).  A polynomial of total degree d becomes degree
d + 1 in u (Jacobian factor 1 - u) and degree d in w, so n = ceil((d + 2)/2)
points per direction integrate it exactly.
"""
from __future__ import annotations

import numpy as np


def triangle_rule(degree: int):
    """Points (Q x 2, reference coordinates (u, v)) and weights (Q) summing to 1/2."""
    n = (degree + 3) // 2                          # ceil((degree + 2) / 2)
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    U, Wg = np.meshgrid(g, g, indexing="ij")
    wu, ww = np.meshgrid(w, w, indexing="ij")
    u = U.ravel()
    v = (1.0 - u) * Wg.ravel()
    wt = (wu * ww).ravel() * (1.0 - u)
    return np.stack([u, v], axis=1), wt
