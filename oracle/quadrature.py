"""Quadrature rules (oracle).

Neither rule is fixed by the paper (it is silent on quadrature); the reading
used throughout is: Gauss-Legendre with q+3 points per time slab, and a 5x5
collapsed (Duffy) Gauss-Legendre rule on triangles, exact for polynomials of
total degree 8.  Nodes come from numpy's ``leggauss``.
"""
import numpy as np


def gauss_01(n):
    """n-point Gauss-Legendre rule on [0, 1]: (points, weights)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def duffy_triangle(n=5):
    """Collapsed rule on the reference triangle {xi, eta >= 0, xi + eta <= 1}.

    xi = u, eta = v (1 - u), weight w_u w_v (1 - u); u, v are n-point
    Gauss-Legendre points on [0, 1].  Returns (points (n*n, 2), weights (n*n,)).
    """
    u, wu = gauss_01(n)
    v, wv = gauss_01(n)
    U, V = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    xi = U.ravel()
    eta = (V * (1.0 - U)).ravel()
    w = (WU * WV * (1.0 - U)).ravel()
    return np.stack([xi, eta], axis=1), w
