"""Reference-triangle Lagrange bases (Sec. 2, Taylor-Hood P2-P1 at k=1).

Reference triangle (0,0), (1,0), (0,1); barycentrics l0 = 1 - xi - eta,
l1 = xi, l2 = eta.  P2 order: three vertex functions l_i (2 l_i - 1), then the
edge functions 4 l1 l2, 4 l0 l2, 4 l0 l1 (edge opposite vertex 0, 1, 2).
"""
import numpy as np

P2_NODES = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0],
                     [0.5, 0.5], [0.0, 0.5], [0.5, 0.0]])


def bary(pts):
    pts = np.atleast_2d(pts)
    xi, eta = pts[:, 0], pts[:, 1]
    return np.stack([1.0 - xi - eta, xi, eta], axis=1)


# d l_i / d(xi, eta)
_DL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])


def p1(pts):
    """P1 values (n, 3) and reference gradients (n, 3, 2)."""
    lam = bary(pts)
    g = np.broadcast_to(_DL, (lam.shape[0], 3, 2)).copy()
    return lam, g


def p2(pts):
    """P2 values (n, 6) and reference gradients (n, 6, 2)."""
    lam = bary(pts)
    n = lam.shape[0]
    val = np.empty((n, 6))
    grad = np.empty((n, 6, 2))
    for i in range(3):
        val[:, i] = lam[:, i] * (2.0 * lam[:, i] - 1.0)
        grad[:, i, :] = np.outer(4.0 * lam[:, i] - 1.0, _DL[i])
    for k, (i, j) in enumerate([(1, 2), (0, 2), (0, 1)]):
        val[:, 3 + k] = 4.0 * lam[:, i] * lam[:, j]
        grad[:, 3 + k, :] = 4.0 * (np.outer(lam[:, j], _DL[i]) + np.outer(lam[:, i], _DL[j]))
    return val, grad
