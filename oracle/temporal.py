"""Upwind DG(q) in time on one slab (Sec. 2, Defs. DG notation and temporal
discretisation, eq. dgintime).

Reading of the paper (it does not name the temporal nodes): by default the
Lagrange basis of each slab sits on the right Gauss-Radau points of [0, 1]
(q=0: {1}; q=1: {1/3, 1}), so the slab end value is the last nodal value.
The nodes also fix where the Dirichlet data is interpolated in time, the only
place they change the discrete solution; the Gauss-Legendre points
(nodes="gauss") are the other family offered (with them the Chorin error table
of Sec. 4.2 is reproduced).  The +/- limit
notation of the paper's definition is read in the standard upwind sense:
psi_n^+ is the value at t_n from inside slab n, Y_n^- the value at t_n from
inside slab n-1 (this is what makes the space-time system block lower
bidiagonal, eq. waveform_patch_solve).
"""
import numpy as np
from numpy.polynomial import legendre as L

from .quadrature import gauss_01


def radau_right_nodes(q):
    """q+1 right Gauss-Radau points on [0, 1] (roots of P_{q+1} - P_q, mapped)."""
    if q == 0:
        return np.array([1.0])
    c = np.zeros(q + 2)
    c[q + 1] = 1.0
    c[q] = -1.0
    r = np.sort(np.real(L.legroots(c)))
    r[-1] = 1.0
    return 0.5 * (r + 1.0)


def lagrange(nodes, s):
    """Values and derivatives of the Lagrange basis on ``nodes`` at points s.

    Returns (phi, dphi) of shape (len(s), len(nodes)).
    """
    s = np.atleast_1d(np.asarray(s, dtype=float))
    m = len(nodes)
    phi = np.ones((len(s), m))
    dphi = np.zeros((len(s), m))
    for a in range(m):
        others = [nodes[b] for b in range(m) if b != a]
        den = np.prod([nodes[a] - o for o in others]) if others else 1.0
        for k in range(len(s)):
            phi[k, a] = np.prod([s[k] - o for o in others]) / den
            tot = 0.0
            for skip in range(len(others)):
                tot += np.prod([s[k] - o for i, o in enumerate(others) if i != skip])
            dphi[k, a] = tot / den
    return phi, dphi


class SlabBasis:
    """Temporal reference data of one slab of DG(q).

    Attributes: nodes, Gauss rule (sg, wg) with q+3 points, Phi/dPhi at the
    Gauss points (G, q+1), e0 = phi(0), e1 = phi(1), and the reference
    matrices T_ab = int phi_b' phi_a + phi_b(0) phi_a(0) and W_ab = int phi_a phi_b.
    """

    def __init__(self, q, nodes="radau"):
        self.q = q
        if nodes == "radau":
            self.nodes = radau_right_nodes(q)
        elif nodes == "gauss":
            self.nodes = gauss_01(q + 1)[0]
        else:
            raise ValueError(f"unknown temporal nodes {nodes!r}")
        self.sg, self.wg = gauss_01(q + 3)
        self.Phi, self.dPhi = lagrange(self.nodes, self.sg)
        self.e0 = lagrange(self.nodes, [0.0])[0][0]
        self.e1 = lagrange(self.nodes, [1.0])[0][0]
        self.W = np.einsum("g,ga,gb->ab", self.wg, self.Phi, self.Phi)
        self.T = (np.einsum("g,ga,gb->ab", self.wg, self.Phi, self.dPhi)
                  + np.outer(self.e0, self.e0))
