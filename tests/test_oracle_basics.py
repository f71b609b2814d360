"""Oracle quadrature, temporal matrices and reference elements against closed
forms (Sec. 2 DG-in-time; Radau IIA equivalence noted in Sec. 4.1)."""
import math

import numpy as np
import pytest

from oracle import fe
from oracle.quadrature import duffy_triangle, gauss_01
from oracle.temporal import SlabBasis


def test_gauss_exactness():
    for n in (1, 2, 3, 4, 5):
        s, w = gauss_01(n)
        for d in range(2 * n):
            assert np.dot(w, s ** d) == pytest.approx(1.0 / (d + 1), rel=1e-14)


def test_duffy_exact_to_degree_8():
    x, w = duffy_triangle(5)
    for i in range(9):
        for j in range(9 - i):
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            assert np.dot(w, x[:, 0] ** i * x[:, 1] ** j) == pytest.approx(exact, rel=1e-13)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_temporal_integration_by_parts(q):
    tb = SlabBasis(q)
    assert np.allclose(tb.T + tb.T.T, np.outer(tb.e1, tb.e1) + np.outer(tb.e0, tb.e0), atol=1e-14)


def test_radau_nodes():
    assert np.allclose(SlabBasis(0).nodes, [1.0])
    assert np.allclose(SlabBasis(1).nodes, [1.0 / 3.0, 1.0])
    assert np.allclose(SlabBasis(2).nodes, [(4 - math.sqrt(6)) / 10, (4 + math.sqrt(6)) / 10, 1.0])


@pytest.mark.parametrize("nodes", ["radau", "gauss"])
@pytest.mark.parametrize("z", [-0.3, -2.0, -17.5, 0.4])
def test_dg_slab_map_is_radau_iia_stability_function(z, nodes):
    """y' = lam y over one slab with z = lam dt: the DG(q) end value is
    R(z) y0 with R the (q, q+1) Pade approximant (Radau IIA), whichever
    Lagrange nodes span the slab's polynomials."""
    r0 = SlabBasis(0, nodes)
    R0 = r0.e1 @ np.linalg.solve(r0.T - z * r0.W, r0.e0)
    assert R0 == pytest.approx(1.0 / (1.0 - z), rel=1e-13)
    r1 = SlabBasis(1, nodes)
    R1 = r1.e1 @ np.linalg.solve(r1.T - z * r1.W, r1.e0)
    assert R1 == pytest.approx((1 + z / 3) / (1 - 2 * z / 3 + z * z / 6), rel=1e-13)


def test_gauss_nodes():
    assert np.allclose(SlabBasis(0, "gauss").nodes, [0.5])
    assert np.allclose(SlabBasis(1, "gauss").nodes, [(3 - math.sqrt(3)) / 6, (3 + math.sqrt(3)) / 6])


def test_p2_basis_nodal_and_partition():
    val, grad = fe.p2(fe.P2_NODES)
    assert np.allclose(val, np.eye(6), atol=1e-15)
    pts = np.random.default_rng(0).uniform(0, 0.5, (20, 2))
    v, g = fe.p2(pts)
    assert np.allclose(v.sum(1), 1.0)
    assert np.allclose(g.sum(1), 0.0)
    eps = 1e-6
    for k in range(2):
        d = np.zeros(2)
        d[k] = eps
        fd = (fe.p2(pts + d)[0] - fe.p2(pts - d)[0]) / (2 * eps)
        assert np.allclose(fd, g[:, :, k], atol=1e-8)


def _bary_integral(alpha):
    """int over the reference triangle of l0^a l1^b l2^c = 2A a! b! c! / (a+b+c+2)!."""
    a, b, c = alpha
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)


def test_p2_mass_matrix_closed_form():
    """Mass matrix by quadrature against exact barycentric-monomial integration."""
    # each P2 function as a polynomial in barycentrics: dict exponent -> coeff
    polys = []
    for i in range(3):
        e2 = [0, 0, 0]; e2[i] = 2
        e1 = [0, 0, 0]; e1[i] = 1
        polys.append({tuple(e2): 2.0, tuple(e1): -1.0})
    for (i, j) in [(1, 2), (0, 2), (0, 1)]:
        e = [0, 0, 0]; e[i] += 1; e[j] += 1
        polys.append({tuple(e): 4.0})
    exact = np.zeros((6, 6))
    for a in range(6):
        for b in range(6):
            for ea, ca in polys[a].items():
                for eb, cb in polys[b].items():
                    exact[a, b] += ca * cb * _bary_integral(tuple(np.add(ea, eb)))
    x, w = duffy_triangle(5)
    v, _ = fe.p2(x)
    quad = np.einsum("q,qi,qj->ij", w, v, v)
    assert np.allclose(quad, exact, atol=1e-15)
    assert quad.sum() == pytest.approx(0.5)
