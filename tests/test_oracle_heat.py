"""The heat-equation oracle (Sec. 2 Definition of the heat equation, Sec. 4.1)
against closed forms: the P_k bases, exact integrals of polynomials, the
vertex-star patch sizes of Sec. 3.1, the DoF count formula, the DG(q) slab
map (Radau IIA stability function, for q up to 3) on the assembled
space-time system, convergence to the Fourier-series solution of the paper's
initial data, and the paper's three FGMRES-WRMG iterations."""
import math

import numpy as np
import pytest
import scipy.linalg as la
import scipy.sparse.linalg as spla

from oracle.heat import HeatLevel, HeatSpace, heat_solve, lagrange_pk, local_nodes
from test_oracle_counts import heat_dofs_formula


@pytest.mark.parametrize("k", [1, 2, 3])
def test_pk_basis_nodal_and_reproduces_polynomials(k):
    nod = np.array(local_nodes(k), dtype=float) / k
    val, grad = lagrange_pk(k, nod)
    assert np.allclose(val, np.eye(len(nod)), atol=1e-12)
    rng = np.random.default_rng(k)
    pts = rng.random((20, 2)) * 0.5
    val, grad = lagrange_pk(k, pts)
    assert np.allclose(val.sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(grad.sum(axis=1), 0.0, atol=1e-10)
    # x^a y^b with a + b = k is reproduced with its gradient
    for a in range(k + 1):
        b = k - a
        p = nod[:, 0] ** a * nod[:, 1] ** b
        assert np.allclose(val @ p, pts[:, 0] ** a * pts[:, 1] ** b, atol=1e-12)
        gx = a * pts[:, 0] ** max(a - 1, 0) * pts[:, 1] ** b if a else 0.0
        assert np.allclose(grad[:, :, 0] @ p, gx, atol=1e-10)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_mass_and_stiffness_are_exact(k):
    S = HeatSpace(4, k)
    Mm, Km = S.matrices()
    x, y = S.xy[:, 0], S.xy[:, 1]
    one = np.ones(S.n)
    assert one @ Mm @ one == pytest.approx(1.0, rel=1e-13)
    assert np.abs(Km @ one).max() < 1e-12
    p = x ** k + 0.5 * y ** k
    # int_0^1 int_0^1 (x^k + y^k / 2)^2 and |grad|^2
    ip2 = 1.0 / (2 * k + 1) * 1.25 + 1.0 / (k + 1) ** 2
    ig = k * k / (2 * k - 1) * 1.25
    assert p @ Mm @ p == pytest.approx(ip2, rel=1e-12)
    assert p @ Km @ p == pytest.approx(ig, rel=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_vertex_star_patches(k):
    S = HeatSpace(6, k)
    pats = S.patches()
    m = S.mesh
    n1 = m.n1
    interior = [v for v in range(m.nv) if 0 < v % n1 < n1 - 1 and 0 < v // n1 < n1 - 1]
    # Sec. 3.1: 3k^2 - 3k + 1 DoFs in the vertex star of an interior vertex
    assert {len(pats[v]) for v in interior} == {3 * k * k - 3 * k + 1}
    # every node belongs to at least one patch, vertices to exactly their own
    cover = np.zeros(S.n, dtype=int)
    for s in pats:
        cover[s] += 1
    assert cover.min() >= 1
    vlat = k * (np.arange(m.nv) % n1) + S.nl * k * (np.arange(m.nv) // n1)
    assert np.all(cover[vlat] == 1)
    assert S.n == heat_dofs_formula(7, k)


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_space_time_slab_map_is_radau_iia(q):
    """Sec. 4.1 notes DG(q) in time is Radau IIA for the heat equation.  On
    every generalized eigenvector of (K, M) the assembled space-time system
    advances the slab-end value by R(-lam dt), R the (q, q+1) Pade
    approximant of exp, the Radau IIA stability function."""
    def pade(z, kk, jj):
        f = math.factorial
        num = sum(f(kk + jj - i) * f(kk) / (f(kk + jj) * f(i) * f(kk - i)) * z ** i for i in range(kk + 1))
        den = sum(f(kk + jj - i) * f(jj) / (f(kk + jj) * f(i) * f(jj - i)) * (-z) ** i for i in range(jj + 1))
        return num / den
    lev = HeatLevel(2, 1, q, 5, 0.5, "gauss")
    b = lev.rhs()
    x = spla.spsolve(lev.A.tocsc(), b)
    ends = lev.end_values(x)
    lam, V = la.eigh(lev.Ks.toarray(), lev.Ms.toarray())
    U0 = np.sin(np.pi * lev.space.xy[:, 0]) + np.cos(2 * np.pi * lev.space.xy[:, 1])
    c = V.T @ (lev.Ms @ U0)
    for n in range(lev.N):
        pred = V @ (c * pade(-lam * lev.dt, q, q + 1) ** (n + 1))
        assert np.allclose(ends[n], pred, rtol=1e-10, atol=1e-12)


def exact_heat(t, x, y, terms=40):
    """Series solution of u_t = Laplace u, Neumann data, u_0 = sin(pi x) +
    cos(2 pi y): sin(pi x) = 2/pi - (4/pi) sum_j cos(2 j pi x) / (4 j^2 - 1)."""
    u = 2.0 / np.pi + np.cos(2 * np.pi * y) * np.exp(-4 * np.pi ** 2 * t)
    for j in range(1, terms + 1):
        u = u - 4.0 / np.pi * np.cos(2 * j * np.pi * x) * np.exp(-4 * j * j * np.pi ** 2 * t) / (4 * j * j - 1)
    return u


@pytest.mark.parametrize("k", [1, 2])
def test_converges_to_series_solution(k):
    errs = []
    for M in (4, 8):
        lev = HeatLevel(M, k, 1, 20, 0.02, "gauss")
        x = spla.spsolve(lev.A.tocsc(), lev.rhs())
        uT = lev.end_values(x)[-1]
        ex = exact_heat(0.02, lev.space.xy[:, 0], lev.space.xy[:, 1])
        errs.append(np.abs(uT - ex).max())
    assert errs[0] / errs[1] > 2 ** (k + 1) * 0.8


def test_paper_iteration_count_three():
    """Sec. 4.1: every FGMRES-WRMG heat solve takes 3 iterations (relative
    1e-6 or absolute 1e-6).  The oracle's solver takes 3 on a 40 x 40 mesh
    with three levels (coarsest 10 x 10, the paper's base mesh), and its
    true residual meets the criterion."""
    for k, q in ((1, 0), (2, 1)):
        x, its, hist, H = heat_solve(40, 3, k, q)
        assert its == 3, (k, q, hist)
        A, b = H.A[0], H.levels[0].rhs()
        assert np.linalg.norm(b - A @ x) <= max(1e-6 * np.linalg.norm(b), 1e-6)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_prolongation_reproduces_coarse_polynomials(k):
    """Nested P_k spaces: interpolating a degree-k polynomial given on the
    coarse nodes reproduces it at the fine nodes; rows sum to one."""
    fine, coarse = HeatSpace(4, k), HeatSpace(2, k)
    P = fine.prolongation(coarse)
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-13)
    for a in range(k + 1):
        pc = coarse.xy[:, 0] ** a * coarse.xy[:, 1] ** (k - a)
        pf = fine.xy[:, 0] ** a * fine.xy[:, 1] ** (k - a)
        assert np.allclose(P @ pc, pf, atol=1e-13)
