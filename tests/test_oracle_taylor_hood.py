"""Pins of the Taylor-Hood P_{k+1}-P_k structure (oracle/taylor_hood.py)
against the closed forms of Sec. 3.1, for the P2-P1 discretization the GPU
path implements (k = 1) and the P3-P2 one (k = 2, the paper's second
discretization) and beyond: global DoFs, DoFs and nonzeros of an interior
Vanka+star patch, the vertex-star pressure count, and at k = 1 the patches
of the independent P2-P1 oracle (oracle/mesh.py)."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.taylor_hood import TaylorHood


def global_dofs(M, k):
    # Sec. 3.1: velocity of degree k + 1 (two components), pressure of degree
    # k, every DoF of the M x M mesh (M_x = M + 1 vertices per side)
    return 3 * M ** 2 * k ** 2 + (4 * M ** 2 + 6 * M) * k + 2 * M ** 2 + 4 * M + 3


def patch_dofs(k):
    return 9 * k ** 2 + 15 * k + 15            # Sec. 3.1, Vanka-star patch


def patch_nnz(k):
    return 12 * k ** 4 + 96 * k ** 3 + 240 * k ** 2 + 252 * k + 128   # Sec. 3.1 / App. A.1


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("M", [2, 3, 5, 8])
def test_global_dof_count(M, k):
    assert TaylorHood(M, k).n_dofs_total() == global_dofs(M, k)


@pytest.mark.parametrize("k,dofs,nnz", [(1, 39, 728), (2, 81, 2552), (3, 141, 6608)])
def test_interior_patch_dofs_and_nonzeros(k, dofs, nnz):
    assert patch_dofs(k) == dofs and patch_nnz(k) == nnz
    th = TaylorHood(6, k)
    for v in [(2, 2), (3, 3), (2, 4), (4, 3)]:   # vertices whose star is away from the boundary
        assert th.patch_dofs(v) == dofs
        assert th.patch_nnz(v) == nnz


@pytest.mark.parametrize("k", [1, 2, 3])
def test_patch_pressure_is_the_vertex_star(k):
    # the pressure part of a Vanka+star patch is the degree-k vertex star:
    # 3k^2 - 3k + 1 nodes (Sec. 3.1, the heat-equation patch count)
    th = TaylorHood(6, k)
    _, pres = th.patch((3, 3))
    assert len(pres) == 3 * k ** 2 - 3 * k + 1


@pytest.mark.parametrize("M", [3, 4, 5])
def test_p2p1_patches_match_the_p2p1_oracle(M):
    # k = 1: the same free DoFs as oracle/mesh.py's patches, at every vertex
    # (boundary vertices included, Dirichlet velocity DoFs left out)
    mesh = Mesh(M)
    th = TaylorHood(M, 1)
    ref = mesh.patches()
    n1 = M + 1
    for vid in range(mesh.nv):
        vel, pres = th.patch((vid % n1, vid // n1))
        free = mesh.node_free[vel]
        assert np.all(free >= 0)
        dofs = np.sort(np.concatenate([2 * free, 2 * free + 1, mesh.p_offset + pres]))
        assert np.array_equal(dofs, ref[vid]), vid


def test_boundary_patches_are_smaller():
    th = TaylorHood(6, 2)
    interior = th.patch_dofs((3, 3))
    assert th.patch_dofs((0, 0)) < th.patch_dofs((0, 3)) < interior
    assert th.n_dofs_free() == 2 * (3 * 6 - 1) ** 2 + (2 * 6 + 1) ** 2


def _mono_integral(p, r):
    """int over the unit square of x^p y^r."""
    return 1.0 / ((p + 1) * (r + 1))


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("M", [2, 4])
def test_spatial_operators_integrate_polynomials_exactly(M, k):
    """The degree-(k+1) velocity and degree-k pressure spaces reproduce
    monomials of their degree, and the degree-8 rule integrates the mass,
    stiffness and divergence integrands exactly: u^T M u, u^T K u and
    q^T B u equal the closed-form integrals over the unit square."""
    from oracle.taylor_hood import spatial_operators
    Mu, Ku, Bx, By, V, P = spatial_operators(M, k)
    K = k + 1
    assert Mu.sum() == pytest.approx(1.0, abs=1e-13)
    assert np.abs(Ku @ np.ones(V.n)).max() < 1e-12
    x, y = V.xy[:, 0], V.xy[:, 1]
    px, py = P.xy[:, 0], P.xy[:, 1]
    for a in range(K + 1):
        b = K - a
        u = x ** a * y ** b
        assert u @ (Mu @ u) == pytest.approx(_mono_integral(2 * a, 2 * b), rel=1e-12)
        grad2 = (a * a * _mono_integral(2 * a - 2, 2 * b) if a else 0.0) + \
                (b * b * _mono_integral(2 * a, 2 * b - 2) if b else 0.0)
        assert u @ (Ku @ u) == pytest.approx(grad2, rel=1e-12, abs=1e-13)
        for c in range(k + 1):
            d = k - c
            q = px ** c * py ** d
            ex = a * _mono_integral(c + a - 1, d + b) if a else 0.0
            ey = b * _mono_integral(c + a, d + b - 1) if b else 0.0
            assert q @ (Bx @ u) == pytest.approx(ex, rel=1e-12, abs=1e-13)
            assert q @ (By @ u) == pytest.approx(ey, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("k,nnz", [(1, 728), (2, 2552)])
def test_assembled_patterns_give_the_patch_nonzeros(k, nnz):
    """The sparsity of the assembled operators, restricted to an interior
    Vanka+star patch, has the structural nonzeros the enumeration and Sec. 3.1
    give: 4 per coupled velocity node pair (the velocity blocks), 2 x 2 per
    coupled (velocity, pressure) node pair."""
    from oracle.taylor_hood import spatial_operators
    Mu, Ku, Bx, By, V, P = spatial_operators(6, k)
    th = TaylorHood(6, k)
    vel, pres = th.patch((3, 3))
    # stored entries (the assembly stores every pair of nodes of a cell, zeros
    # included); Bx and By share one pattern
    vv = Mu[vel][:, vel].nnz
    pv = Bx[pres][:, vel].nnz
    assert By[pres][:, vel].nnz == pv
    assert 4 * vv + 4 * pv == nnz == th.patch_nnz((3, 3))


@pytest.mark.parametrize("k", [1, 2])
def test_prolongation_reproduces_the_coarse_fields(k):
    """Nested spaces: prolonging the coarse interpolant of any polynomial of
    the space's degree gives the fine interpolant exactly, and constants are
    kept (rows sum to one), for velocity (degree k+1) and pressure (degree k)."""
    from oracle.heat import HeatSpace
    from oracle.taylor_hood import prolongation
    M = 4
    Pu, Pp = prolongation(M, k)
    for P, K in ((Pu, k + 1), (Pp, k)):
        fine, coarse = HeatSpace(M, K), HeatSpace(M // 2, K)
        assert np.allclose(P @ np.ones(coarse.n), 1.0, atol=1e-13)
        for a in range(K + 1):
            for b in range(K + 1 - a):
                fc = coarse.xy[:, 0] ** a * coarse.xy[:, 1] ** b
                ff = fine.xy[:, 0] ** a * fine.xy[:, 1] ** b
                assert np.abs(P @ fc - ff).max() < 1e-12, (K, a, b)


@pytest.mark.parametrize("k", [1, 2])
def test_convection_operators_integrate_polynomials_exactly(k):
    """For a velocity field and test/trial fields of the velocity degree
    (monomials), v^T C(u) w = int v (u . grad w) and v^T D_ab(u) w =
    int v w du_a/dx_b, the closed forms over the unit square."""
    from oracle.taylor_hood import convection_operators
    K = k + 1
    mono = [(a, K - a) for a in range(K + 1)] + [(1, 0), (0, 1)]
    from oracle.heat import HeatSpace
    sp_ = HeatSpace(3, K)
    x, y = sp_.xy[:, 0], sp_.xy[:, 1]
    f = lambda e: x ** e[0] * y ** e[1]
    for ue_x, ue_y in (((K, 0), (0, K)), ((1, K - 1), (K - 1, 1))):
        C, D, _ = convection_operators(3, k, f(ue_x), f(ue_y))
        for ve in mono:
            for we in mono:
                vv, ww = f(ve), f(we)
                # u . grad w = ux dw/dx + uy dw/dy, all monomial products
                ex = 0.0
                if we[0]:
                    ex += we[0] * _mono_integral(ve[0] + ue_x[0] + we[0] - 1, ve[1] + ue_x[1] + we[1])
                if we[1]:
                    ex += we[1] * _mono_integral(ve[0] + ue_y[0] + we[0], ve[1] + ue_y[1] + we[1] - 1)
                assert vv @ (C @ ww) == pytest.approx(ex, rel=1e-11, abs=1e-13)
                for a, ue in enumerate((ue_x, ue_y)):
                    for b in range(2):
                        if ue[b] == 0:
                            exd = 0.0
                        else:
                            de = [ue[0], ue[1]]
                            de[b] -= 1
                            exd = ue[b] * _mono_integral(ve[0] + we[0] + de[0], ve[1] + we[1] + de[1])
                        assert vv @ (D[a][b] @ ww) == pytest.approx(exd, rel=1e-11, abs=1e-13)


def _mms(R, seed=5):
    import stwr_workloads as w
    from oracle.mms import MMS
    psi_ab, psi_coef, p_ab, p_coef = w.draw_modes(seed, 4, 3, 4, np.pi)
    return MMS(psi_ab, psi_coef, p_ab, p_coef, R)


@pytest.mark.parametrize("q", [0, 1])
def test_space_time_jacobian_k1_equals_the_p2p1_oracle(q):
    """At k = 1 the degree-generic space-time Jacobian is the P2-P1 one of
    oracle/assembly.py (independent code: its own bases, cell maps and
    numbering), entry by entry at a seeded state."""
    from oracle.assembly import Level
    from oracle.taylor_hood import TaylorHoodLevel
    mms = _mms(7.0)
    L = Level(4, q, 3, 1.0, mms)
    T = TaylorHoodLevel(4, 1, q, 3, 1.0, mms)
    assert T.n_free == L.n_free and T.n_st == L.n_st
    x = 0.3 * np.random.default_rng(3).standard_normal((L.n_free, 3, q + 1))
    A, B = L.jacobian(x), T.jacobian(x)
    assert abs(A - B).max() <= 1e-14 * abs(A).max()


def test_space_time_jacobian_k2_stokes_blocks():
    """P3-P2 at R = 0 (Stokes): the diagonal slab block of the x velocity is
    T (x) M_u + dt W (x) K_u on the free nodes, and the velocity-pressure
    blocks are -dt W (x) B, with M_u, K_u, B the pinned spatial operators and
    T, W the DG(q) temporal matrices."""
    from oracle.taylor_hood import TaylorHoodLevel, spatial_operators
    M, k, q, N = 4, 2, 1, 2
    T = TaylorHoodLevel(M, k, q, N, 1.0, _mms(0.0))
    J = T.jacobian(np.zeros(T.n_st)).tocsr()
    Mu, Ku, Bx, By, V, P = spatial_operators(M, k)
    tb, nq, st = T.tb, T.nq, T.N * T.nq
    Tq = np.einsum("g,ga,gb->ab", tb.wg, tb.Phi, tb.dPhi) + np.outer(tb.e0, tb.e0)
    Wt = np.einsum("g,ga,gb->ab", tb.wg, tb.Phi, tb.Phi)
    free = np.nonzero(T.node_free >= 0)[0]
    fx = 2 * T.node_free[free]
    pd = T.p_offset + np.arange(P.n)
    Muf, Kuf = Mu[free][:, free].toarray(), Ku[free][:, free].toarray()
    Bxf = Bx[:, free].toarray()
    for n in range(N):
        for a in range(nq):
            for b in range(nq):
                blk = J[fx * st + n * nq + a][:, fx * st + n * nq + b].toarray()
                assert np.abs(blk - (Tq[a, b] * Muf + T.dt * Wt[a, b] * Kuf)).max() < 1e-13
                pu = J[pd * st + n * nq + a][:, fx * st + n * nq + b].toarray()
                assert np.abs(pu + T.dt * Wt[a, b] * Bxf).max() < 1e-13


def test_patch_smoother_k1_equals_the_p2p1_oracle():
    """The WR Vanka+star smoother (oracle/smoother.py) on the degree-generic
    level at k = 1 is the P2-P1 oracle's: same patches, same Jacobian."""
    from oracle.assembly import Level
    from oracle.smoother import PatchSmoother
    from oracle.taylor_hood import TaylorHoodLevel
    mms = _mms(7.0)
    L = Level(4, 1, 3, 1.0, mms)
    T = TaylorHoodLevel(4, 1, 1, 3, 1.0, mms)
    x = 0.3 * np.random.default_rng(6).standard_normal((L.n_free, 3, 2))
    r = np.random.default_rng(7).standard_normal(L.n_st)
    za = PatchSmoother(L, L.jacobian(x)).apply(r)
    zb = PatchSmoother(T, T.jacobian(x), T.patches()).apply(r)
    assert np.linalg.norm(za - zb) <= 1e-12 * np.linalg.norm(za)


def test_p3p2_patch_blocks_and_solves():
    """P3-P2 x DG(1): interior slab blocks of 81 x 2 = 162 rows (Sec. 3.1's
    81 patch DoFs, two temporal nodes), and every patch solve satisfies its
    space-time patch system A_v y = r_v (forward block substitution)."""
    from oracle.smoother import PatchSmoother
    from oracle.taylor_hood import TaylorHoodLevel
    T = TaylorHoodLevel(4, 2, 1, 2, 1.0, _mms(5.0))
    A = T.jacobian(0.2 * np.random.default_rng(8).standard_normal(T.n_st)).tocsr()
    S = PatchSmoother(T, A, T.patches())
    sizes = [k for (_, _, _, _, k) in S.blocks]
    # full patches: vertices at least two squares from the boundary (whose
    # star closure holds no Dirichlet node), (M - 3)^2 of them
    assert max(sizes) == 162 and sizes.count(162) == (4 - 3) ** 2
    rng = np.random.default_rng(9)
    for i in (0, 12, 24):
        idx, perm, lus, subs, k = S.blocks[i]
        Ap = A[idx][:, idx].toarray()[np.ix_(perm, perm)]
        rp = rng.standard_normal(len(idx))
        y = S.patch_solve(i, rp)
        assert np.linalg.norm(Ap @ y - rp) <= 1e-10 * np.linalg.norm(rp)


@pytest.mark.parametrize("q", [0, 1])
def test_residual_k1_equals_the_p2p1_oracle(q):
    """At k = 1 the degree-generic space-time residual is oracle/assembly.py's."""
    from oracle.assembly import Level
    from oracle.taylor_hood import TaylorHoodLevel
    mms = _mms(7.0)
    L = Level(4, q, 3, 1.0, mms)
    T = TaylorHoodLevel(4, 1, q, 3, 1.0, mms)
    x = 0.3 * np.random.default_rng(3).standard_normal((L.n_free, 3, q + 1))
    a, b = L.residual(x), T.residual(x)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


@pytest.mark.parametrize("q", [0, 1])
def test_p3p2_jacobian_is_the_derivative_of_the_residual(q):
    """P3-P2: the Jacobian is the exact derivative of the residual (full
    Newton): a central difference of F along a seeded direction matches J d
    to the difference's own error."""
    from oracle.taylor_hood import TaylorHoodLevel
    T = TaylorHoodLevel(4, 2, q, 2, 1.0, _mms(5.0))
    x = 0.3 * np.random.default_rng(4).standard_normal(T.n_st)
    d = np.random.default_rng(5).standard_normal(T.n_st)
    Jd = T.jacobian(x) @ d
    eps = 1e-6
    fd = (T.residual(x + eps * d).ravel() - T.residual(x - eps * d).ravel()) / (2 * eps)
    assert np.linalg.norm(fd - Jd) <= 1e-8 * np.linalg.norm(Jd)


def test_hierarchy_k1_vcycle_equals_the_p2p1_oracle():
    """At k = 1 the Taylor-Hood hierarchy (its levels, transfers and state
    injection) gives the P2-P1 oracle hierarchy's V-cycle (Alg. 1)."""
    import stwr_workloads as w
    from oracle.multigrid import Hierarchy
    from oracle.taylor_hood import TaylorHoodHierarchy
    prob = w.small_problem(8, 2, 1, 3, 10.0, 11)
    H = Hierarchy(prob)
    T = TaylorHoodHierarchy(8, 2, 1, 1, 3, prob.t_final, H.mms)
    x = 0.3 * np.random.default_rng(2).standard_normal(H.levels[0].n_st)
    H.assemble(x)
    T.assemble(x)
    b = np.random.default_rng(3).standard_normal(H.levels[0].n_st)
    a1, a2 = H.vcycle(b), T.vcycle(b)
    assert np.linalg.norm(a1 - a2) <= 1e-12 * np.linalg.norm(a1)


def test_p3p2_fgmres_wrmg_solves():
    """P3-P2 x DG(1) on an 8 x 8 mesh with two levels: FGMRES(30)
    right-preconditioned by one V-cycle with the WR Vanka+star smoother
    (Alg. 1, Sec. 3) reduces the residual of a consistent system by 1e-10
    in a handful of iterations and recovers its solution (pressure up to its
    constant)."""
    import stwr_workloads as w
    from oracle.mms import MMS
    from oracle.multigrid import fgmres, project_pressure
    from oracle.taylor_hood import TaylorHoodHierarchy
    psi_ab, psi_coef, p_ab, p_coef = w.draw_modes(11, 4, 3, 4, np.pi)
    T = TaylorHoodHierarchy(8, 2, 2, 1, 2, 0.1, MMS(psi_ab, psi_coef, p_ab, p_coef, 10.0))
    L0 = T.levels[0]
    T.assemble(0.1 * np.random.default_rng(2).standard_normal(L0.n_st))
    A = T.A[0]
    xt = project_pressure(L0, np.random.default_rng(3).standard_normal(L0.n_st))
    b = A @ xt
    x, its, _ = fgmres(A, T.vcycle, b, 1e-10, 30, 200, project=lambda v: project_pressure(L0, v))
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-8)
    assert its <= 20
    assert np.linalg.norm(project_pressure(L0, x) - xt) <= 1e-5 * np.linalg.norm(xt)


class _CubicFlow:
    """u = (1 + t) (2 x^2 y, -2 x y^2) (stream function (1 + t) x^2 y^2,
    divergence-free), p = x^2 - y^2, and the forcing that makes them solve
    eq. nsfem's strong form u_t + R (u . grad) u - lap u + grad p = f:
    (u . grad) u = (1 + t)^2 (4 x^3 y^2, 4 x^2 y^3), lap u = (1 + t) (4 y, -4 x)."""

    def __init__(self, R):
        self.R = R

    def velocity(self, t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float), np.asarray(y, float))
        return (1 + t) * 2 * x ** 2 * y, -(1 + t) * 2 * x * y ** 2

    def forcing(self, t, x, y):
        t, x, y = np.broadcast_arrays(np.asarray(t, float), np.asarray(x, float), np.asarray(y, float))
        s = 1 + t
        fx = 2 * x ** 2 * y + self.R * s ** 2 * 4 * x ** 3 * y ** 2 - s * 4 * y + 2 * x
        fy = -2 * x * y ** 2 + self.R * s ** 2 * 4 * x ** 2 * y ** 3 + s * 4 * x - 2 * y
        return fx, fy


def _exact_free(T, flow):
    t = (np.arange(T.N)[:, None] + T.tb.nodes[None, :]) * T.dt
    ux, uy = flow.velocity(t[None], T.V.xy[:, 0][:, None, None], T.V.xy[:, 1][:, None, None])
    x = np.zeros((T.n_free, T.N, T.nq))
    fr = T.node_free >= 0
    kf = T.node_free[fr]
    x[2 * kf], x[2 * kf + 1] = ux[fr], uy[fr]
    p = T.P.xy[:, 0] ** 2 - T.P.xy[:, 1] ** 2
    x[T.p_offset:] = p[:, None, None]
    return x


@pytest.mark.parametrize("q", [1, 2])
def test_p3p2_residual_vanishes_at_a_solution_in_the_space(q):
    """Galerkin consistency: when the exact solution lies in P3-P2 x DG(q)
    (cubic velocity, quadratic pressure, polynomial in time) and every
    integrand is integrated exactly, the space-time residual at its
    interpolant is zero to rounding.  P2-P1 cannot represent the cubic, so
    there the residual is far from zero."""
    from oracle.taylor_hood import TaylorHoodLevel
    flow = _CubicFlow(3.0)
    T = TaylorHoodLevel(4, 2, q, 2, 0.5, flow)
    F = T.residual(_exact_free(T, flow))
    assert np.abs(F).max() < 1e-13
    T1 = TaylorHoodLevel(4, 1, q, 2, 0.5, flow)
    assert np.abs(T1.residual(_exact_free(T1, flow))).max() > 1e-5
