"""Oracle smoother, transfers and multigrid pinned by dense solves, closed
forms and invariants (Sec. 3: eq. waveform_patch_solve, Chebyshev interval,
P = I (x) P_h, R = P^T, Alg. 1)."""
import numpy as np
import pytest
import scipy.sparse as sp

import stwr_workloads as w
from oracle.assembly import Level
from oracle.mesh import Mesh
from oracle.mms import MMS
from oracle.multigrid import Hierarchy, Options, fgmres, project_pressure
from oracle.smoother import PatchSmoother, chebyshev, eig_estimate
from oracle.transfer import spatial_prolongation, spacetime_prolongation


def level_and_jac(M=4, q=1, N=3, R=10.0, seed=5):
    psi_ab, psi_coef, p_ab, p_coef = w.draw_modes(seed, 4, 3, 4)
    L = Level(M, q, N, 1.0, MMS(psi_ab, psi_coef, p_ab, p_coef, R))
    x = np.random.default_rng(seed).standard_normal((L.n_free, N, L.nq)) * 0.3
    return L, L.jacobian(x)


@pytest.mark.parametrize("q", [0, 1])
def test_patch_solve_equals_dense_solve(q):
    L, A = level_and_jac(q=q)
    sm = PatchSmoother(L, A)
    rng = np.random.default_rng(1)
    Ad = A.toarray()
    for v in (0, 7, 12, 24):
        idx, perm, lus, subs, k = sm.blocks[v]
        Ap = Ad[np.ix_(idx, idx)][np.ix_(perm, perm)]
        # block lower bidiagonal: nothing above the diagonal blocks
        for n in range(L.N):
            assert not np.any(Ap[n * k:(n + 1) * k, (n + 1) * k:])
            if n >= 2:
                assert not np.any(Ap[n * k:(n + 1) * k, :(n - 1) * k])
        r = rng.standard_normal(len(idx))
        y = sm.patch_solve(v, r)
        assert np.allclose(y, np.linalg.solve(Ap, r), rtol=1e-12, atol=1e-12)


def test_additive_smoother_is_sum_of_patch_corrections():
    L, A = level_and_jac(q=1)
    sm = PatchSmoother(L, A)
    r = np.random.default_rng(2).standard_normal(L.n_st)
    Ad = A.toarray()
    z = np.zeros(L.n_st)
    for S in L.mesh.patches():
        st = L.N * L.nq
        idx = (S[:, None] * st + np.arange(st)).ravel()
        z[idx] += np.linalg.solve(Ad[np.ix_(idx, idx)], r[idx])
    assert np.allclose(sm.apply(r), z, rtol=1e-11, atol=1e-12)


def test_chebyshev_one_step_is_weighted_relaxation():
    L, A = level_and_jac(q=0)
    sm = PatchSmoother(L, A)
    b = np.random.default_rng(3).standard_normal(L.n_st)
    x0 = np.random.default_rng(4).standard_normal(L.n_st)
    lam = 7.0
    x1 = chebyshev(A, sm.apply, b, x0, 1, 0.25 * lam, 1.05 * lam)
    assert np.allclose(x1, x0 + sm.apply(b - A @ x0) / (0.65 * lam), rtol=1e-13, atol=1e-13)


def test_chebyshev_error_polynomial_on_diagonal_matrix():
    """With M = I and A = diag(l), the error after k steps is
    T_k((theta - l)/delta) / T_k(theta/delta) times the initial error."""
    lam = np.linspace(0.3, 2.0, 40)
    A = sp.diags(lam)
    e0 = np.random.default_rng(5).standard_normal(40)
    a, bnd = 0.5, 2.1
    th, de = 0.5 * (a + bnd), 0.5 * (bnd - a)
    for k in (1, 2, 3, 5):
        x = chebyshev(A, lambda r: r, np.zeros(40), e0.copy(), k, a, bnd)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
        expect = Tk((th - lam) / de) / Tk(th / de) * e0
        assert np.allclose(x, expect, atol=1e-12)


def test_eig_estimate_exact_for_few_distinct_eigenvalues():
    vals = np.array([0.5, 1.0, 2.0, 3.5, 4.25, 5.0, 6.0, 7.75])
    d = np.repeat(vals, 25)
    A = sp.diags(d)
    lam = eig_estimate(A, lambda r: r, len(d), 10)
    assert lam == pytest.approx(7.75, rel=1e-10)
    # non-normal preconditioned operator: still below and close to the true max
    rng = np.random.default_rng(0)
    B = np.diag(np.linspace(1, 9, 60)) + 0.05 * np.triu(rng.standard_normal((60, 60)), 1)
    lam = eig_estimate(sp.csr_matrix(B), lambda r: r, 60, 10)
    assert 7.0 < lam <= 9.0 + 1e-9


def test_prolongation_reproduces_polynomials():
    f, c = Mesh(8), Mesh(4)
    P = spatial_prolongation(f, c)
    quad = lambda xy: 1 + 2 * xy[:, 0] - xy[:, 1] + 3 * xy[:, 0] ** 2 - xy[:, 0] * xy[:, 1] + 0.5 * xy[:, 1] ** 2
    lin = lambda xy: 0.3 - 1.5 * xy[:, 0] + 2.5 * xy[:, 1]
    vc = np.zeros(c.n_free)
    cxy = c.free_node_xy()
    vc[0:c.p_offset:2] = quad(cxy)
    vc[1:c.p_offset:2] = -2 * quad(cxy)
    vc[c.p_offset:] = lin(c.vxy)
    vf = P @ vc
    fxy = f.free_node_xy()
    deep = (fxy.min(1) > c.h + 1e-12) & (fxy.max(1) < 1 - c.h - 1e-12)
    assert np.allclose(vf[0:f.p_offset:2][deep], quad(fxy)[deep], atol=1e-13)
    assert np.allclose(vf[1:f.p_offset:2][deep], -2 * quad(fxy)[deep], atol=1e-13)
    assert np.allclose(vf[f.p_offset:], lin(f.vxy), atol=1e-13)
    # pressure rows are a partition of unity
    assert np.allclose(np.asarray(P[f.p_offset:].sum(1)).ravel(), 1.0)


def test_spacetime_transfer_is_kron_and_adjoint():
    f, c = Mesh(8), Mesh(4)
    Ph = spatial_prolongation(f, c).toarray()
    P = spacetime_prolongation(f, c, 6)
    rng = np.random.default_rng(7)
    ec = rng.standard_normal((c.n_free, 6))
    assert np.allclose((P @ ec.ravel()).reshape(f.n_free, 6), Ph @ ec)
    r = rng.standard_normal(f.n_free * 6)
    assert np.dot(P.T @ r, ec.ravel()) == pytest.approx(np.dot(r, P @ ec.ravel()), rel=1e-12)


def test_mesh_independent_iterations():
    """FGMRES-WRMG counts stay flat under refinement (the paper's scalability claim)."""
    its = []
    for M, L in ((8, 2), (16, 3)):
        p = w.small_problem(M, L, 1, 3, 10.0, seed=3)
        H = Hierarchy(p, Options())
        L0 = H.levels[0]
        x0 = L0.initial_guess()
        H.assemble(x0.ravel())
        F = L0.residual(x0).ravel()
        _, n, _ = fgmres(H.A[0], H.vcycle, -F, 1e-8, 30, 100, lambda v: project_pressure(L0, v))
        its.append(n)
    assert abs(its[1] - its[0]) <= 3 and max(its) <= 25, its


def test_newton_with_eisenstat_walker_reaches_the_exact_solution():
    """Newton with Eisenstat-Walker forcing terms (choice 2) converges to the
    exact discrete solution (slab-by-slab direct route) like the fixed
    tolerance does, with fewer linear iterations; the forcing terms start at
    eta_0 and shrink as the residual ratio does."""
    from oracle.direct import solve_slab_by_slab
    from oracle.multigrid import newton_solve
    p = w.small_problem(8, 2, 0, 3, 10.0, seed=31)
    L = Level(8, 0, 3, 1.0, MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds))
    xs = solve_slab_by_slab(L).ravel()
    x1, s1, _ = newton_solve(p, Options(newton_rtol=1e-12))
    x2, s2, _ = newton_solve(p, Options(newton_rtol=1e-12, newton_ew=True))
    assert np.linalg.norm(x1 - xs) <= 1e-10 * np.linalg.norm(xs)
    assert np.linalg.norm(x2 - xs) <= 1e-10 * np.linalg.norm(xs)
    assert sum(s2["linear"]) < sum(s1["linear"])
    eta = s2["eta"]
    assert eta[0] == 0.3 and all(0.0 < e <= 0.9 for e in eta)
    assert eta[-1] < eta[0]


def test_eisenstat_walker_forcing_gives_newton_order_golden_ratio():
    """The forcing terms pinned by what they do, not by their formula:
    Eisenstat and Walker's choice 2 with exponent (1 + sqrt 5) / 2 makes an
    inexact Newton iteration whose linear solves leave exactly the relative
    residual eta_k converge with q-order (1 + sqrt 5) / 2 (SIAM J. Sci.
    Comput. 17, 1996).  On x^3 = 2 in 200-digit arithmetic the observed order
    log(e_k+1 / e_k) / log(e_k / e_k-1) settles at the golden ratio to 1e-9;
    a fixed tolerance would give order 1, exact solves order 2, another
    exponent that exponent.  A growing residual is capped at eta_max = 0.9."""
    import decimal
    from oracle.multigrid import ew_forcing
    ctx = decimal.Context(prec=200)
    D = ctx.create_decimal
    root = ctx.power(D(2), ctx.divide(D(1), D(3)))
    x, fprev, eta, errs = D("2.0"), None, 0.0, []
    for k in range(12):
        fx = ctx.subtract(ctx.power(x, 3), D(2))
        eta = ew_forcing(k, float(abs(fx)), float(fprev) if fprev is not None else 1.0, eta)
        x = ctx.subtract(x, ctx.multiply(ctx.subtract(D(1), D(eta)), ctx.divide(fx, ctx.multiply(D(3), ctx.power(x, 2)))))
        fprev = abs(fx)
        errs.append(abs(ctx.subtract(x, root)))
    e = [float(v) for v in errs]
    orders = [np.log(e[k] / e[k - 1]) / np.log(e[k - 1] / e[k - 2]) for k in range(9, 12)]
    phi = (1 + 5 ** 0.5) / 2
    assert all(abs(o - phi) < 1e-9 for o in orders), orders
    assert ew_forcing(3, 2.0, 1.0, 0.5) == 0.9


def _interpolant(level, prob_mms):
    """Free space-time vector of the nodal interpolant of the manufactured
    velocity and of the pressure p(t, x, y) = cos(x + 2 y + t) on a level."""
    t = level.node_times()[None, :, :]
    m = level.mesh
    ux, uy = prob_mms.velocity(t, m.nxy[:, 0][:, None, None], m.nxy[:, 1][:, None, None])
    p = np.cos(m.vxy[:, 0][:, None, None] + 2 * m.vxy[:, 1][:, None, None] + t)
    x = np.zeros((level.n_free, level.N, level.nq))
    fr = m.node_free >= 0
    k = m.node_free[fr]
    x[2 * k], x[2 * k + 1] = ux[fr], uy[fr]
    x[m.p_offset:] = p
    return x


def test_state_injection_of_an_interpolant_is_the_coarse_interpolant():
    """The Newton iterate reaches the coarse levels by injection (every coarse
    node is a fine node).  Injecting the fine interpolant of a smooth field
    gives the coarse interpolant of the same field, value for value, on every
    level of a three-level hierarchy, for both node families of the mesh (P2
    velocity nodes, P1 vertices)."""
    import stwr_workloads as w
    from oracle.multigrid import Hierarchy, Options
    prob = w.small_problem(16, 3, 1, 3, 10.0, 17)
    H = Hierarchy(prob, Options())
    xs = H.level_states(_interpolant(H.levels[0], H.mms))
    for l, lev in enumerate(H.levels):
        assert np.array_equal(xs[l], _interpolant(lev, H.mms)), l


def test_taylor_hood_state_injection_of_an_interpolant():
    """The same on the P3-P2 lattices (velocity (3M+1)^2, pressure (2M+1)^2)."""
    import stwr_workloads as w
    from oracle.mms import make_flow
    from oracle.taylor_hood import TaylorHoodHierarchy
    prob = w.small_problem(8, 3, 1, 2, 10.0, 18)
    T = TaylorHoodHierarchy(8, 3, 2, 1, 2, 1.0, make_flow(prob))

    def interp(L):
        t = ((np.arange(L.N)[:, None] + L.tb.nodes[None, :]) * L.dt)[None, :, :]
        ux, uy = L.mms.velocity(t, L.V.xy[:, 0][:, None, None], L.V.xy[:, 1][:, None, None])
        p = np.cos(L.P.xy[:, 0][:, None, None] + 2 * L.P.xy[:, 1][:, None, None] + t)
        x = np.zeros((L.n_free, L.N, L.nq))
        fr = L.node_free >= 0
        k = L.node_free[fr]
        x[2 * k], x[2 * k + 1] = ux[fr], uy[fr]
        x[L.p_offset:] = p
        return x

    xs = T.level_states(interp(T.levels[0]))
    for l, lev in enumerate(T.levels):
        assert np.array_equal(xs[l], interp(lev)), l
