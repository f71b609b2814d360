"""Taylor-Hood P3-P2 (the paper's second discretisation: Sec. 3 Vanka+star
patches of 81 DoFs, Sec. 3.1) on the GPU against the P3-P2 oracle, through
the C ABI, on seeded inputs: residual and Jacobian of eq. nsfem on every
level, operator applications, transfers, patch applications (FP64 and FP32
large blocks), Chebyshev relaxation, eigen-estimate, coarsest solve,
V-cycle, FGMRES and Newton.

Bars as for P2-P1: residual, Jacobian and operator 1e-13 relative, transfers
1e-14, one FP64 patch application and one or three relaxation sweeps 1e-12
(per slab, element by element), V-cycle 1e-12, FGMRES and Newton 1e-10; FP32
patch blocks 1e-5 per slab; the coarsest solve condition-aware."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import (entrywise, gpu_problem, log, rel, seeded, spacetime_from_bsr, to_dev, to_host,
                        torch_cuda)

pytestmark = pytest.mark.gpu

CASES = {
    "p3p2_q0_m4_n3": dict(mesh_n=4, n_levels=2, q=0, n_slabs=3, reynolds=1.0, seed=701),
    "p3p2_q1_m4_n2": dict(mesh_n=4, n_levels=2, q=1, n_slabs=2, reynolds=10.0, seed=702),
    "p3p2_q1_m8_n2": dict(mesh_n=8, n_levels=2, q=1, n_slabs=2, reynolds=5.0, seed=703),
}


def make(case):
    c = CASES[case]
    return w.small_problem(c["mesh_n"], c["n_levels"], c["q"], c["n_slabs"], c["reynolds"], c["seed"],
                           t_final=0.5, degree=2)


def oracle_hierarchy(prob):
    from oracle.mms import make_flow
    from oracle.taylor_hood import TaylorHoodHierarchy
    return TaylorHoodHierarchy(prob.mesh_n, prob.n_levels, 2, prob.q, prob.n_slabs, prob.t_final,
                               make_flow(prob))


_state = {}


def setup_case(case):
    if case in _state:
        return _state[case]
    torch_cuda()
    prob = make(case)
    log(f"[p3p2 setup] {case}")
    G = gpu_problem(prob, time_chunks=1)
    H = oracle_hierarchy(prob)
    L0 = H.levels[0]
    U = seeded(L0.n_st, 1100 + prob.seed, 0.3)
    assert G.sizes(0)[0] == L0.n_st
    Ud = to_dev(U)
    G.assemble(Ud)
    H.assemble(U, with_smoothers=True)
    _state[case] = (prob, G, H, U, Ud)
    return _state[case]


@pytest.mark.parametrize("case", list(CASES))
def test_p3p2_residual(case):
    prob, G, H, U, Ud = setup_case(case)
    L0 = H.levels[0]
    F = G.vec()
    G.nonlinear_residual(Ud, F)
    Fo = L0.residual(U.reshape(L0.n_free, L0.N, L0.nq)).ravel()
    e = rel(to_host(F), Fo)
    log(f"[p3p2 residual] {case} rel={e:.2e}")
    assert e < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_p3p2_jacobian_entries_all_levels(case):
    prob, G, H, U, Ud = setup_case(case)
    for l, lev in enumerate(H.levels):
        rp, col, val, mass = G.get_operator(l)
        A = spacetime_from_bsr(rp, col, val, mass, lev.n_free, lev.N, lev.nq, lev.tb.e0, lev.tb.e1)
        err = abs(A - H.A[l]).max() / abs(H.A[l]).max()
        log(f"[p3p2 jacobian] {case} level {l} maxrel={err:.2e}")
        assert err < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_p3p2_apply_and_transfers(case):
    prob, G, H, U, Ud = setup_case(case)
    for l, lev in enumerate(H.levels):
        x, b = seeded(lev.n_st, 17 + l), seeded(lev.n_st, 19 + l)
        y, r = G.vec(l), G.vec(l)
        G.apply(l, to_dev(x), y)
        G.residual(l, to_dev(b), to_dev(x), r)
        e1, e2 = rel(to_host(y), H.A[l] @ x), rel(to_host(r), b - H.A[l] @ x)
        log(f"[p3p2 apply] {case} level {l} {e1:.2e} {e2:.2e}")
        assert e1 < 1e-13 and e2 < 1e-13
    for l in range(len(H.levels) - 1):
        nf_, nc_ = H.levels[l].n_st, H.levels[l + 1].n_st
        rf, ec, xf = seeded(nf_, 21), seeded(nc_, 22), seeded(nf_, 23)
        rc = G.vec(l + 1)
        G.restrict(l, to_dev(rf), rc)
        xd = to_dev(xf)
        G.prolong_add(l, to_dev(ec), xd)
        e1, e2 = rel(to_host(rc), H.P[l].T @ rf), rel(to_host(xd), xf + H.P[l] @ ec)
        log(f"[p3p2 transfer] {case} level {l} {e1:.2e} {e2:.2e}")
        assert e1 < 1e-14 and e2 < 1e-14


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec,bars", [(0, (1e-12, 1e-10)), (1, (1e-5, 1e-4))])
def test_p3p2_patch_apply(case, prec, bars):
    prob, G, H, U, Ud = setup_case(case)
    for l in range(len(H.levels) - 1):
        G.patch_factor(l, prec)
        lev = H.levels[l]
        r = seeded(lev.n_st, 41 + l)
        z = G.vec(l)
        G.patch_apply(l, to_dev(r), z)
        es, ee = entrywise(to_host(z), H.smoothers[l].apply(r), lev.n_free, lev.N, lev.nq)
        log(f"[p3p2 patch prec={prec}] {case} level {l} slab {es:.2e} entry {ee:.2e}")
        assert es <= bars[0] and ee <= bars[1]
    for l in range(len(H.levels) - 1):
        G.patch_factor(l, 0)


@pytest.mark.parametrize("case", list(CASES))
def test_p3p2_relax_and_eig(case):
    from oracle.smoother import chebyshev
    prob, G, H, U, Ud = setup_case(case)
    for l in range(len(H.levels) - 1):
        G.patch_factor(l, 0)
        lev = H.levels[l]
        b, x0 = seeded(lev.n_st, 61), seeded(lev.n_st, 62)
        for steps in (1, 3):
            x = to_dev(x0)
            G.relax(l, to_dev(b), x, steps, 1.9, 8.3)
            xo = chebyshev(H.A[l], H.smoothers[l].apply, b, x0, steps, 1.9, 8.3)
            es, ee = entrywise(to_host(x) - x0, xo - x0, lev.n_free, lev.N, lev.nq)
            log(f"[p3p2 relax] {case} level {l} steps {steps} slab {es:.2e} entry {ee:.2e}")
            assert es <= 1e-12 and ee <= 1e-10
        lam = G.eig_estimate(l)
        log(f"[p3p2 eig] {case} level {l} gpu={lam:.15f} oracle={H.lams[l]:.15f}")
        assert abs(lam - H.lams[l]) < 1e-10 * abs(H.lams[l])


@pytest.mark.parametrize("case", list(CASES))
def test_p3p2_coarse_vcycle(case):
    from oracle.multigrid import project_pressure
    prob, G, H, U, Ud = setup_case(case)
    lev = H.levels[-1]
    xt = project_pressure(lev, seeded(lev.n_st, 31))
    b = H.A[-1] @ xt
    x = G.vec(len(H.levels) - 1)
    G.coarse_solve(to_dev(b), x)
    e_o, e_t = rel(to_host(x), H.coarse.solve(b)), rel(to_host(x), xt)
    log(f"[p3p2 coarse] {case} vs oracle {e_o:.2e} vs truth {e_t:.2e}")
    assert e_o < 1e-9 and e_t < 1e-9
    G.setup_smoothers()
    b0 = seeded(H.levels[0].n_st, 71)
    xv = G.vec(0)
    G.vcycle(to_dev(b0), xv)
    e = rel(to_host(xv), H.vcycle(b0))
    log(f"[p3p2 vcycle] {case} rel={e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("case", ["p3p2_q1_m4_n2", "p3p2_q1_m8_n2"])
def test_p3p2_fgmres(case):
    from oracle.multigrid import fgmres, project_pressure
    torch_cuda()
    prob = make(case)
    G = gpu_problem(prob, time_chunks=1)
    H = oracle_hierarchy(prob)
    lev = H.levels[0]
    U0 = 0.1 * seeded(lev.n_st, 91)
    G.assemble(to_dev(U0))
    G.setup_smoothers()
    H.assemble(U0)
    b = H.A[0] @ project_pressure(lev, seeded(lev.n_st, 81))
    x = G.vec(0)
    st = G.fgmres(to_dev(b), x)
    xo, its, _ = fgmres(H.A[0], H.vcycle, b, 1e-10, 30, 200, lambda v: project_pressure(lev, v))
    e = rel(to_host(x), xo)
    log(f"[p3p2 fgmres] {case} gpu its={st['linear_total']} oracle its={its} rel={e:.2e}")
    assert e < 1e-10 and abs(st["linear_total"] - its) <= 1
    G.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-8)])
def test_p3p2_newton_exact_solution(prec, tol):
    """Full Newton (FP64 and FP32 smoother) on a 4x4 P3-P2 x DG(1) problem
    against the oracle's Newton with exact space-time linear solves."""
    torch_cuda()
    from oracle.direct import newton_exact_linear
    prob = make("p3p2_q1_m4_n2")
    H = oracle_hierarchy(prob)
    xo, fn = newton_exact_linear(H.levels[0], rtol=1e-13, maxit=20)
    G = gpu_problem(prob, smoother_prec=prec, time_chunks=1, newton_rtol=1e-12)
    U = G.vec()
    st = G.newton_solve(U)
    e = rel(to_host(U), xo.ravel())
    log(f"[p3p2 newton prec={prec}] newton={st['newton']} linear={st['linear']} rel_vs_exact={e:.2e} "
        f"(oracle newton steps {len(fn) - 1})")
    assert e < tol
    err = G.velocity_l2_error(U)
    log(f"[p3p2 newton prec={prec}] velocity L2 error {err:.3e}")
    assert np.isfinite(err)
    G.close()
