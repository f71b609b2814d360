"""Reproducibility.

Every step of a solve runs in a fixed order: the residual and Jacobian are
assembled cell colour by cell colour with plain additions (no FP64 atomics),
and with the solver option deterministic = 1 the time-chunk choice is the
plain sweep instead of a choice by timing, so a solve gives the same bits
every run.  Checked: the assembled Jacobian (every level) and the residual
against the oracle, P2-P1 and P3-P2; an assembly equal bit for bit to a
second one; two independent Newton solves, with fresh problems, equal bit
for bit (solution, residual history and iteration counts); the solution
with the timed chunk choice equal to them to the Newton tolerance."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import (gpu_problem, log, oracle_hierarchy, rel, seeded, spacetime_from_bsr, to_dev, to_host,
                        torch_cuda)

pytestmark = pytest.mark.gpu


def _oracle(prob, degree):
    if degree == 1:
        return oracle_hierarchy(prob)
    from oracle.mms import make_flow
    from oracle.taylor_hood import TaylorHoodHierarchy
    return TaylorHoodHierarchy(prob.mesh_n, prob.n_levels, 2, prob.q, prob.n_slabs, prob.t_final,
                               make_flow(prob))


@pytest.mark.parametrize("degree", [1, 2])
def test_colour_assembly_matches_oracle(degree):
    torch_cuda()
    prob = w.small_problem(8, 2, 1, 3, 30.0, 611, t_final=0.5, degree=degree)
    G = gpu_problem(prob, deterministic=1, time_chunks=1)
    H = _oracle(prob, degree)
    L0 = H.levels[0]
    U = seeded(L0.n_st, 612, 0.3)
    Ud = to_dev(U)
    G.assemble(Ud)
    H.assemble(U, with_smoothers=False)
    ops = []
    for l, lev in enumerate(H.levels):
        rp, col, val, mass = G.get_operator(l)
        ops.append((val.copy(), mass.copy()))
        A = spacetime_from_bsr(rp, col, val, mass, lev.n_free, lev.N, lev.nq, lev.tb.e0, lev.tb.e1)
        err = abs((A - H.A[l]).tocsr()).max() / abs(H.A[l]).max()
        log(f"[det jacobian] degree {degree} level {l} maxrel={err:.2e}")
        assert err < 1e-13
    F = G.vec()
    G.nonlinear_residual(Ud, F)
    Fo = np.asarray(L0.residual(U.reshape(L0.n_free, L0.N, L0.nq))).ravel()
    e = rel(to_host(F), Fo)
    log(f"[det residual] degree {degree} rel={e:.2e}")
    assert e < 1e-13
    # a second assembly and residual: the same bits
    F1 = to_host(F).copy()
    G.assemble(Ud)
    G.nonlinear_residual(Ud, F)
    assert np.array_equal(to_host(F), F1)
    for l in range(len(H.levels)):
        _, _, val, mass = G.get_operator(l)
        assert np.array_equal(val, ops[l][0]) and np.array_equal(mass, ops[l][1])
    G.close()


def _solve(prob, det, prec):
    G = gpu_problem(prob, deterministic=det, smoother_prec=prec, newton_rtol=1e-10, newton_ew=1)
    U = G.vec()
    st = G.newton_solve(U)
    out = to_host(U).copy()
    G.close()
    return out, st


@pytest.mark.parametrize("prec", [0, 1])
def test_deterministic_solves_equal_bit_for_bit(prec):
    torch_cuda()
    prob = w.small_problem(16, 3, 1, 6, 30.0, 613)
    a, sa = _solve(prob, 1, prec)
    b, sb = _solve(prob, 1, prec)
    c, sc = _solve(prob, 0, prec)
    log(f"[det solve] prec={prec} newton={sa['newton']} linear={sa['linear']} "
        f"max|a-b|={np.abs(a - b).max():.1e} atomic vs det rel={rel(c, a):.1e}")
    assert np.array_equal(a, b)
    assert sa["newton"] == sb["newton"] and list(sa["linear"]) == list(sb["linear"])
    assert list(sa["fnorm"]) == list(sb["fnorm"])
    assert rel(c, a) < 1e-9
