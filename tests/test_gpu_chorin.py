"""The Chorin test problem (Sec. 2) on the GPU.

* Parity with the oracle on small meshes (Gauss-Legendre and right-Radau
  temporal nodes, q = 0 and 1): the residual at a seeded state, and Newton
  solves with the FP64 and FP32 smoothers against the oracle's exact discrete
  solution.
* The paper's table of Chorin velocity errors (Sec. 4.2: 80 x 80 mesh, four
  levels from a 10 x 10 base, R = 10, t in [0, 0.1], P2-P1 x DG(q)):
  q = 0: 6.51e-3, 3.32e-3, 1.70e-3 and q = 1: 1.77e-3, 4.60e-5, 1.18e-5 for
  N = 10, 20, 40.  The q = 1, N = 10 entry is read as 1.77e-4: the other five
  entries and the 1/N^2 rate the paper describes put it there, and 1.77e-3
  would be larger than the q = 0 value at N = 40.  With Gauss-Legendre nodes
  every entry is reproduced within 10 % (the paper prints three digits; the
  remaining few per cent are the same for the oracle on small meshes, so they
  come from details the paper does not state, not from the GPU path); the
  right-Radau reading gives errors about 1.5-1.9 times larger.  The runs use
  Eisenstat-Walker linear tolerances and Newton to 1e-8, as the paper's did,
  and reproduce its Newton and linear iteration counts (exactly for q = 0)."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, rel, seeded, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

PAPER = {(0, 10): 6.51e-3, (0, 20): 3.32e-3, (0, 40): 1.70e-3,
         (1, 10): 1.77e-4, (1, 20): 4.60e-5, (1, 40): 1.18e-5}


@pytest.mark.parametrize("q,N,nodes", [(0, 4, 1), (1, 3, 1), (1, 3, 0)])
def test_chorin_small_matches_oracle(q, N, nodes):
    torch_cuda()
    from oracle.assembly import Level
    from oracle.direct import solve_slab_by_slab
    from oracle.mms import Chorin
    p = w.chorin_problem(8, 2, q, N, nodes=nodes)
    lev = Level(8, q, N, 0.1, Chorin(10.0), "gauss" if nodes else "radau")
    # residual at a seeded state
    G = gpu_problem(p)
    U = seeded(lev.n_st, 77, 0.2)
    F = G.vec()
    G.nonlinear_residual(to_dev(U), F)
    e_res = rel(to_host(F), lev.residual(U.reshape(lev.n_free, lev.N, lev.nq)))
    x = solve_slab_by_slab(lev, tol=0.0).ravel()
    errs = {}
    for prec, tol in ((0, 1e-10), (1, 1e-8)):
        Gp = gpu_problem(p, smoother_prec=prec, newton_rtol=1e-12)
        Ud = Gp.vec()
        Gp.newton_solve(Ud)
        errs[prec] = rel(to_host(Ud), x)
        assert errs[prec] < tol, (prec, errs[prec])
        Gp.close()
    log(f"[chorin 8x8 q={q} N={N} nodes={nodes}] residual rel={e_res:.1e} "
        f"solution rel fp64={errs[0]:.1e} fp32={errs[1]:.1e}")
    assert e_res < 1e-13
    G.close()


def _error(q, N, nodes):
    p = w.chorin_problem(80, 4, q, N, nodes=nodes)
    G = gpu_problem(p, smoother_prec=1, newton_rtol=1e-8, newton_ew=1)
    U = G.vec()
    st = G.newton_solve(U)
    e = G.velocity_l2_error(U)
    G.close()
    return e, st


@pytest.mark.parametrize("q,N", sorted(PAPER))
def test_chorin_error_table_80x80(q, N):
    torch_cuda()
    e, st = _error(q, N, 1)
    log(f"[chorin 80x80 q={q} N={N}] error={e:.4e} paper={PAPER[(q, N)]:.2e} "
        f"ratio={e / PAPER[(q, N)]:.3f} newton={st['newton']} linear={st['linear']}")
    assert abs(e / PAPER[(q, N)] - 1.0) < 0.10
    # the paper's iteration table for these runs (Newton to 1e-8 with
    # Eisenstat-Walker tolerances): 4 Newton steps everywhere, 11 linear
    # iterations in total for q = 0 at every N, 12, 10 and 17 for q = 1
    assert st["newton"] == 4
    if q == 0:
        assert sum(st["linear"]) == 11
    else:
        assert 10 <= sum(st["linear"]) <= 17


def test_chorin_radau_reading_does_not_reproduce_the_table():
    torch_cuda()
    e, _ = _error(0, 10, 0)
    assert e / PAPER[(0, 10)] > 1.6


def test_newton_eisenstat_walker_matches_oracle():
    """Newton with Eisenstat-Walker linear tolerances: the same Newton steps
    and linear iteration counts (within one per step) as the oracle's Newton,
    and the exact discrete solution."""
    torch_cuda()
    from oracle.multigrid import Options, newton_solve
    p = w.chorin_problem(8, 2, 0, 4, nodes=1)
    xo, so, H = newton_solve(p, Options(newton_rtol=1e-10, newton_ew=True))
    G = gpu_problem(p, newton_rtol=1e-10, newton_ew=1)
    U = G.vec()
    st = G.newton_solve(U)
    log(f"[chorin ew] gpu newton={st['newton']} linear={st['linear']} "
        f"oracle newton={so['newton']} linear={so['linear']}")
    assert st["newton"] == so["newton"]
    assert all(abs(a - b) <= 1 for a, b in zip(st["linear"], so["linear"]))
    assert rel(to_host(U), xo) < 1e-9
    G.close()


# The paper's P3-P2 column of the same table (Sec. 4.2): its spatial degree 2
# errors equal its degree 1 ones (the error is temporal); q = 1 was run at
# N = 10 only (the others ran out of memory).
PAPER_P3P2 = {(0, 10): 6.51e-3, (0, 20): 3.32e-3, (0, 40): 1.70e-3, (1, 10): 1.77e-4}


@pytest.mark.parametrize("q,N", sorted(PAPER_P3P2))
def test_chorin_p3p2_error_table_80x80(q, N):
    """P3-P2 x DG(q) on 80 x 80 (4 levels; 5 at q = 1, whose 10 x 10 coarsest
    bordered blocks would exceed the dense coarse solve's order), FP32
    smoother, Newton to 1e-8 with Eisenstat-Walker tolerances: the space-time
    velocity error within 10% of the paper's."""
    torch_cuda()
    p = w.chorin_problem(80, 5 if q == 1 else 4, q, N, nodes=1, degree=2)
    G = gpu_problem(p, smoother_prec=1, newton_rtol=1e-8, newton_ew=1)
    U = G.vec()
    st = G.newton_solve(U)
    e = G.velocity_l2_error(U)
    G.close()
    log(f"[chorin p3p2 80x80 q={q} N={N}] error={e:.4e} paper={PAPER_P3P2[(q, N)]:.2e} "
        f"ratio={e / PAPER_P3P2[(q, N)]:.3f} newton={st['newton']} linear={st['linear']}")
    assert abs(e / PAPER_P3P2[(q, N)] - 1.0) < 0.10
    assert 4 <= st["newton"] <= 5
