"""The lid-driven cavity (Sec. 2 definition; runs of Sec. 4.3) on the GPU.

* Parity with the oracle on a small mesh (q = 0 and 1, R = 100): the
  residual at a seeded state, and Newton solves with the FP64 and FP32
  smoothers against the oracle's exact discrete solution.
* The paper's remark on Newton with direct linear solves (Sec. 4.3): 2, 3
  and 4 Newton steps for R = 1, 10 and 100 on its meshes.  Linear solves to
  1e-12 stand in for the direct solver; Newton stops at 1e-8 relative, as
  in the paper's runs.  The counts hold exactly on the 40 x 40 and 80 x 80
  meshes (three and four levels from a 10 x 10 base), t in [0, 0.02], N = 20.
* The paper's iteration table for FGMRES-WRMG with Eisenstat-Walker
  tolerances (P2-P1 columns): 4 Newton steps everywhere and 8-15 linear
  iterations in total.  This solver takes 4-5 Newton steps and 13-20 linear
  iterations on the same runs (its preconditioner contracts by about 0.2
  per FGMRES iteration here, where the paper's counts imply about 0.1; on
  the Chorin runs the two agree).  The test holds it to at most 5 Newton
  steps and 24 linear iterations, and logs the paper's counts beside."""
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, rel, seeded, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

MESHES = {40: 3, 80: 4}
DIRECT_NEWTON = {1.0: 2, 10.0: 3, 100.0: 4}
# (mesh, q, R) -> (Newton steps, total linear iterations) of the paper's table
PAPER_EW = {(40, 1, 1.0): (4, 10), (40, 1, 10.0): (4, 10), (40, 1, 100.0): (4, 13),
            (40, 0, 1.0): (4, 10), (40, 0, 10.0): (4, 11), (40, 0, 100.0): (4, 15),
            (80, 1, 1.0): (4, 8), (80, 1, 10.0): (4, 8), (80, 1, 100.0): (4, 13),
            (80, 0, 1.0): (4, 8), (80, 0, 10.0): (4, 8), (80, 0, 100.0): (4, 12)}


@pytest.mark.parametrize("q,N", [(0, 4), (1, 3)])
def test_cavity_small_matches_oracle(q, N):
    torch_cuda()
    from oracle.assembly import Level
    from oracle.direct import solve_slab_by_slab
    from oracle.mms import Cavity
    p = w.cavity_problem(8, 2, q, N, 100.0)
    lev = Level(8, q, N, 0.02, Cavity(100.0), "gauss")
    G = gpu_problem(p)
    U = seeded(lev.n_st, 91, 0.3)
    F = G.vec()
    G.nonlinear_residual(to_dev(U), F)
    e_res = rel(to_host(F), lev.residual(U.reshape(lev.n_free, lev.N, lev.nq)))
    G.close()
    x = solve_slab_by_slab(lev, tol=0.0).ravel()
    errs = {}
    for prec, tol in ((0, 1e-10), (1, 1e-8)):
        Gp = gpu_problem(p, smoother_prec=prec, newton_rtol=1e-12)
        Ud = Gp.vec()
        Gp.newton_solve(Ud)
        errs[prec] = rel(to_host(Ud), x)
        Gp.close()
    log(f"[cavity 8x8 q={q} N={N}] residual rel={e_res:.1e} "
        f"solution rel fp64={errs[0]:.1e} fp32={errs[1]:.1e}")
    assert e_res < 1e-13
    assert errs[0] < 1e-10 and errs[1] < 1e-8, errs


@pytest.mark.parametrize("M", sorted(MESHES))
@pytest.mark.parametrize("q", [0, 1])
@pytest.mark.parametrize("R", sorted(DIRECT_NEWTON))
def test_cavity_newton_steps_with_exact_linear_solves(M, q, R):
    torch_cuda()
    p = w.cavity_problem(M, MESHES[M], q, 20, R)
    G = gpu_problem(p, smoother_prec=1, newton_rtol=1e-8, gmres_rtol=1e-12)
    U = G.vec()
    st = G.newton_solve(U)
    G.close()
    f = st["fnorm"]
    log(f"[cavity {M}x{M} q={q} R={R:g} exact linear] newton={st['newton']} "
        f"(paper {DIRECT_NEWTON[R]}) final ratio={f[-1] / f[0]:.1e}")
    assert st["newton"] == DIRECT_NEWTON[R]


@pytest.mark.parametrize("key", sorted(PAPER_EW))
def test_cavity_eisenstat_walker_runs(key):
    torch_cuda()
    M, q, R = key
    p = w.cavity_problem(M, MESHES[M], q, 20, R)
    G = gpu_problem(p, smoother_prec=1, newton_rtol=1e-8, newton_ew=1)
    U = G.vec()
    st = G.newton_solve(U)
    G.close()
    pn, pl = PAPER_EW[key]
    lin = sum(st["linear"])
    log(f"[cavity {M}x{M} q={q} R={R:g} ew] newton={st['newton']} linear={lin} "
        f"per step={st['linear']} paper={pn} ({pl})")
    assert st["fnorm"][-1] <= 1e-8 * st["fnorm"][0]
    assert st["newton"] <= 5
    assert lin <= 24
