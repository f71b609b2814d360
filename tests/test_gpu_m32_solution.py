"""The 32x32, P2-P1 x DG(1), 32-slab, Re 100 workload at full size (577,728
space-time DoFs): the GPU Newton-FGMRES-WRMG solve, with FP64 and with FP32
patch factors/relaxation, against the oracle's exact discrete solution
(sampled entries and norms in
tests/golden/ns_p2p1_dg1_m32_n32_re100_reference.json, written by
tests/golden/make_m32_reference.py from the oracle alone).

The hierarchy has 3 levels (coarsest 8x8): with the workload's 4 levels
(coarsest 4x4) the rediscretised coarsest operator at Re 100 is too
convection-dominated and FGMRES stalls; test_m32_four_levels_stalls records
that behaviour."""
import json
import os

import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, to_host, torch_cuda

pytestmark = pytest.mark.gpu
REF = os.path.join(os.path.dirname(__file__), "golden", "ns_p2p1_dg1_m32_n32_re100_reference.json")


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-8)])
def test_m32_solution(prec, tol):
    torch_cuda()
    ref = json.load(open(REF))
    p0 = w.named_problem(w.MEDIUM)
    p = w.Problem(p0.mesh_n, 3, p0.q, p0.n_slabs, p0.t_final, p0.reynolds,
                  p0.psi_ab, p0.psi_coef, p0.p_ab, p0.p_coef, seed=p0.seed)
    # Newton is driven to 1e-13 (not the workload's 1e-10) so that the solution,
    # not the stopping point, is compared: at 1e-10 the remaining residual,
    # amplified by the conditioning of the space-time Jacobian, leaves the
    # iterate ~1e-8 from the exact discrete solution in any precision
    G = gpu_problem(p, smoother_prec=prec, newton_rtol=1e-13)
    U = G.vec()
    assert U.numel() == ref["n_st"]
    st = G.newton_solve(U)
    u = to_host(U)
    idx = np.array(ref["index"])
    val = np.array(ref["value"])
    e_sample = np.abs(u[idx] - val).max() / ref["norminf"]
    e_norm = abs(np.linalg.norm(u) - ref["norm2"]) / ref["norm2"]
    log(f"[m32 prec={prec}] newton={st['newton']} linear={st['linear']} "
        f"sampled max err {e_sample:.2e} norm err {e_norm:.2e}")
    assert st["fnorm"][-1] <= 1e-13 * st["fnorm"][0]
    assert e_sample < tol and e_norm < tol


def test_m32_four_levels_stalls():
    """The workload's own 4-level hierarchy (coarsest 4x4), FP64 smoother:
    the first Newton step (at the zero start, where the convection is that of
    the boundary data alone) converges in FGMRES(30), but the second step's
    FGMRES stalls: after 90 iterations its residual is still above 1e-2 of the
    right-hand side.  Newton stops with STWR_ERR_NOT_CONVERGED after its
    2-step limit and the statistics are filled.  The 3-level hierarchy above
    converges on the same problem."""
    torch_cuda()
    from paper_2407_13997_amd import binding
    p = w.named_problem(w.MEDIUM)
    assert p.n_levels == 4
    G = gpu_problem(p, newton_maxit=2, gmres_maxit=90)
    U = G.vec()
    st = binding.Stats()
    rc = G.lib.stwr_newton_solve(G.h, binding._ptr(U), binding.ctypes.byref(st))
    d = st.as_dict()
    log(f"[m32 4 levels] rc={rc} newton={d['newton']} linear={d['linear']} "
        f"linear_rel={d['linear_rel']} fnorm={d['fnorm']} lambda={d['lambda'][:3]}")
    assert rc == -7
    assert d["newton"] == 2 and d["linear"][0] < 90 and d["linear"][1] == 90
    assert d["linear_rel"][0] <= 1e-10 and d["linear_rel"][1] > 1e-2
    assert np.all(np.isfinite(to_host(U)))
