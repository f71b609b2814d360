"""Failure paths of the C ABI, each forced from the host, with every kernel
exiting normally: a problem larger than the context's HBM budget (rejected
before anything is allocated), a non-finite right-hand side, iteration
limits (statistics still filled), a non-finite linearisation state (zero or
non-finite pivots), calls made before the data they need exists, and bad
arguments.  After each failure the problem stays usable."""
import math

import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, torch_cuda

pytestmark = pytest.mark.gpu

ERR_ARG, ERR_BUDGET, ERR_SINGULAR, ERR_NONFINITE, ERR_NOT_CONVERGED, ERR_STATE = -1, -3, -5, -6, -7, -8


def _problem():
    return w.small_problem(8, 2, 1, 4, 10.0, 11)


def _ready(p, **opt):
    G = gpu_problem(p, **opt)
    U = G.vec()
    G.assemble(U)
    G.setup_smoothers()
    return G


def _rhs(G, seed):
    """A right-hand side in the operator's range (A times a seeded vector), so
    the pressure null space leaves FGMRES a consistent system."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(G.sizes(0)[0], generator=g, dtype=torch.float64).to("cuda")
    b = G.vec()
    G.apply(0, v, b)
    return b


def test_budget_rejects_before_allocating():
    torch_cuda()
    from paper_2407_13997_amd import binding
    p = _problem()
    need = binding.problem_bytes(p)
    small = binding.Context(0, hbm_budget=need // 2)
    before = small.bytes_in_use()
    with pytest.raises(binding.StwrError) as e:
        binding.Problem(small, p, binding.default_opts())
    assert e.value.code == ERR_BUDGET
    assert small.bytes_in_use() == before
    roomy = binding.Context(0, hbm_budget=2 * need)
    P = binding.Problem(roomy, p, binding.default_opts())
    assert roomy.bytes_in_use() >= need
    P.close()
    assert roomy.bytes_in_use() == 0
    small.close()
    roomy.close()


def test_nonfinite_right_hand_side():
    torch_cuda()
    from paper_2407_13997_amd import binding
    G = _ready(_problem())
    b = _rhs(G, 1)
    b[17] = float("nan")
    x = G.vec()
    with pytest.raises(binding.StwrError) as e:
        G.fgmres(b, x)
    assert e.value.code == ERR_NONFINITE
    st = G.fgmres(_rhs(G, 2), x)
    assert math.isfinite(float(x.norm())) and st["final_rel_residual"] <= 1e-10
    G.close()


def test_iteration_limits_fill_statistics():
    torch_cuda()
    from paper_2407_13997_amd import binding
    p = _problem()
    G = _ready(p, gmres_maxit=1, gmres_rtol=1e-12)
    b, x = _rhs(G, 3), G.vec()
    with pytest.raises(binding.StwrError) as e:
        G.fgmres(b, x)
    assert e.value.code == ERR_NOT_CONVERGED
    st = G.fgmres(b, x, allow_unconverged=True)
    assert st["linear_total"] == 1 and st["final_rel_residual"] > 1e-12
    G.close()
    G = gpu_problem(p, newton_maxit=1, newton_rtol=1e-14)
    U = G.vec()
    with pytest.raises(binding.StwrError) as e:
        G.newton_solve(U)
    assert e.value.code == ERR_NOT_CONVERGED
    U.zero_()
    st = G.newton_solve(U, allow_unconverged=True)
    assert st["newton"] == 1 and st["fnorm"][1] < st["fnorm"][0]
    G.close()


def test_nonfinite_state_reports_singular_pivots():
    torch_cuda()
    from paper_2407_13997_amd import binding
    G = gpu_problem(_problem())
    U = G.vec()
    U.fill_(float("nan"))
    with pytest.raises(binding.StwrError) as e:
        G.assemble(U)
    assert e.value.code == ERR_SINGULAR
    U.zero_()
    G.assemble(U)
    G.setup_smoothers()
    x = G.vec()
    st = G.fgmres(_rhs(G, 4), x)
    assert st["final_rel_residual"] <= 1e-10
    G.close()


def test_calls_out_of_order_and_bad_arguments():
    torch_cuda()
    from paper_2407_13997_amd import binding
    G = gpu_problem(_problem())
    b, x = G.vec(), G.vec()
    codes = {}
    for name, call in (("vcycle", lambda: G.vcycle(b, x)),
                       ("patch_apply", lambda: G.patch_apply(0, b, x)),
                       ("fgmres", lambda: G.fgmres(b, x)),
                       ("level", lambda: G.apply(7, b, x))):
        with pytest.raises(binding.StwrError) as e:
            call()
        codes[name] = e.value.code
    U = G.vec()
    G.assemble(U)
    with pytest.raises(binding.StwrError) as e:
        G.vcycle(b, x)                       # smoothers not set up yet
    codes["vcycle_no_smoothers"] = e.value.code
    G.close()
    with pytest.raises(binding.StwrError) as e:
        binding.problem_bytes(w.small_problem(6, 3, 1, 4, 1.0, 1))   # 6 not divisible by 4
    codes["mesh"] = e.value.code
    H = gpu_problem(w.heat_problem(8, 2, 1, 0, 3))
    with pytest.raises(binding.StwrError) as e:
        H.velocity_l2_error(H.vec())
    codes["heat_velocity_error"] = e.value.code
    H.close()
    log(f"[errors] {codes}")
    assert codes == {"vcycle": ERR_STATE, "patch_apply": ERR_STATE, "fgmres": ERR_STATE, "level": ERR_ARG,
                     "vcycle_no_smoothers": ERR_STATE, "mesh": ERR_ARG, "heat_velocity_error": ERR_STATE}
