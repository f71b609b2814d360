"""The MFMA blocked Gauss-Jordan inversion of the FP32 patch blocks over 64
rows (the interior Vanka+star patches at q = 1) against the column-at-a-time
register Gauss-Jordan and the oracle's patch solves (Sec. 3, eq.
waveform_patch_solve): one patch application on small meshes and on the
full 128 x 128, q = 1, 64-slab workload's first slabs."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, oracle_hierarchy, rel, seeded, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _apply(p, mfma, r, U=None):
    G = gpu_problem(p, smoother_prec=1, factor_mfma=mfma)
    Ud = G.vec() if U is None else to_dev(U)
    G.assemble(Ud)
    G.patch_factor(0, 1)
    z = G.vec()
    G.patch_apply(0, to_dev(r), z)
    G.close()
    return to_host(z)


@pytest.mark.parametrize("M,N,seed", [(8, 3, 201), (16, 5, 202)])
def test_mfma_factor_matches_register_factor_and_oracle(M, N, seed):
    torch_cuda()
    p = w.small_problem(M, 2, 1, N, 30.0, seed)
    H = oracle_hierarchy(p)
    U = seeded(H.levels[0].n_st, seed, 0.3)
    H.assemble(U)
    r = seeded(H.levels[0].n_st, seed + 1)
    ref = H.smoothers[0].apply(r)
    z_mfma = _apply(p, 1, r, U)
    z_reg = _apply(p, 0, r, U)
    e_mr, e_mo, e_ro = rel(z_mfma, z_reg), rel(z_mfma, ref), rel(z_reg, ref)
    log(f"[factor mfma {M}x{M} N={N}] mfma vs register {e_mr:.1e}, mfma vs oracle {e_mo:.1e}, "
        f"register vs oracle {e_ro:.1e}")
    assert e_mo < 1e-4 and e_mr < 1e-4
    assert e_mo < 3 * e_ro + 1e-6
