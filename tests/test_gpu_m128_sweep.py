"""The WR patch application at the full size of the sweep benchmark
(128x128 mesh, P2-P1 x DG(1), 64 slabs, Re 1000, 18,776,448 space-time DoFs,
16,641 patches), in the launch configuration the benchmark times, against
sampled outputs of the oracle's patch smoother (slabs 0-2, every patch that
contains a sampled DoF; tests/golden/ns_p2p1_dg1_m128_n64_re1000_sweep_reference.json,
written by tests/golden/make_m128_sweep_reference.py from the oracle alone).

FP64 factors: within 1e-12 of the oracle.  FP32 factors and sweep: within
the FP32 rounding of 78 x 78 solves, 1e-4 relative to the largest output."""
import json
import os

import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu
REF = os.path.join(os.path.dirname(__file__), "golden",
                   "ns_p2p1_dg1_m128_n64_re1000_sweep_reference.json")


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-4)])
def test_m128_patch_apply_samples(prec, tol):
    torch = torch_cuda()
    ref = json.load(open(REF))
    p = w.named_problem(w.LARGE)
    G = gpu_problem(p, smoother_prec=prec)
    n_st, _, n_patch = G.sizes(0)
    assert n_st == ref["n_st"] and n_patch == 16641
    G.assemble(G.vec())
    G.patch_factor(0, prec)
    r = to_dev(w.seeded_vector(n_st, 4100))
    z = G.vec()
    G.patch_apply(0, r, z)
    torch.cuda.synchronize()
    idx = np.array(ref["index"])
    got = to_host(z)[idx]
    want = np.array(ref["value"])
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    log(f"[m128 patch apply prec={prec}] samples={idx.size} max rel err={err:.2e}")
    assert np.all(np.isfinite(to_host(z)))
    assert err <= tol
    G.close()
