"""The WR patch application at the full size of the sweep benchmark
(128x128 mesh, P2-P1 x DG(1), 64 slabs, Re 1000, 18,776,448 space-time DoFs,
16,641 patches), in the launch configuration the benchmark times, against
sampled outputs of the oracle's patch smoother on slabs 0-2 and 8-9 (every
patch that contains a sampled DoF; tests/golden/
ns_p2p1_dg1_m128_n64_re1000_sweep_reference.json, written by
tests/golden/make_m128_sweep_reference.py from the oracle alone).  Slabs 8-9
lie past the FP32 sweep's first 8-slab residual line.

Bars, per sampled slab: FP64 factors, max |error| within 1e-12 of the
slab's largest sampled output and every sample of at least 1% of it within
1e-10 relative; FP32 factors and sweep, 1e-5 and 1e-4 (the FP32 rounding of
the inverse blocks, 6e-8 per entry, summed over 78-term products and at most
seven patches)."""
import json
import os

import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu
REF = os.path.join(os.path.dirname(__file__), "golden",
                   "ns_p2p1_dg1_m128_n64_re1000_sweep_reference.json")


@pytest.mark.parametrize("prec,tol_slab,tol_entry", [(0, 1e-12, 1e-10), (1, 1e-5, 1e-4)])
def test_m128_patch_apply_samples(prec, tol_slab, tol_entry):
    torch = torch_cuda()
    ref = json.load(open(REF))
    p = w.named_problem(w.LARGE)
    G = gpu_problem(p, smoother_prec=prec, time_chunks=1)
    n_st, _, n_patch = G.sizes(0)
    assert n_st == ref["n_st"] and n_patch == 16641
    G.assemble(G.vec())
    G.patch_factor(0, prec)
    r = to_dev(w.seeded_vector(n_st, 4100))
    z = G.vec()
    G.patch_apply(0, r, z)
    torch.cuda.synchronize()
    zh = to_host(z)
    assert np.all(np.isfinite(zh))
    idx = np.array(ref["index"])
    got = zh[idx]
    want = np.array(ref["value"])
    nq = p.q + 1
    slab = (idx // nq) % p.n_slabs
    assert sorted(set(slab.tolist())) == ref["slabs_checked"]
    for n in ref["slabs_checked"]:
        sel = slab == n
        d = np.abs(got[sel] - want[sel])
        wmax = np.max(np.abs(want[sel]))
        big = np.abs(want[sel]) >= 1e-2 * wmax
        e_slab = np.max(d) / wmax
        e_entry = np.max(d[big] / np.abs(want[sel][big]))
        log(f"[m128 patch apply prec={prec}] slab {n}: samples={sel.sum()} slab {e_slab:.2e} "
            f"entry {e_entry:.2e}")
        assert e_slab <= tol_slab and e_entry <= tol_entry
    G.close()
