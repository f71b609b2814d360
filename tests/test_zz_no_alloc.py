"""stwr_patch_apply_noalloc (patch outputs in the library's fixed per-device
area, no allocation) against stwr_patch_apply (the level's own output buffer),
through the C ABI: two calls in a row, the second on a smaller problem, FP64
and FP32 factors, and a level too large for the area rejected with
STWR_ERR_ARG.  Both entry points run the same kernels on the same inputs in
the same order, so the outputs agree bit for bit."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, seeded, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _pair(prob, prec, seed):
    torch = torch_cuda()
    G = gpu_problem(prob, smoother_prec=prec, time_chunks=1)
    n = G.sizes(0)[0]
    G.assemble(to_dev(seeded(n, seed, 0.3)))
    G.patch_factor(0, prec)
    r = to_dev(seeded(n, seed + 1))
    z1, z2 = G.vec(0), G.vec(0)
    z2.fill_(7.0)
    G.patch_apply(0, r, z1)
    G.patch_apply_noalloc(0, r, z2)
    torch.cuda.synchronize()
    a, b = to_host(z1), to_host(z2)
    G.close()
    return a, b


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_patch_apply_two_calls(prec):
    big = w.small_problem(16, 2, 1, 9, 10.0, 901)
    small = w.small_problem(4, 2, 0, 3, 1.0, 902)
    for name, prob, seed in (("16x16 q=1 N=9", big, 910), ("4x4 q=0 N=3", small, 920)):
        log(f"[noalloc] prec={prec} {name}")
        a, b = _pair(prob, prec, seed)
        log(f"[noalloc] prec={prec} {name} n={a.size} max|diff|={np.max(np.abs(a - b)):.1e}")
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)


def test_noalloc_rejects_level_beyond_area():
    from paper_2407_13997_amd import binding
    torch_cuda()
    # 64x64, q = 1, 40 slabs: 157,071 patch DoFs x 80 values x 8 bytes (100 MB) > 64 MiB
    prob = w.small_problem(64, 4, 1, 40, 10.0, 903)
    G = gpu_problem(prob)
    n = G.sizes(0)[0]
    r, z = G.vec(0), G.vec(0)
    with pytest.raises(binding.StwrError) as e:
        G.patch_apply_noalloc(0, r, z)
    log(f"[noalloc] rejected: {e.value}")
    assert e.value.code == -1 and "scratch" in str(e.value)
    assert n == prob.n_st
    G.close()
