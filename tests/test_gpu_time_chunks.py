"""Cyclic reduction in time (Sec. 3.1, single-GPU form): sweeps split into
time chunks, each swept from zero incoming slab-end values, joined by the
per-patch recurrence over the chunk transfer matrices and swept again.  The
result is the plain forward substitution of eq. waveform_patch_solve up to
rounding, so the oracle's patch smoother is the reference, for Navier-Stokes
(Vanka+star patches, q = 0, 1) and the heat equation (vertex stars,
q = 1, 3), with chunk counts that do and do not divide N; the autotuned
solve matches the plain one."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, oracle_hierarchy, rel, seeded, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _patch_apply(p, chunks, prec, r):
    G = gpu_problem(p, smoother_prec=prec, time_chunks=chunks)
    U = G.vec()
    G.assemble(U)
    G.patch_factor(0, prec)
    G.setup_smoothers()
    z = G.vec()
    G.patch_apply(0, to_dev(r), z)
    got = G.time_chunks(0)
    G.close()
    return to_host(z), got


@pytest.mark.parametrize("q,N", [(0, 7), (1, 5), (1, 16)])
def test_ns_chunked_patch_apply_matches_oracle(q, N):
    torch_cuda()
    p = w.small_problem(8, 2, q, N, 30.0, 101)
    H = oracle_hierarchy(p)
    H.assemble(np.zeros(H.levels[0].n_st))
    r = seeded(H.levels[0].n_st, 5)
    ref = H.smoothers[0].apply(r)
    errs = {}
    for c in (2, 3, 4, N):
        z, got = _patch_apply(p, c, 0, r)
        errs[(c, got)] = rel(z, ref)
        assert errs[(c, got)] < 1e-12, (c, got, errs[(c, got)])
    z32p, _ = _patch_apply(p, 1, 1, r)
    z32c, _ = _patch_apply(p, 3, 1, r)
    e32 = rel(z32c, z32p)
    log(f"[chunks ns q={q} N={N}] fp64 " + " ".join(f"c={c}->{g}:{e:.1e}" for (c, g), e in errs.items())
        + f" fp32 chunked vs plain {e32:.1e} vs oracle {rel(z32c, ref):.1e}")
    assert e32 < 1e-5


@pytest.mark.parametrize("k,q", [(2, 1), (3, 3)])
def test_heat_chunked_patch_apply_matches_oracle(k, q):
    torch_cuda()
    from oracle.heat import HeatHierarchy
    N = 9
    p = w.heat_problem(8, 2, k, q, N)
    H = HeatHierarchy(8, 2, k, q, N, 0.02, None, "gauss")
    r = seeded(H.levels[0].n_st, 6)
    ref = H.smoothers[0].apply(r)
    errs = {}
    for c in (2, 4, 9):
        for prec, tol in ((0, 1e-12), (1, 1e-5)):
            G = gpu_problem(p, smoother_prec=prec, time_chunks=c)
            G.setup_smoothers()
            z = G.vec()
            G.patch_apply(0, to_dev(r), z)
            errs[(c, prec)] = rel(to_host(z), ref)
            G.close()
            assert errs[(c, prec)] < tol, (c, prec, errs[(c, prec)])
    log(f"[chunks heat k={k} q={q}] " + " ".join(f"c={c} p={pr}:{e:.1e}" for (c, pr), e in errs.items()))


def test_autotuned_solves_match_plain():
    torch_cuda()
    p = w.small_problem(16, 2, 1, 48, 10.0, 102)
    res = {}
    for chunks in (1, 0):
        G = gpu_problem(p, smoother_prec=1, newton_rtol=1e-10, time_chunks=chunks)
        U = G.vec()
        st = G.newton_solve(U)
        res[chunks] = (to_host(U), st["newton"], sum(st["linear"]), G.time_chunks(0), G.time_chunks(1))
        G.close()
    log(f"[chunks auto] plain its={res[1][1:3]} tuned its={res[0][1:3]} chosen={res[0][3:]} "
        f"diff={rel(res[0][0], res[1][0]):.1e}")
    assert rel(res[0][0], res[1][0]) < 1e-8
    assert res[0][1] == res[1][1]
    assert abs(res[0][2] - res[1][2]) <= res[1][1]
