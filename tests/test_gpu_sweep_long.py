"""The WR patch sweep over many slabs (eq. waveform_patch_solve) against the
oracle's patch smoother, element by element.

The FP32 sweep kernel stages the residual 16 values of a DoF at a time (8
slabs at q = 1, 16 at q = 0) and writes its outputs every 32 (q = 1) or 64
(q = 0) slabs; N = 37 and N = 40 cross several staging boundaries and, at
q = 1, an output flush, and end on a ragged tail (37 divides by neither);
N = 70 at q = 0 crosses a flush there.  The 8x8 mesh has interior patches
(nb = 39, the compile-time specialisation) and every boundary patch size.
Each case is checked for one patch application and for one and three
Chebyshev relaxation sweeps, FP64 and FP32 factors, plain and time-chunked.

Bars.  FP64: every slab's max |error| within 1e-12 of that slab's largest
output, and every entry of at least 1% of it within 1e-10 relative.  FP32:
the inverse blocks are rounded to 2^-24 (6e-8) relative per entry and each
output is a sum over at most seven patches of 78-term products, amplified
along the slab chain by the jump coupling (a contraction), which puts the
error near 1e-6 of the output; a slab's max |error| must stay within 1e-5 of
its largest output and an entry of at least 1% of it within 1e-4 relative.
A wrong slab, residual line, flush or tail gives errors of order one."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import entrywise, gpu_problem, log, seeded, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [(1, 37), (1, 40), (0, 37), (0, 40), (0, 70)]
BARS = {0: (1e-12, 1e-10), 1: (1e-5, 1e-4)}

_cache = {}


def oracle_case(q, N):
    """Oracle level 0 of an 8x8 problem, its Jacobian at a seeded state and
    its patch smoother (level 0 only: no coarse levels are needed)."""
    if (q, N) in _cache:
        return _cache[(q, N)]
    from oracle.assembly import Level
    from oracle.mms import make_flow
    from oracle.smoother import PatchSmoother
    prob = w.small_problem(8, 2, q, N, 10.0, 300 + 10 * q + N)
    lev = Level(8, q, N, 1.0, make_flow(prob))
    U = seeded(lev.n_st, 400 + N, 0.3)
    A = lev.jacobian(U.reshape(lev.n_free, lev.N, lev.nq))
    S = PatchSmoother(lev, A)
    _cache[(q, N)] = (prob, lev, U, A, S)
    return _cache[(q, N)]


def gpu_case(prob, U, chunks, prec):
    """GPU problem assembled at U with the smoothers of every level set up at
    precision prec and the sweeps split into `chunks` time chunks."""
    G = gpu_problem(prob, time_chunks=chunks, smoother_prec=prec)
    G.assemble(to_dev(U))
    G.setup_smoothers()
    return G


@pytest.mark.parametrize("q,N", CASES)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("chunks", [1, 3])
def test_patch_apply_long(q, N, prec, chunks):
    torch_cuda()
    prob, lev, U, A, S = oracle_case(q, N)
    log(f"[sweep long] apply q={q} N={N} prec={prec} chunks={chunks}")
    r = seeded(lev.n_st, 500 + N)
    ref = S.apply(r)
    G = gpu_case(prob, U, chunks, prec)
    assert G.time_chunks(0) == chunks
    z = G.vec(0)
    G.patch_apply(0, to_dev(r), z)
    es, ee = entrywise(to_host(z), ref, lev.n_free, N, lev.nq)
    log(f"[sweep long] apply q={q} N={N} prec={prec} chunks={chunks} slab {es:.2e} entry {ee:.2e}")
    G.close()
    assert es <= BARS[prec][0] and ee <= BARS[prec][1]


@pytest.mark.parametrize("q,N", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_relax_long(q, N, prec):
    from oracle.smoother import chebyshev
    torch_cuda()
    prob, lev, U, A, S = oracle_case(q, N)
    G = gpu_case(prob, U, 1, prec)
    b, x0 = seeded(lev.n_st, 600 + N), seeded(lev.n_st, 700 + N)
    a, bnd = 1.9, 8.3
    for steps in (1, 3):
        log(f"[sweep long] relax q={q} N={N} prec={prec} steps={steps}")
        x = to_dev(x0)
        G.relax(0, to_dev(b), x, steps, a, bnd)
        xo = chebyshev(A, S.apply, b, x0, steps, a, bnd)
        es, ee = entrywise(to_host(x) - x0, xo - x0, lev.n_free, N, lev.nq)
        log(f"[sweep long] relax q={q} N={N} prec={prec} steps={steps} slab {es:.2e} entry {ee:.2e}")
        assert es <= BARS[prec][0] and ee <= BARS[prec][1]
    G.close()


@pytest.mark.parametrize("q,N", [(1, 37), (0, 40)])
def test_relax_f32_residual_is_the_rounded_fp64_one(q, N):
    """With FP32 factors a relaxation sweep stores the residual rounded to
    FP32 and the sweep reads it; a patch application on the FP64 residual
    rounds it on reading instead.  Both must give the same correction bit for
    bit: one sweep from x0 equals x0 + (2 / (a + bnd)) M^-1 (b - A x0)."""
    torch = torch_cuda()
    prob, lev, U, A, S = oracle_case(q, N)
    G = gpu_case(prob, U, 1, 1)
    b, x0 = to_dev(seeded(lev.n_st, 800 + N)), to_dev(seeded(lev.n_st, 900 + N))
    a, bnd = 1.9, 8.3
    x = x0.clone()
    G.relax(0, b, x, 1, a, bnd)
    r, z = G.vec(0), G.vec(0)
    G.residual(0, b, x0, r)
    G.patch_apply(0, r, z)
    ref = x0 + (1.0 / (0.5 * (a + bnd))) * z
    log(f"[sweep long] f32 residual q={q} N={N} max diff {float((x - ref).abs().max()):.3e}")
    G.close()
    assert torch.equal(x, ref)
