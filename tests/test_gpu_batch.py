"""Batched solves (stwr_batch_*) against the same problems solved alone.

Every problem of a batch runs the operations of stwr_newton_solve with FP32
patch factors and sweeps and the plain sweep in time, in the same order; its
patch factorizations and sweeps share persistent launches with the other
problems of the batch.  Each result must equal the solo solve with the same
options bit for bit (the iteration counts equal), with and without the
captured V-cycle graph, for problems added before the first step and while
others are running; one problem is checked against the oracle's exact
discrete solution (1e-8, the FP32-smoother bar).  A problem that does not
fit the context's budget is rejected with nothing kept."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import ctx, gpu_problem, log, rel, to_host, torch_cuda

pytestmark = pytest.mark.gpu

# uneven problems: meshes 8 and 16 (2 and 3 levels), q = 0 and 1, 3..9 slabs
SPECS = [(8, 2, 1, 5, 10.0, 501), (16, 3, 0, 9, 3.0, 502), (8, 2, 0, 7, 1.0, 503),
         (16, 2, 1, 3, 30.0, 504), (8, 3, 1, 4, 5.0, 505)]


def opts():
    from paper_2407_13997_amd import binding
    o = binding.default_opts()
    o.smoother_prec = binding.FP32
    o.time_chunks = 1
    return o


def problems():
    return [w.small_problem(m, l, q, n, re, s) for (m, l, q, n, re, s) in SPECS]


_solo = {}


def solo(p):
    if p.seed not in _solo:
        G = gpu_problem(p, smoother_prec=1, time_chunks=1)
        U = G.vec()
        st = G.newton_solve(U)
        _solo[p.seed] = (to_host(U), st)
        G.close()
    return _solo[p.seed]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_equals_solo(use_graph):
    torch_cuda()
    from paper_2407_13997_amd import binding
    probs = problems()
    B = binding.Batch(ctx(), use_graph=use_graph)
    ids = {B.add(p, opts()): p for p in probs}
    log(f"[batch graph={use_graph}] {len(ids)} problems added")
    res = B.run(max_steps=5000)
    info = B.info()
    B.close()
    log(f"[batch graph={use_graph}] info {info}")
    assert len(res) == len(probs)
    for r in res:
        p = ids[r["id"]]
        u_solo, st = solo(p)
        e = rel(r["solution"], u_solo)
        log(f"[batch graph={use_graph}] M={p.mesh_n} q={p.q} N={p.n_slabs} status={r['status']} "
            f"newton={r['newton_its']} (solo {st['newton']}) linear={r['linear_its']} "
            f"(solo {st['linear_total']}) rel diff {e:.1e}")
        assert r["status"] == 0
        assert r["newton_its"] == st["newton"] and r["linear_its"] == st["linear_total"]
        # the same operations in the same order, and no atomic or timed choice
        # among them: the same bits
        assert np.array_equal(r["solution"], u_solo)
    assert info["sweep_tile_q0"] > 0 and info["sweep_tile_q1"] > 0
    assert info["graph_captures"] > 0 if use_graph else info["graph_captures"] == 0


def test_batch_continuous_admission_and_oracle():
    """Problems added while others are in their Krylov phase join at the next
    step; all results equal their solo solves; the first matches the oracle's
    exact discrete solution."""
    torch_cuda()
    from oracle.assembly import Level
    from oracle.direct import solve_slab_by_slab
    from oracle.mms import MMS
    from paper_2407_13997_amd import binding
    probs = problems()
    B = binding.Batch(ctx())
    ids = {}
    for p in probs[:2]:
        ids[B.add(p, opts())] = p
    res = []
    for _ in range(4):
        B.step()
        res += B.poll()
    for p in probs[2:]:
        ids[B.add(p, opts())] = p
    log(f"[batch continuous] {len(ids)} problems, 3 added after 4 steps")
    res += B.run(max_steps=5000)
    B.close()
    assert len(res) == len(probs)
    for r in res:
        p = ids[r["id"]]
        u_solo, st = solo(p)
        e = rel(r["solution"], u_solo)
        log(f"[batch continuous] seed={p.seed} newton={r['newton_its']} linear={r['linear_its']} rel diff {e:.1e}")
        assert r["status"] == 0 and np.array_equal(r["solution"], u_solo)
    p = probs[0]
    lev = Level(p.mesh_n, p.q, p.n_slabs, p.t_final, MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds))
    xs = solve_slab_by_slab(lev).ravel()
    r0 = [r for r in res if ids[r["id"]] is p][0]
    e = rel(r0["solution"], xs)
    log(f"[batch continuous] vs oracle exact solution {e:.1e}")
    assert e <= 1e-8


def test_batch_budget_rejection():
    torch_cuda()
    from paper_2407_13997_amd import binding
    p = problems()[1]
    small = binding.Context(0, hbm_budget=binding.problem_bytes(p, opts()) // 2)
    B = binding.Batch(small)
    with pytest.raises(binding.StwrError) as e:
        B.add(p, opts())
    assert e.value.code == -3
    assert small.bytes_in_use() == 0
    assert B.info()["live"] == 0
    B.close()
    small.close()


def test_batch_rejects_p3p2():
    """The batch's sweep and factorization kernels take P2-P1 patches (at
    most 39 DoFs): a P3-P2 problem (81-DoF patches) is refused as an
    argument error before anything is created."""
    torch_cuda()
    from paper_2407_13997_amd import binding
    p = w.small_problem(8, 2, 0, 3, 1.0, 506, degree=2)
    c = binding.Context(0)
    B = binding.Batch(c)
    with pytest.raises(binding.StwrError) as e:
        B.add(p, opts())
    assert e.value.code == -1
    assert c.bytes_in_use() == 0 and B.info()["live"] == 0
    B.close()
    c.close()
