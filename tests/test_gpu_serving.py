"""Continuous-batching server (stwr_server_*) on the GPU: results in the mix
equal the same solve run alone, FP32-smoother solutions match the oracle's
exact discrete solution to 1e-8, and HBM-budget admission behaves."""
import numpy as np
import pytest

import stwr_workloads as w
from gpu_common import gpu_problem, log, rel, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def mix():
    return [w.small_problem(8, 2, 1, 4, 10.0, seed=31),
            w.small_problem(16, 2, 0, 6, 3.0, seed=32),
            w.small_problem(8, 2, 0, 3, 1.0, seed=33),
            w.small_problem(16, 2, 1, 3, 20.0, seed=34),
            w.small_problem(8, 1, 1, 2, 5.0, seed=35),
            w.small_problem(16, 2, 0, 8, 10.0, seed=36)]


def opts(prec=1):
    from paper_2407_13997_amd import binding
    o = binding.default_opts()
    o.smoother_prec = prec
    return o


def test_mix_equals_alone_and_oracle():
    torch_cuda()
    from paper_2407_13997_amd import binding
    from oracle.assembly import Level
    from oracle.direct import solve_slab_by_slab
    from oracle.mms import MMS
    probs = mix()
    srv = binding.Server(0, n_slots=3)
    ids = [srv.submit(p, opts()) for p in probs]
    assert srv.wait(300.0)
    res = {r["id"]: r for r in srv.poll()}
    srv.close()
    assert sorted(res) == sorted(ids)
    starts = sorted((r["start_time"], r["end_time"]) for r in res.values())
    overlap = any(starts[i + 1][0] < starts[i][1] for i in range(len(starts) - 1))
    slots = sorted({r['slot'] for r in res.values()})
    log(f"[serve] overlap in flight: {overlap}; slots used {slots}")
    # continuous batching, not a queue: solves were in flight together on
    # more than one slot
    assert overlap and len(slots) > 1
    for rid, p in zip(ids, probs):
        r = res[rid]
        assert r["status"] == 0, r
        G = gpu_problem(p, smoother_prec=1)
        U = G.vec()
        st = G.newton_solve(U)
        alone = to_host(U)
        e_alone = rel(r["solution"], alone)
        lev = Level(p.mesh_n, p.q, p.n_slabs, p.t_final,
                    MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds))
        e_exact = rel(r["solution"], solve_slab_by_slab(lev))
        log(f"[serve] id={rid} M={p.mesh_n} q={p.q} N={p.n_slabs} Re={p.reynolds} newton={r['newton_its']} "
            f"linear={r['linear_its']} vs alone {e_alone:.1e} vs exact {e_exact:.1e}")
        assert r["newton_its"] == st["newton"]
        assert e_alone <= 1e-12
        assert e_exact <= 1e-8


def test_budget_admission():
    torch_cuda()
    from paper_2407_13997_amd import binding
    probs = [w.small_problem(8, 2, 1, 4, 10.0, seed=40 + k) for k in range(3)]
    sizes = [binding.problem_bytes(p, opts()) + p.n_st * 8 for p in probs]
    assert len(set(sizes)) == 1
    # a budget that holds one request but never two at once
    budget = sizes[0] * 3 // 2
    srv = binding.Server(0, n_slots=3, hbm_budget=budget)
    for p in probs:
        srv.submit(p, opts(), want_solution=False)
    big = w.small_problem(32, 3, 1, 8, 1.0, seed=37)
    srv.submit(big, opts(), want_solution=False)
    assert srv.wait(300.0)
    res = sorted(srv.poll(), key=lambda r: r["id"])
    srv.close()
    assert res[-1]["status"] == -3 and res[-1]["slot"] == -1   # larger than the whole budget
    done = sorted((r["start_time"], r["end_time"]) for r in res[:-1])
    assert all(r["status"] == 0 for r in res[:-1])
    for i in range(len(done) - 1):
        assert done[i + 1][0] >= done[i][1] - 1e-6, done   # never two in flight
    log(f"[serve] budget {budget} serialised {len(done)} solves; oversize request rejected")


def test_heat_and_navier_stokes_requests_in_one_mix():
    """Heat requests (P1 and P3 lattices, whose solution lengths are smaller
    and larger than the Navier-Stokes count of the same mesh) served together
    with Navier-Stokes ones: every solution has its problem's length and
    equals the same solve run alone."""
    torch_cuda()
    from paper_2407_13997_amd import binding
    probs = [w.heat_problem(8, 2, 1, 1, 5), w.small_problem(8, 2, 1, 4, 10.0, seed=31),
             w.heat_problem(8, 2, 3, 1, 5), w.small_problem(8, 2, 0, 3, 1.0, seed=33),
             w.heat_problem(8, 2, 2, 0, 4)]
    srv = binding.Server(0, n_slots=3)
    ids = [srv.submit(p, opts()) for p in probs]
    assert srv.wait(300.0)
    res = {r["id"]: r for r in srv.poll()}
    srv.close()
    assert sorted(res) == sorted(ids)
    for rid, p in zip(ids, probs):
        r = res[rid]
        assert r["status"] == 0, r
        assert r["solution"].size == binding.problem_n_st(p) == p.n_st
        G = gpu_problem(p, smoother_prec=1)
        U = G.vec()
        assert U.numel() == p.n_st
        G.newton_solve(U)
        e_alone = rel(r["solution"], to_host(U))
        log(f"[serve mix] id={rid} equation={p.equation} k={p.degree} M={p.mesh_n} q={p.q} "
            f"N={p.n_slabs} n_st={p.n_st} vs alone {e_alone:.1e}")
        assert e_alone <= 1e-12
        G.close()
