"""Benchmark: space-time DoFs relaxed per second by one waveform-relaxation
Vanka sweep on the finest level of the largest single solve (128x128
triangle-split mesh, Taylor-Hood P2-P1, DG(1) in time, 64 slabs, Re = 1000,
16 stream-function modes), FP32 patch factors with FP64 residual and update.

One timed step = one Chebyshev-weighted relaxation sweep on the finest level:
space-time residual r = b - A x (FP64), waveform-relaxation patch sweep over
all 16,641 vertex patches x 64 slabs (forward block substitution in time),
deterministic gather of the patch corrections fused with the Chebyshev update.
The operator is assembled at the Newton start (the first Jacobian a solve
needs), factors and the eigen-estimate come from the library's setup; none of
that setup is inside the timed region.

Prints ONE JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, AMD-published


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds_budget: float = 5.0) -> dict:
    """Time the oracle's sweep (residual + patch solves + Chebyshev update) on a
    bounded sample with the same per-patch work as the benchmark workload:
    16x16 mesh (289 patches, interior blocks of 78x78 per slab), q = 1,
    64 slabs, Re = 1000; single-threaded BLAS/LAPACK.  First on one core, then
    on every core of the process's affinity set with the patches split over a
    pool of worker processes (each holding the factors of its share of the
    patches), the residual and the update in the parent."""
    code = r"""
import os, sys, time, json
sys.path.insert(0, %r)
import multiprocessing as mp
import numpy as np
import stwr_workloads as w
from oracle.multigrid import Hierarchy, Options
from oracle.smoother import chebyshev, PatchSmoother
prob = w.Problem(16, 2, 1, 64, 1.0, 1000.0, *w.draw_modes(4000, 16, 3, 8), seed=4000)
H = Hierarchy(prob, Options())
L0 = H.levels[0]
H.assemble(L0.initial_guess().ravel(), with_smoothers=False)
sm = PatchSmoother(L0, H.A[0])
b = np.random.default_rng(1).standard_normal(L0.n_st)
x0 = np.random.default_rng(2).standard_normal(L0.n_st)
budget = %f
t0 = time.perf_counter(); n = 0
while True:
    x = chebyshev(H.A[0], sm.apply, b, x0, 1, 5.0, 22.0)
    n += 1
    if time.perf_counter() - t0 > budget: break
dt1 = (time.perf_counter() - t0) / n
cores = len(os.sched_getaffinity(0))
import copy
SHARE = []
for k in range(cores):
    part = copy.copy(sm)
    part.blocks = sm.blocks[k::cores]
    SHARE.append(part)
def work(args):
    k, r = args
    return SHARE[k].apply(r)
ctx = mp.get_context("fork")
with ctx.Pool(cores) as pool:
    def par_apply(r):
        return np.sum(pool.map(work, [(k, r) for k in range(cores)]), axis=0)
    xp = chebyshev(H.A[0], par_apply, b, x0, 1, 5.0, 22.0)
    err = float(np.max(np.abs(xp - x)) / np.max(np.abs(x)))
    t0 = time.perf_counter(); m = 0
    while True:
        chebyshev(H.A[0], par_apply, b, x0, 1, 5.0, 22.0)
        m += 1
        if time.perf_counter() - t0 > budget: break
    dtp = (time.perf_counter() - t0) / m
print(json.dumps({"n_st": L0.n_st, "sweep_s": dt1, "sweeps": n, "cores": cores,
                  "sweep_s_all": dtp, "sweeps_all": m, "all_vs_one_maxrel": err}))
""" % (ROOT, seconds_budget)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    t0 = time.perf_counter()
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=900)
    if res.returncode != 0:
        log(res.stderr[-2000:])
        return {"value": None, "unit": "st-DoF/s", "cores": 1, "kind": "oracle",
                "sample": "failed"}
    out = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": out["n_st"] / out["sweep_s"], "unit": "st-DoF/s", "cores": 1,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": (f"oracle WR sweep (residual + 289 vertex-patch solves x 64 slabs + "
                       f"Chebyshev update) on a 16x16 mesh, q=1, N=64, Re=1000 "
                       f"({out['n_st']} st-DoFs, same per-patch work as the 128x128 workload), "
                       f"{out['sweeps']} sweeps on one core, {out['sweeps_all']} on {out['cores']}, "
                       f"wall {time.perf_counter() - t0:.1f}s incl. setup"),
            "sweep_s": out["sweep_s"],
            "all_cores": {"value": out["n_st"] / out["sweep_s_all"], "unit": "st-DoF/s",
                          "cores": out["cores"], "sweep_s": out["sweep_s_all"],
                          "max_rel_diff_vs_one_core": out["all_vs_one_maxrel"],
                          "how": "patches dealt round-robin to a fork pool of one process per core"},
            "note": "reported baseline, not the target"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mesh", type=int, default=128)
    ap.add_argument("--slabs", type=int, default=64)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-context", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--vcycles", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--no-uneven-batch", action="store_true")
    ap.add_argument("--p3p2-steps", type=int, default=10,
                    help="timed sweeps of the P3-P2 leg (80x80 Chorin, q=1, 10 slabs); 0 skips it")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="also run the Poisson-rate sweep of the batched server (about ten minutes)")
    ap.add_argument("--batch-problems", type=int, default=64)
    ap.add_argument("--largest-solve", type=int, default=0,
                    help="also run the 128x128 Newton solve with this many levels (0: skip)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0)
    ap.add_argument("--read-rate-gib", type=float, default=8.0,
                    help="buffer for the measured HBM read rate (0 = skip)")
    ap.add_argument("--paper-run", default=None,
                    help="only solve this one of the paper's runs and print its record (for profiling): "
                         "chorin_q<q>_n<N>, chorin_p3p2_q<q>_n<N> or cavity_m<M>_q<q>_r<R>")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.paper_run:
        print(json.dumps({"paper_run": paper_run(args.paper_run)}), flush=True)
        return
    prob = w.named_problem(w.LARGE)
    if (args.mesh, args.slabs, args.levels) != (128, 64, 6):
        prob = w.Problem(args.mesh, args.levels, 1, args.slabs, 1.0, 1000.0,
                         prob.psi_ab, prob.psi_coef, prob.p_ab, prob.p_coef, seed=prob.seed)
    prec = binding.FP32 if args.prec == "fp32" else binding.FP64
    ctx = binding.Context(0)
    opts = binding.default_opts()
    opts.smoother_prec = prec
    t = time.perf_counter()
    P = binding.Problem(ctx, prob, opts)
    n_st, nf, n_patch = P.sizes(0)
    log(f"[bench] problem created: n_st={n_st} patches={n_patch} "
        f"bytes={ctx.bytes_in_use() / 1e9:.1f} GB ({time.perf_counter() - t:.1f}s)")
    U = P.vec()
    torch.cuda.synchronize()
    t = time.perf_counter(); P.assemble(U); torch.cuda.synchronize(); t_asm0 = time.perf_counter() - t
    # timed again once the kernels are loaded
    t = time.perf_counter(); P.assemble(U); torch.cuda.synchronize(); t_asm = time.perf_counter() - t
    log(f"[bench] assembled all levels in {t_asm0:.2f}s (first), {t_asm:.2f}s")
    t = time.perf_counter(); P.patch_factor(0, prec); torch.cuda.synchronize(); t_fac = time.perf_counter() - t
    log(f"[bench] factored finest level in {t_fac:.2f}s")
    t = time.perf_counter(); lam = P.eig_estimate(0); t_eig = time.perf_counter() - t
    log(f"[bench] lambda={lam:.6f} ({t_eig:.2f}s)")
    a, bnd = opts.cheb_lo * lam, opts.cheb_hi * lam

    g = torch.Generator(device="cpu").manual_seed(4000)
    b = torch.randn(n_st, generator=g, dtype=torch.float64).to("cuda")
    x = torch.zeros(n_st, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        P.relax(0, b, x, 1, a, bnd)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.kernel_times()   # reset
    # one event between consecutive steps (the library works on torch's
    # current stream), so the per-step distribution comes with the total
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        P.relax(0, b, x, 1, a, bnd)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev[0].elapsed_time(ev[-1])
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    ms_step = ms_total / args.steps
    if not math.isfinite(float(x.norm())):
        raise RuntimeError("relaxation produced non-finite values")
    log(f"[bench] {args.steps} sweeps: {ms_step:.3f} ms/sweep (wall {wall:.3f}s) kernels={kt}")

    # algorithmic bytes of one patch-sweep launch: every (patch, slab) inverse
    # block once, the residual of every patch DoF once per slab, the patch
    # outputs once
    s_f = 4 if prec == binding.FP32 else 8
    sweep_ms, sweep_n = kt["sweep"]
    s_r = 4 if prec == binding.FP32 else 8   # the FP32 sweep reads an FP32-rounded residual
    io_bytes = patch_sweep_bytes(prob, s_f, s_r)
    algo_bytes = patch_sweep_bytes_algorithmic(prob, s_f, n_st, s_r)
    sweep_avg_ms = sweep_ms / max(sweep_n, 1)
    achieved = algo_bytes / (sweep_avg_ms * 1e-3) / 1e9
    achieved_io = io_bytes / (sweep_avg_ms * 1e-3) / 1e9

    # the plain form on the same workload: FP64 factors and sweep (outside
    # the timed region; the FP32 factors are replaced)
    fp64_leg = None
    if prec == binding.FP32 and args.fp64_steps > 0:
        P.patch_factor(0, binding.FP64)
        x64 = torch.zeros(n_st, dtype=torch.float64, device="cuda")
        P.relax(0, b, x64, 2, a, bnd)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        ctx.kernel_times()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.fp64_steps):
            P.relax(0, b, x64, 1, a, bnd)
        e1.record()
        torch.cuda.synchronize()
        kt64 = ctx.kernel_times()
        ctx.set_timing(False)
        ms64 = e0.elapsed_time(e1) / args.fp64_steps
        sw64 = kt64["sweep"][0] / max(kt64["sweep"][1], 1)
        algo64 = patch_sweep_bytes_algorithmic(prob, 8, n_st, 8)
        fp64_leg = {"smoother_prec": "fp64", "ms_per_step": ms64, "value": n_st / (ms64 * 1e-3),
                    "unit": "st-DoF/s", "steps": args.fp64_steps,
                    "kernels_ms_per_sweep": {k: v[0] / max(v[1], 1) for k, v in kt64.items()},
                    "roofline": {"bound": "hbm", "kernel": "k_patch_sweep (FP64)", "avg_ms": sw64,
                                 "algorithmic_bytes": algo64,
                                 "achieved": algo64 / (sw64 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": algo64 / (sw64 * 1e-3) / 1e9 / HBM_PEAK_GBS}}
        log(f"[bench] fp64 sweep: {fp64_leg}")
        P.patch_factor(0, prec)

    # one full V(2,2) cycle on all levels (outside the timed region)
    vc_ms = None
    if args.vcycles > 0:
        P.setup_smoothers()
        vx = P.vec()
        torch.cuda.synchronize()
        tv = time.perf_counter()
        for _ in range(args.vcycles):
            P.vcycle(b, vx)
        torch.cuda.synchronize()
        vc_ms = (time.perf_counter() - tv) / args.vcycles * 1e3
    # the device's attainable HBM read rate (a plain streaming read of 8 GiB,
    # outside the timed region), reported beside the published peak
    read_gbs = None
    if args.read_rate_gib > 0:
        rb = torch.ones(int(args.read_rate_gib * (1 << 30)) // 4, dtype=torch.float32, device="cuda")
        read_gbs = ctx.read_rate(rb, 10)
        del rb
        log(f"[bench] measured HBM read rate {read_gbs:.1f} GB/s")
    if args.copy_calibration_gib > 0:
        # a plain device copy of known size, for scaling hardware byte counters
        nb = int(args.copy_calibration_gib * (1 << 30)) // 8
        src = torch.ones(nb, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nb * 8} bytes done")
        del src, dst

    out = {
        "metric": "space-time DoFs relaxed/s per WR sweep",
        "value": n_st / (ms_step * 1e-3),
        "unit": "st-DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 patch factors/solves (residual input rounded to f32), f64 residual/update"
                  if prec == binding.FP32 else "f64"),
        "data": "synthetic manufactured solution (seeded Fourier modes)",
        "config": {"workload": f"{w.LARGE} finest-level WR sweep" if args.mesh == 128
                   else f"ns_p2p1_dg1_m{args.mesh}_n{args.slabs} finest-level WR sweep",
                   "mesh": args.mesh, "q": 1, "slabs": args.slabs, "reynolds": 1000.0,
                   "levels": args.levels, "st_dofs": n_st, "patches": n_patch,
                   "smoother_prec": args.prec, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (profiled_traffic() if (args.mesh, args.slabs, args.prec) == (128, 64, "fp32")
                                 else None),
                     "kernel": ("k_patch_sweep_f32 (interior + boundary launches)" if prec == binding.FP32
                                else "k_patch_sweep"), "avg_ms": sweep_avg_ms,
                     "algorithmic_bytes": algo_bytes,
                     "measured_read_gbs": read_gbs,
                     "frac_of_measured_read": achieved / read_gbs if read_gbs else None,
                     "algorithmic_bytes_def": f"sum over (patch, slab) of m^2 s_f + {s_r + 16} n_st "
                                              f"(r read, {s_r} bytes; z read-modify-write)",
                     "with_patch_io": {"bytes": io_bytes, "achieved": achieved_io,
                                       "frac": achieved_io / HBM_PEAK_GBS,
                                       "def": f"sum over (patch, slab) of m^2 s_f + {s_r} m + s_f m "
                                              "(each patch's residual gather and its own outputs)"}},
        "ms_per_step_p10_p50_p90": [float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
        "kernels_ms_per_sweep": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "setup_s": {"assemble_all_levels": t_asm, "factor_finest": t_fac, "eig_estimate": t_eig},
        "vcycle_ms": vc_ms,
        "fp64_sweep": fp64_leg,
        "lambda_finest": lam,
    }
    P.close()
    if not args.no_serving:
        out["single_solve"] = single_solve()
        log(f"[bench] single solve: {out['single_solve']}")
        out["serving"] = serving_benchmark()
        log(f"[bench] serving: {out['serving']}")
    if args.p3p2_steps > 0:
        out["p3p2_sweep"] = p3p2_sweep(args.p3p2_steps)
        log(f"[bench] P3-P2 sweep: {out['p3p2_sweep']}")
    if not args.no_uneven_batch:
        out["uneven_batch"] = uneven_batch(args.batch_problems)
        log(f"[bench] uneven batch: {out['uneven_batch']}")
    if args.serving_sweep:
        out["serving_sweep"] = serving_sweep()
        log(f"[bench] serving sweep: {out['serving_sweep']}")
    if args.largest_solve > 0:
        out["largest_solve"] = largest_solve(args.largest_solve)
        log(f"[bench] largest solve: {out['largest_solve']}")
    if not args.no_paper_context:
        out["paper_context"] = paper_context()
        log(f"[bench] paper context: {out['paper_context']}")
        out["paper_context"]["heat"] = heat_context()
        log(f"[bench] heat context: {out['paper_context']['heat']}")
        out["time_chunks"] = time_chunk_context()
        log(f"[bench] time chunks: {out['time_chunks']}")
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    ctx.close()


PROFILE = os.path.join(ROOT, "profiles", "k_patch_sweep_f32_ns_p2p1_dg1_m128_n64_re1000.md")


def profiled_traffic() -> int | None:
    """HBM bytes of one FP32 patch sweep (its interior and boundary launches)
    from the committed rocprofv3 byte counters, only while the kernel source is
    the one that was profiled."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    src = open(os.path.join(ROOT, "paper_2407_13997_amd", "csrc", "patch.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()[:16]
    rec_sha = rec_bytes = None
    for line in text.splitlines():
        if line.startswith("patch.hip sha256 (first 16 hex):"):
            rec_sha = line.split(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch:"):
            rec_bytes = int(line.split(":", 1)[1].strip())
    return rec_bytes if (rec_sha == sha and rec_bytes) else None


# The paper's Chorin runs (Sec. 4.2 tables of errors, times and iterations;
# 80 x 80 mesh, R = 10, t in [0, 0.1], P2-P1, FGMRES-WRMG with Eisenstat-Walker
# tolerances, Newton to 1e-8; 8 Xeon cores at 1.7 GHz, Firedrake/PETSc).
# The q = 1, N = 10 error is printed as 1.77e-3 and read as 1.77e-4.
PAPER_CHORIN = {
    (0, 10): (6.51e-3, 110.0, "4 (11)"), (0, 20): (3.32e-3, 395.3, "4 (11)"),
    (0, 40): (1.70e-3, 2596.8, "4 (11)"), (1, 10): (1.77e-4, 432.2, "4 (12)"),
    (1, 20): (4.60e-5, 1971.7, "4 (10)"), (1, 40): (1.18e-5, 13964.7, "4 (17)"),
}


# The paper's P3-P2 Chorin runs (the spatial-degree-2 columns of the same
# tables; q = 1 at N = 20, 40 ran out of memory there).
PAPER_CHORIN_P3P2 = {
    (0, 10): (6.51e-3, 629.8, "5 (29)"), (0, 20): (3.32e-3, 2326.1, "4 (19)"),
    (0, 40): (1.70e-3, 16979.7, "4 (19)"), (1, 10): (1.77e-4, 2868.7, "5 (26)"),
}


# The paper's lid-driven cavity runs (Sec. 4.3, P2-P1 columns): (mesh, q, R)
# -> (time to solution in s, "Newton (linear)" with Eisenstat-Walker
# tolerances); 40 x 40 and 80 x 80 are its two and three refinements of the
# 10 x 10 base mesh, N = 20, t in [0, 0.02].
PAPER_CAVITY = {
    (40, 1, 1.0): (432.8, "4 (10)"), (40, 1, 10.0): (434.2, "4 (10)"), (40, 1, 100.0): (456.6, "4 (13)"),
    (40, 0, 1.0): (90.6, "4 (10)"), (40, 0, 10.0): (90.3, "4 (11)"), (40, 0, 100.0): (98.8, "4 (15)"),
    (80, 1, 1.0): (1798.1, "4 (8)"), (80, 1, 10.0): (1782.4, "4 (8)"), (80, 1, 100.0): (1894.1, "4 (13)"),
    (80, 0, 1.0): (347.7, "4 (8)"), (80, 0, 10.0): (348.9, "4 (8)"), (80, 0, 100.0): (381.9, "4 (12)"),
}


def _timed_newton(ctx, prob):
    """Newton to 1e-8 with Eisenstat-Walker linear tolerances and the FP32
    smoother, as the paper's runs were set; returns (stats, seconds, error)."""
    import torch
    from paper_2407_13997_amd import binding
    o = binding.default_opts()
    o.smoother_prec = binding.FP32
    o.newton_rtol = 1e-8
    o.newton_ew = 1
    P = binding.Problem(ctx, prob, o)
    U = P.vec()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = P.newton_solve(U)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = P.velocity_l2_error(U) if prob.flow != 2 else None
    P.close()
    return st, dt, err


def paper_run(name: str) -> dict:
    """One of the paper's runs by name, as paper_context runs it: the Chorin
    problem on 80 x 80 (P2-P1 from four levels, P3-P2 from four, five at
    q = 1) or the lid-driven cavity (M = 40 from three levels, 80 from four;
    20 slabs)."""
    import re
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    m = re.fullmatch(r"chorin(_p3p2)?_q([01])_n(\d+)", name)
    if m:
        p3, q, N = m.group(1) is not None, int(m.group(2)), int(m.group(3))
        prob = w.chorin_problem(80, 5 if (p3 and q == 1) else 4, q, N, nodes=1, degree=2 if p3 else 1)
    else:
        m = re.fullmatch(r"cavity_m(40|80)_q([01])_r(\d+)", name)
        if not m:
            raise SystemExit(f"unknown paper run {name!r}")
        M, q, R = int(m.group(1)), int(m.group(2)), float(m.group(3))
        prob = w.cavity_problem(M, 3 if M == 40 else 4, q, 20, R)
    ctx = binding.Context(0)
    st, dt, err = _timed_newton(ctx, prob)
    ctx.close()
    return {"run": name, "st_dofs": prob.n_st, "time_s": dt, "error": err, "newton": st["newton"],
            "linear": list(st["linear"])}


def paper_context() -> dict:
    """The Chorin and lid-driven cavity runs of the paper's tables on this GPU
    (Gauss-Legendre temporal nodes, FP32 smoother, Newton to 1e-8 with
    Eisenstat-Walker linear tolerances, as the paper ran them): space-time
    velocity error (Chorin), Newton (linear) iterations and time to solution,
    beside the paper's figures (context on other hardware, not a target)."""
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    ctx = binding.Context(0)
    chorin, cavity = [], []
    for (q, N), (p_err, p_time, p_its) in sorted(PAPER_CHORIN.items()):
        prob = w.chorin_problem(80, 4, q, N, nodes=1)
        st, dt, err = _timed_newton(ctx, prob)
        chorin.append({"q": q, "N": N, "st_dofs": prob.n_st, "error": err, "paper_error": p_err,
                       "time_s": dt, "paper_time_s": p_time,
                       "iterations": f"{st['newton']} ({sum(st['linear'])})", "paper_iterations": p_its})
    chorin_p3p2 = []
    for (q, N), (p_err, p_time, p_its) in sorted(PAPER_CHORIN_P3P2.items()):
        # five levels at q = 1: the 10 x 10 coarsest bordered blocks of P3-P2
        # x DG(1) would exceed the dense coarse solve's order
        prob = w.chorin_problem(80, 5 if q == 1 else 4, q, N, nodes=1, degree=2)
        st, dt, err = _timed_newton(ctx, prob)
        chorin_p3p2.append({"q": q, "N": N, "levels": prob.n_levels, "st_dofs": prob.n_st, "error": err,
                            "paper_error": p_err, "time_s": dt, "paper_time_s": p_time,
                            "iterations": f"{st['newton']} ({sum(st['linear'])})", "paper_iterations": p_its})
    for (M, q, R), (p_time, p_its) in sorted(PAPER_CAVITY.items()):
        prob = w.cavity_problem(M, 3 if M == 40 else 4, q, 20, R)
        st, dt, _ = _timed_newton(ctx, prob)
        cavity.append({"mesh": M, "q": q, "R": R, "st_dofs": prob.n_st, "time_s": dt,
                       "paper_time_s": p_time,
                       "iterations": f"{st['newton']} ({sum(st['linear'])})", "paper_iterations": p_its})
    ctx.close()
    return {"chorin": chorin, "chorin_p3p2": chorin_p3p2, "cavity": cavity}


# The paper's FGMRES-WRMG heat runs (Sec. 4.1, times to solution at Mref = 3
# and 4, i.e. 80 x 80 and 160 x 160 meshes from a 10 x 10 base; N = 20,
# t in [0, 0.02]): (mesh, k, q) -> seconds on 8 Xeon cores (its P3 runs at
# q = 2, 3 on 160 x 160 ran out of memory)
PAPER_HEAT = {
    (80, 1, 0): 7.0, (80, 2, 0): 17.9, (80, 3, 0): 48.9,
    (80, 1, 1): 14.0, (80, 2, 1): 48.4, (80, 3, 1): 183.1,
    (80, 1, 2): 23.1, (80, 2, 2): 113.4, (80, 3, 2): 424.4,
    (80, 1, 3): 35.3, (80, 2, 3): 187.0, (80, 3, 3): 784.6,
    (160, 1, 0): 21.4, (160, 2, 0): 148.7, (160, 3, 0): 373.4,
    (160, 1, 1): 50.8, (160, 2, 1): 375.5, (160, 3, 1): 1090.0,
    (160, 1, 2): 86.3, (160, 2, 2): 633.6,
    (160, 1, 3): 132.2, (160, 2, 3): 1064.0,
}


def heat_context(sweep_steps: int = 20, runs_too: bool = True) -> dict:
    """The paper's heat runs on this GPU (FP32 smoother, FGMRES to a residual
    reduction of 1e-6 or below 1e-6): iterations and time to solution (problem
    set-up with the operator's assembly, smoother set-up, solve), beside the
    paper's times; and the WR sweep of the largest run (160 x 160, P3 x DG(1),
    9.25 M st-DoFs) against the HBM roofline: per patch its one FP32 inverse
    block (every slab shares it), per (patch, slab) the FP64 residual gather
    and the FP64 output."""
    import numpy as np
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    ctx = binding.Context(0)

    def opts():
        o = binding.default_opts()
        o.smoother_prec = binding.FP32
        o.gmres_rtol = 1e-6
        o.gmres_atol = 1e-6
        return o

    runs = []
    for (M, k, q), p_time in (sorted(PAPER_HEAT.items()) if runs_too else []):
        prob = w.heat_problem(M, 4 if M == 80 else 5, k, q)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = binding.Problem(ctx, prob, opts())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.setup_smoothers()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        b = P.vec()
        P.linear_rhs(b)
        x = P.vec()
        st = P.fgmres(b, x)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        P.close()
        runs.append({"mesh": M, "k": k, "q": q, "st_dofs": prob.n_st, "iterations": st["linear_total"],
                     "paper_iterations": 4 if (M, k, q) == (80, 2, 3) else 3, "time_s": t3 - t0, "create_s": t1 - t0,
                     "smoother_setup_s": t2 - t1, "solve_s": t3 - t2, "paper_time_s": p_time})
    # sweep of the largest run
    prob = w.heat_problem(160, 5, 3, 1)
    P = binding.Problem(ctx, prob, opts())
    P.setup_smoothers()
    lam = P.eig_estimate(0)
    n_st = P.sizes(0)[0]
    g = torch.Generator(device="cpu").manual_seed(4100)
    b = torch.randn(n_st, generator=g, dtype=torch.float64).to("cuda")
    x = torch.zeros(n_st, dtype=torch.float64, device="cuda")
    a, bnd = 0.25 * lam, 1.05 * lam
    P.relax(0, b, x, 2, a, bnd)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.kernel_times()
    t0 = time.perf_counter()
    for _ in range(sweep_steps):
        P.relax(0, b, x, 1, a, bnd)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    nq, N = prob.q + 1, prob.n_slabs
    m = P.patch_sizes(0).astype(np.int64) * nq
    # the heat operator is the same on every slab: one FP32 block per patch,
    # then per slab the FP64 residual gather and the FP64 output
    algo = int(np.sum(m * m * 4) + N * np.sum(8 * m + 8 * m))
    sweep_ms = kt["sweep"][0] / max(kt["sweep"][1], 1)
    achieved = algo / (sweep_ms * 1e-3) / 1e9
    P.close()
    ctx.close()
    return {"runs": runs,
            "sweep": {"workload": "heat_p3_dg1_m160_n20 finest-level WR sweep", "st_dofs": n_st,
                      "ms_per_step": wall / sweep_steps * 1e3,
                      "st_dof_per_s": n_st / (wall / sweep_steps),
                      "kernels_ms_per_sweep": {k2: v[0] / max(v[1], 1) for k2, v in kt.items()},
                      "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                   "kernel": "k_patch_sweep (FP32 block per patch, FP64 outputs)",
                                   "avg_ms": sweep_ms, "algorithmic_bytes": algo}}}


def single_solve() -> dict:
    """The 32 x 32, P2-P1 x DG(1), 32-slab, Re 100 Newton solve to 1e-10 with
    the FP64 smoother (the plain form) and with FP32 patch factors and
    relaxation (FP64 FGMRES, Newton, residual and coarse solve): time,
    iterations, and the relative difference of the two solutions.  Three
    levels (coarsest 8 x 8): with four, the rediscretised 4 x 4 operator is
    too convection-dominated for the V-cycle at Re 100."""
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    base = w.named_problem(w.MEDIUM)
    prob = w.Problem(base.mesh_n, 3, base.q, base.n_slabs, base.t_final, base.reynolds, base.psi_ab,
                     base.psi_coef, base.p_ab, base.p_coef, seed=base.seed)
    ctx = binding.Context(0)
    out, sol = {}, {}
    for name, prec in (("fp64", binding.FP64), ("fp32", binding.FP32)):
        o = binding.default_opts()
        o.smoother_prec = prec
        o.newton_rtol = 1e-10
        P = binding.Problem(ctx, prob, o)
        U = P.vec()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = P.newton_solve(U)
        torch.cuda.synchronize()
        out[name] = {"time_s": time.perf_counter() - t0, "newton": st["newton"],
                     "linear_total": sum(st["linear"])}
        sol[name] = U.clone()
        P.close()
    ctx.close()
    out["workload"] = f"{w.MEDIUM} (3 levels), Newton to 1e-10"
    out["st_dofs"] = prob.n_st
    out["rel_diff_fp32_vs_fp64"] = float((sol["fp32"] - sol["fp64"]).norm() / sol["fp64"].norm())
    out["speedup"] = out["fp64"]["time_s"] / out["fp32"]["time_s"]
    return out


def largest_solve(levels: int, newton_maxit: int = 8, gmres_maxit: int = 120) -> dict:
    """The largest single solve: 128 x 128, P2-P1 x DG(1), 64 slabs, Re 1000,
    16 stream-function modes; Newton to 1e-10 from zero with FGMRES(30)
    preconditioned by V(2,2) cycles over `levels` levels, FP32 patch factors
    and relaxation, FP64 Krylov, Newton, residual and coarsest solve.  Records
    Newton and linear iterations, the residual history, the linear relative
    residual each step reached, time and device bytes."""
    import numpy as np
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    base = w.named_problem(w.LARGE)
    prob = w.Problem(base.mesh_n, levels, base.q, base.n_slabs, base.t_final, base.reynolds, base.psi_ab,
                     base.psi_coef, base.p_ab, base.p_coef, seed=base.seed)
    ctx = binding.Context(0)
    o = binding.default_opts()
    o.smoother_prec = binding.FP32
    o.newton_rtol = 1e-10
    o.newton_maxit = newton_maxit
    o.gmres_maxit = gmres_maxit
    t0 = time.perf_counter()
    P = binding.Problem(ctx, prob, o)
    t_create = time.perf_counter() - t0
    U = P.vec()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = "converged"
    try:
        st = P.newton_solve(U, allow_unconverged=True)
        if st["fnorm"][-1] > 1e-10 * st["fnorm"][0]:
            status = "not converged"
    except binding.StwrError as e:
        st, status = None, str(e)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": f"{w.LARGE} Newton solve, {levels} levels (coarsest {128 >> (levels - 1)}x"
                       f"{128 >> (levels - 1)}), FP32 smoother, newton_maxit {newton_maxit}, "
                       f"FGMRES(30) maxit {gmres_maxit} per step",
           "st_dofs": prob.n_st, "status": status, "create_s": t_create, "solve_s": dt,
           "device_bytes": ctx.bytes_in_use(), "stats": st}
    P.close()
    ctx.close()
    return out


def uneven_batch(n_problems: int = 64, newton_maxit: int = 8, gmres_maxit: int = 30) -> dict:
    """The uneven batch: n_problems independent solves drawn as the batch
    distribution states (meshes {8,16,32,64}^2, N in [8,128], q in {0,1},
    Re log-uniform in [1,1000], seeds 2000+j), Newton to 1e-10 with
    Eisenstat-Walker linear tolerances, at most newton_maxit Newton steps of at
    most gmres_maxit FGMRES(30) iterations each (the unstabilised Galerkin
    convection stalls the V-cycle at the higher Reynolds numbers, and the caps
    bound what those solves cost every path).  Three paths on the same
    problems, all submitted at time zero: the plain FP64-smoother path one solve
    at a time, the FP32-smoother path one at a time, and the FP32 batch
    (stwr_batch_*: shared persistent factor and sweep launches, captured
    V-cycles).  Reports converged solves per second, p50/p99 completion
    latency over the converged solves, and the largest relative difference
    between each FP32 path's solutions and the plain path's."""
    import numpy as np
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    probs = w.batch_problems(n_problems, seed0=2000)
    ctx = binding.Context(0)

    def opts(prec, chunks):
        o = binding.default_opts()
        o.smoother_prec = prec
        o.newton_ew = 1
        o.newton_maxit = newton_maxit
        o.gmres_maxit = gmres_maxit
        o.time_chunks = chunks
        return o

    def summary(lat_ok, span, n_fail):
        lat = np.array(lat_ok) if lat_ok else np.array([np.nan])
        return {"solves": len(lat_ok), "failed": n_fail, "makespan_s": span,
                "solves_per_s": len(lat_ok) / span, "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99))}

    def one_at_a_time(prec):
        sols, lat, fail = {}, [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j, p in enumerate(probs):
            P = binding.Problem(ctx, p, opts(prec, 0))
            U = P.vec()
            try:
                st = P.newton_solve(U, allow_unconverged=True)
                ok = st["fnorm"][-1] <= 1e-10 * st["fnorm"][0]
            except binding.StwrError:
                ok = False
            torch.cuda.synchronize()
            if ok:
                lat.append(time.perf_counter() - t0)
                sols[j] = U.cpu().numpy()
            else:
                fail += 1
            P.close()
            if (j + 1) % 16 == 0:
                log(f"[bench] uneven batch: {j + 1} solves done ({time.perf_counter() - t0:.1f}s)")
        return summary(lat, time.perf_counter() - t0, fail), sols

    log(f"[bench] uneven batch: {n_problems} problems, plain FP64 one at a time")
    plain, s64 = one_at_a_time(binding.FP64)
    log(f"[bench] uneven batch: plain {plain}; FP32 one at a time")
    solo32, s32 = one_at_a_time(binding.FP32)
    log(f"[bench] uneven batch: FP32 solo {solo32}; FP32 batch")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = binding.Batch(ctx, use_graph=True)
    t_create = time.perf_counter() - t0   # the batch's clock starts here
    ids = {B.add(p, opts(binding.FP32, 1)): j for j, p in enumerate(probs)}
    t_add = time.perf_counter() - t0
    res = B.run()
    span = time.perf_counter() - t0
    info = B.info()
    B.close()
    lat, sb, fail = [], {}, 0
    for r in res:
        if r["status"] == 0:
            lat.append(r["end_time"] + t_create)
            sb[ids[r["id"]]] = r["solution"]
        else:
            fail += 1
    batched = summary(sorted(lat), span, fail)
    batched.update({"add_s": t_add, "info": info})

    def worst(sols):
        e = [float(np.linalg.norm(sols[j] - s64[j]) / np.linalg.norm(s64[j])) for j in sols if j in s64]
        return max(e) if e else None

    ctx.close()
    return {"problems": n_problems,
            "workload": "uneven batch: meshes {8,16,32,64}^2, N in [8,128], q in {0,1}, Re 10^U[0,3], seeds 2000+j",
            "caps": {"newton_maxit": newton_maxit, "gmres_maxit": gmres_maxit, "newton_ew": 1},
            "plain_fp64_one_at_a_time": plain, "fp32_one_at_a_time": solo32, "fp32_batched": batched,
            "speedup_solves_per_s_vs_plain": batched["solves_per_s"] / plain["solves_per_s"],
            "speedup_solves_per_s_vs_fp32_solo": batched["solves_per_s"] / solo32["solves_per_s"],
            "max_rel_diff_fp32_solo_vs_plain": worst(s32), "max_rel_diff_batched_vs_plain": worst(sb),
            "converged_sets_equal": sorted(s64) == sorted(sb)}


def fifo_latencies(arrivals, service):
    """Completion latencies of one server taking requests in arrival order:
    start_j = max(a_j, finish_{j-1}), finish_j = start_j + s_j."""
    out, finish = [], 0.0
    for a, s in zip(arrivals, service):
        finish = max(a, finish) + s
        out.append(finish - a)
    return out


def serving_sweep(rates=(1.0, 2.0, 5.0, 200.0), n_req: int = 100, budget_gb: float = 200.0,
                  newton_maxit: int = 8, gmres_maxit: int = 30) -> dict:
    """Serving with kernel-level continuous batching: a seeded Poisson stream
    of n_req solves drawn from the uneven-batch distribution (seeds 3000+j) at
    each rate, admitted into one stwr_batch as they arrive while their device
    bytes fit the budget (else they wait, first in first out), so the sweeps
    and factorizations of every live solve share launches.  Beside it, the
    plain FP64-smoother path and the FP32 path serving one solve at a time in
    arrival order: their per-request service times are measured once and the
    single-server queue replayed for each rate's arrivals.  Same caps and
    Eisenstat-Walker tolerances as the uneven batch; latency = completion -
    arrival over the converged requests."""
    import numpy as np
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    probs = w.batch_problems(n_req, seed0=3000)

    def opts(prec, chunks):
        o = binding.default_opts()
        o.smoother_prec = prec
        o.newton_ew = 1
        o.newton_maxit = newton_maxit
        o.gmres_maxit = gmres_maxit
        o.time_chunks = chunks
        return o

    ctx = binding.Context(0)
    service, ok_solo, sols = {}, {}, {}
    for name, prec in (("fp64", binding.FP64), ("fp32", binding.FP32)):
        s, okl = [], []
        for j, p in enumerate(probs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = binding.Problem(ctx, p, opts(prec, 0))
            U = P.vec()
            try:
                st = P.newton_solve(U, allow_unconverged=True)
                ok = st["fnorm"][-1] <= 1e-10 * st["fnorm"][0]
            except binding.StwrError:
                ok = False
            torch.cuda.synchronize()
            s.append(time.perf_counter() - t0)
            okl.append(ok)
            if ok and name == "fp64":
                sols[j] = U.cpu().numpy()
            P.close()
            if (j + 1) % 20 == 0:
                log(f"[bench] serving sweep: {name} service times {j + 1}/{n_req} ({sum(s):.1f}s)")
        service[name], ok_solo[name] = s, okl
    ctx.close()

    rows = []
    for rate in rates:
        arr = w.arrival_times(rate, n_req, seed=3000)
        rec = {"rate_per_s": rate}
        for name in ("fp64", "fp32"):
            lat = fifo_latencies(arr, service[name])
            okl = [l for l, ok in zip(lat, ok_solo[name]) if ok]
            span = max(a + l for a, l in zip(arr, lat))
            rec[f"{name}_one_at_a_time"] = {"solves": len(okl), "makespan_s": span, "solves_per_s": len(okl) / span,
                                            "p50_latency_s": float(np.percentile(okl, 50)),
                                            "p99_latency_s": float(np.percentile(okl, 99))}
        bctx = binding.Context(0, hbm_budget=int(budget_gb * 1e9))
        B = binding.Batch(bctx, use_graph=True)
        t0 = time.perf_counter()
        nxt, waiting, ids, done, lat, errs = 0, [], {}, 0, [], []
        max_live, n_fail = 0, 0
        while done < n_req:
            now = time.perf_counter() - t0
            while nxt < n_req and arr[nxt] <= now:
                waiting.append(nxt)
                nxt += 1
            while waiting:
                j = waiting[0]
                try:
                    ids[B.add(probs[j], opts(binding.FP32, 1))] = j
                    waiting.pop(0)
                except binding.StwrError as e:
                    if e.code != -3:
                        raise
                    if B.info()["live"] == 0:   # larger than the whole budget: rejected
                        waiting.pop(0)
                        done += 1
                        n_fail += 1
                        continue
                    break
            live = B.info()["live"]
            max_live = max(max_live, live)
            if live:
                B.step()
            elif nxt < n_req:
                time.sleep(max(0.0, min(0.05, arr[nxt] - (time.perf_counter() - t0))))
            for r in B.poll():
                done += 1
                j = ids[r["id"]]
                if r["status"] == 0:
                    lat.append(time.perf_counter() - t0 - arr[j])
                    if j in sols:
                        errs.append(float(np.linalg.norm(r["solution"] - sols[j]) / np.linalg.norm(sols[j])))
                else:
                    n_fail += 1
        span = time.perf_counter() - t0
        info = B.info()
        B.close()
        bctx.close()
        rec["fp32_batched"] = {"solves": len(lat), "failed": n_fail, "makespan_s": span,
                               "solves_per_s": len(lat) / span,
                               "p50_latency_s": float(np.percentile(lat, 50)) if lat else None,
                               "p99_latency_s": float(np.percentile(lat, 99)) if lat else None,
                               "max_live": max_live, "steps": info["steps"], "graph_captures": info["graph_captures"],
                               "max_rel_diff_vs_plain": max(errs) if errs else None}
        log(f"[bench] serving sweep rate {rate}: {rec}")
        rows.append(rec)
    return {"requests_per_rate": n_req, "budget_gb": budget_gb,
            "workload": "Poisson arrivals (seed 3000) of uneven solves: meshes {8,16,32,64}^2, N in [8,128], "
                        "q in {0,1}, Re 10^U[0,3], seeds 3000+j",
            "caps": {"newton_maxit": newton_maxit, "gmres_maxit": gmres_maxit, "newton_ew": 1},
            "one_at_a_time_converged": {k: int(sum(v)) for k, v in ok_solo.items()}, "rates": rows}


def time_chunk_context(steps: int = 10) -> list:
    """Cyclic reduction in time on small meshes with long time axes (the
    uneven-batch distribution's small end: P2-P1 x DG(1), 128 slabs, Re 10):
    finest-level sweep time of the plain sweep and of the autotuned chunking,
    FP64 and FP32 factors."""
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    ctx = binding.Context(0)
    rows = []
    for M in (4, 8, 16):
        prob = w.small_problem(M, 2, 1, 128, 10.0, 103)
        for prec in (binding.FP64, binding.FP32):
            t = {}
            for chunks in (1, 0):
                o = binding.default_opts()
                o.smoother_prec = prec
                o.time_chunks = chunks
                P = binding.Problem(ctx, prob, o)
                U = P.vec()
                P.assemble(U)
                P.setup_smoothers()
                lam = P.eig_estimate(0)
                g = torch.Generator(device="cpu").manual_seed(4200)
                b = torch.randn(P.sizes(0)[0], generator=g, dtype=torch.float64).to("cuda")
                x = P.vec()
                P.relax(0, b, x, 2, 0.25 * lam, 1.05 * lam)
                ctx.set_timing(True)
                ctx.kernel_times()
                for _ in range(steps):
                    P.relax(0, b, x, 1, 0.25 * lam, 1.05 * lam)
                kt = ctx.kernel_times()
                ctx.set_timing(False)
                t[chunks] = (kt["sweep"][0] / steps, P.time_chunks(0))
                P.close()
            rows.append({"mesh": M, "slabs": 128, "patches": (M + 1) ** 2,
                         "smoother_prec": "fp32" if prec == binding.FP32 else "fp64",
                         "plain_sweep_ms": t[1][0], "tuned_sweep_ms": t[0][0], "tuned_chunks": t[0][1],
                         "speedup": t[1][0] / t[0][0]})
    ctx.close()
    return rows


def serving_benchmark(n_req: int = 16, slots: int = 4) -> dict:
    """Solves/s and latency of independent Newton solves, plain (FP64 smoother,
    one at a time) vs served (FP32 smoother, continuous batching over `slots`
    streams), on requests drawn from the uneven-batch distribution restricted
    to meshes {8, 16, 32}, N in [8, 64], Re in [1, 100] so the run stays short."""
    import numpy as np
    import stwr_workloads as w
    from paper_2407_13997_amd import binding

    probs = w.batch_problems(n_req, seed0=2000, meshes=(8, 16, 32), slab_range=(8, 64),
                             log10_re=(0.0, 2.0))

    def opts(prec):
        o = binding.default_opts()
        o.smoother_prec = prec
        o.newton_maxit = 12
        return o

    def closed_batch(prec, n_slots):
        srv = binding.Server(0, n_slots=n_slots)
        t0 = srv.now()
        ids = [srv.submit(p, opts(prec)) for p in probs]
        srv.wait(1200.0)
        res = {r["id"]: r for r in srv.poll()}
        srv.close()
        span = max(r["end_time"] for r in res.values()) - t0
        ok = [res[i] for i in ids if res[i]["status"] == 0]
        lat = [r["end_time"] - r["submit_time"] for r in res.values()]
        return {"solves": len(ok), "makespan_s": span, "solves_per_s": len(ok) / span,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99))}, [res[i] for i in ids]

    log(f"[bench] serving: {n_req} requests, plain FP64 x1 slot")
    plain, rp = closed_batch(0, 1)
    log(f"[bench] serving: FP32 x{slots} slots")
    served, rs = closed_batch(1, slots)
    errs = [float(np.linalg.norm(a["solution"] - b["solution"]) / max(np.linalg.norm(a["solution"]), 1e-300))
            for a, b in zip(rp, rs) if a["status"] == 0 and b["status"] == 0]
    # open loop: Poisson arrivals at 70% of the served closed-batch rate
    rate = 0.7 * served["solves_per_s"]
    arr = w.arrival_times(rate, n_req, seed=3000)
    srv = binding.Server(0, n_slots=slots)
    t0 = srv.now()
    for a, p in zip(arr, probs):
        while srv.now() - t0 < a:
            time.sleep(min(0.002, max(0.0, a - (srv.now() - t0))))
        srv.submit(p, opts(1), want_solution=False)
    srv.wait(1200.0)
    res = srv.poll()
    srv.close()
    lat = [r["end_time"] - r["submit_time"] for r in res if r["status"] == 0]
    return {
        "requests": n_req,
        "workload": "uneven batch: meshes {8,16,32}, N in [8,64], q in {0,1}, Re in [1,100], seeds 2000+",
        "plain_fp64_serial": plain,
        "served_fp32": dict(served, slots=slots),
        "speedup_solves_per_s": served["solves_per_s"] / plain["solves_per_s"],
        "max_rel_diff_served_vs_plain": max(errs) if errs else None,
        "poisson": {"rate_per_s": rate, "completed": len(lat),
                    "p50_latency_s": float(np.percentile(lat, 50)) if lat else None,
                    "p99_latency_s": float(np.percentile(lat, 99)) if lat else None},
    }


def p3p2_sweep(steps: int = 10) -> dict:
    """The Taylor-Hood P3-P2 x DG(1) relaxation sweep on the paper's largest
    P3-P2 run (Sec. 4.2: Chorin problem on 80 x 80, 10 slabs; five levels),
    FP32 factors of the 81-DoF Vanka+star patches (slab blocks of order 162),
    timed as the main workload: operator, large-block sweep and gather.  Its
    roofline counts every (patch, slab) inverse block once (m^2 4 bytes) and
    the FP64 residual and correction (24 n_st)."""
    import numpy as np
    import torch
    import stwr_workloads as w
    from paper_2407_13997_amd import binding
    prob = w.chorin_problem(80, 5, 1, 10, nodes=1, degree=2)
    ctx = binding.Context(0)
    o = binding.default_opts()
    o.smoother_prec = binding.FP32
    P = binding.Problem(ctx, prob, o)
    n_st, nf, n_patch = P.sizes(0)
    U = P.vec()
    P.assemble(U)
    t = time.perf_counter()
    P.patch_factor(0, binding.FP32)
    torch.cuda.synchronize()
    t_fac = time.perf_counter() - t
    lam = P.eig_estimate(0)
    a, bnd = o.cheb_lo * lam, o.cheb_hi * lam
    g = torch.Generator(device="cpu").manual_seed(4001)
    b = torch.randn(n_st, generator=g, dtype=torch.float64).to("cuda")
    x = torch.zeros(n_st, dtype=torch.float64, device="cuda")
    P.relax(0, b, x, 2, a, bnd)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.kernel_times()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        P.relax(0, b, x, 1, a, bnd)
    e1.record()
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    P.close()
    ctx.close()
    ms = e0.elapsed_time(e1) / steps
    sw = kt["sweep"][0] / max(kt["sweep"][1], 1)
    _, ptr, _ = binding.level_patches(prob.mesh_n, 2)
    m = np.diff(ptr).astype(np.int64) * (prob.q + 1)
    algo = int((m * m).sum()) * prob.n_slabs * 4 + 24 * int(n_st)
    return {"workload": "chorin_p3p2_dg1_m80_n10 finest-level WR sweep", "st_dofs": int(n_st),
            "patches": int(n_patch), "steps": steps, "ms_per_step": ms, "value": n_st / (ms * 1e-3),
            "unit": "st-DoF/s", "factor_finest_s": t_fac,
            "kernels_ms_per_sweep": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
            "roofline": {"bound": "hbm", "kernel": "k_patch_sweep_big (FP32 blocks)", "avg_ms": sw,
                         "algorithmic_bytes": algo, "achieved": algo / (sw * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": algo / (sw * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def patch_sweep_bytes_algorithmic(prob, s_f: int, n_st: int, s_r: int) -> int:
    """Algorithmic bytes of one WR sweep's patch kernel: every (patch, slab)
    inverse block once, m^2 s_f bytes (m = (q+1) nb), plus the residual read
    once (s_r n_st: 4 for the FP32 sweep, which reads it rounded to FP32, 8
    otherwise) and the FP64 correction read and written once (16 n_st)."""
    from paper_2407_13997_amd import binding
    hist = binding.mesh_info(prob.mesh_n)[12:52]
    nq = prob.q + 1
    blocks = sum(int(cnt) * prob.n_slabs * (nb * nq) ** 2 * s_f for nb, cnt in enumerate(hist))
    return blocks + (s_r + 16) * int(n_st)


def patch_sweep_bytes(prob, s_f: int, s_r: int) -> int:
    """Algorithmic bytes of one patch-sweep launch on the finest level:
    sum over patches of N (m^2 s_f + s_r m + s_f m), m = (q+1) nb the slab
    block size: the inverse block, the residual gather (s_r bytes a value)
    and the patch output (in the smoother's precision) per slab."""
    from paper_2407_13997_amd import binding
    info = binding.mesh_info(prob.mesh_n)
    hist = info[12:52]
    nq = prob.q + 1
    tot = 0
    for nb, cnt in enumerate(hist):
        m = nb * nq
        tot += int(cnt) * prob.n_slabs * (m * m * s_f + s_r * m + s_f * m)
    return tot


if __name__ == "__main__":
    main()
