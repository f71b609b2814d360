"""Plain FP64 CPU oracle of the space-time waveform-relaxation multigrid method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the two meet
only through the seeded input arrays of ``stwr_workloads``.

Everything here is slow on purpose: NumPy/SciPy, float64, literal quadrature
of the weak form (eq. nsfem, Sec. 2), algebraic extraction of patch blocks from
the assembled space-time Jacobian (Sec. 3), and the solver steps in the
paper's order (Alg. 1 V-cycle, Chebyshev-accelerated relaxation, FGMRES,
Newton).  Each module names the passage it follows.

Parity pins: every function is pinned by tests under tests/ against closed
forms, the paper's printed counts, invariants or independent routes; no
function here is "parity unpinned" except where a module header says so.
"""
