"""Write sampled outputs of one additive WR patch application (Sec. 3,
eq. waveform_patch_solve) on the 128x128, P2-P1 x DG(1), 64-slab, Re 1000
workload (seed 4000) at the Newton start U = 0, to
ns_p2p1_dg1_m128_n64_re1000_sweep_reference.json.

The patch solves are forward substitutions in time, so the outputs of slabs
0 .. S-1 depend only on the residual of those slabs and on the Jacobian
blocks of those slabs; at U = 0 those blocks are the ones of the same problem
truncated to S slabs of the same length (t_final = S / 64).  The oracle
assembles that truncated space-time Jacobian and applies its patch smoother
on every vertex patch that contains a sampled DoF, so each sampled output is
the complete additive sum.  Samples are taken on slabs 0-2 and 8-9, so the
check crosses the FP32 sweep's first 8-slab residual line.  Calls only the
oracle and the seeded generators.
Run: python tests/golden/make_m128_sweep_reference.py   (a few minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import stwr_workloads as w  # noqa: E402
from oracle.assembly import Level  # noqa: E402
from oracle.mms import MMS  # noqa: E402
from oracle.smoother import PatchSmoother  # noqa: E402

S = 10                # slabs of the truncated problem
CHECKED = (0, 1, 2, 8, 9)   # slabs sampled: the first ones and two past the
                            # first 8-slab residual line of the FP32 sweep
R_SEED = 4100         # residual of the full problem: seeded_vector(n_st, R_SEED)
N_SAMPLES = 400


def main():
    p = w.named_problem(w.LARGE)
    t = time.time()
    nq = p.q + 1
    lev = Level(p.mesh_n, p.q, S, S / p.n_slabs * p.t_final,
                MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds))
    nf = lev.n_free
    n_st_full = nf * p.n_slabs * nq
    r_full = w.seeded_vector(n_st_full, R_SEED).reshape(nf, p.n_slabs, nq)
    r = np.ascontiguousarray(r_full[:, :S, :]).ravel()
    A = lev.jacobian(lev.initial_guess())
    rng = np.random.default_rng(4101)
    # sampled (DoF, slab, node): DoFs spread over velocity and pressure
    dofs = np.sort(rng.choice(nf, N_SAMPLES // len(CHECKED), replace=False))
    samples = [(int(d), n, int(rng.integers(nq))) for d in dofs for n in CHECKED]
    patches = [P for P in lev.mesh.patches() if np.isin(P, dofs).any()]
    z = PatchSmoother(lev, A, patches=patches).apply(r).reshape(nf, S, nq)
    idx = [(d * p.n_slabs + n) * nq + a for d, n, a in samples]
    val = [float(z[d, n, a]) for d, n, a in samples]
    out = {"workload": "128x128, P2-P1 x DG(1), 64 slabs, Re 1000, seed 4000, U = 0",
           "operation": "one additive WR Vanka+star patch application z = M^{-1} r",
           "residual": f"seeded_vector(n_st, {R_SEED}) of the full problem",
           "slabs_checked": list(CHECKED), "n_st": int(n_st_full), "patches_used": len(patches),
           "index": idx, "value": val, "seconds": time.time() - t}
    with open(os.path.join(HERE, "ns_p2p1_dg1_m128_n64_re1000_sweep_reference.json"), "w") as f:
        json.dump(out, f)
    print(len(idx), len(patches), out["seconds"])


if __name__ == "__main__":
    main()
