"""Write sampled values of the exact discrete solution on slabs 0 and 1 of the
128x128, P2-P1 x DG(1), 64-slab, Re 1000 workload (seed 4000, 16
stream-function modes) to ns_p2p1_dg1_m128_n64_re1000_newton_reference.json.

The space-time residual of slab n depends only on the values of slabs n and
n-1 (eq. nsfem: the upwind jump couples a slab to its predecessor alone), so
the solution on slabs 0 and 1 of the 64-slab problem is the solution of the
same problem truncated to its first two slabs (t_final = 2/64).  The oracle
computes that by its slab-by-slab route: Newton on each slab with a sparse
direct solve of the bordered slab Jacobian, to its rounding floor.  Calls only
the oracle and the seeded generators.
Run: python tests/golden/make_m128_newton_reference.py   (tens of minutes)
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
from oracle.direct import solve_slab_by_slab  # noqa: E402
from oracle.mms import MMS  # noqa: E402

S = 2                 # slabs of the truncated problem
N_SAMPLES = 800


def main():
    p = w.named_problem(w.LARGE)
    t = time.time()
    nq = p.q + 1
    lev = Level(p.mesh_n, p.q, S, S / p.n_slabs * p.t_final,
                MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds))
    info = []
    x = solve_slab_by_slab(lev, info=info)            # [free DoF][slab][node]
    nf = lev.n_free
    rng = np.random.default_rng(4201)
    dofs = np.sort(rng.choice(nf, N_SAMPLES // (S * nq), replace=False))
    samples = [(int(d), n, a) for d in dofs for n in range(S) for a in range(nq)]
    idx = [(d * p.n_slabs + n) * nq + a for d, n, a in samples]
    val = [float(x[d, n, a]) for d, n, a in samples]
    norms = [float(np.linalg.norm(x[:, n, :])) for n in range(S)]
    maxabs = [float(np.max(np.abs(x[:, n, :]))) for n in range(S)]
    out = {"workload": "128x128, P2-P1 x DG(1), 64 slabs, Re 1000, seed 4000, 16 modes",
           "solution": "exact discrete solution (slab-by-slab Newton with sparse direct solves) "
                       "of the problem truncated to its first 2 slabs",
           "n_st": int(nf * p.n_slabs * nq), "slabs": S, "slab_fnorm_final": info,
           "slab_norm": norms, "slab_maxabs": maxabs,
           "index": idx, "value": val, "seconds": time.time() - t}
    with open(os.path.join(HERE, "ns_p2p1_dg1_m128_n64_re1000_newton_reference.json"), "w") as f:
        json.dump(out, f)
    print(len(idx), info, norms, out["seconds"])


if __name__ == "__main__":
    main()
