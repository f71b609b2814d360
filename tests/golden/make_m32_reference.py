"""Write the sampled exact discrete solution of the 32x32, DG(1), 32-slab,
Re = 100 workload (seed 1000) to ns_p2p1_dg1_m32_n32_re100_reference.json.

The discrete solution does not depend on the multigrid hierarchy, so the same
reference serves every level count.

Calls only the oracle: the slab-by-slab direct route (Newton per slab with a
sparse direct solve), whose result is the exact discrete space-time solution
(pressure normalised to zero mean per temporal node).  Stored: the 2-norm and
max-norm of the solution and 400 seeded sample entries.
Run: python tests/golden/make_m32_reference.py   (about 10 minutes on one core)
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


def main():
    p = w.named_problem(w.MEDIUM)
    lev = Level(p.mesh_n, p.q, p.n_slabs, p.t_final,
                MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds))
    t = time.time()
    info = []
    x = solve_slab_by_slab(lev, info=info).ravel()
    idx = np.sort(np.random.default_rng(1001).choice(x.size, 400, replace=False))
    out = {"workload": "32x32, P2-P1 x DG(1), 32 slabs, Re 100, seed 1000",
           "route": "oracle slab-by-slab Newton with sparse direct solves",
           "n_st": int(x.size), "norm2": float(np.linalg.norm(x)),
           "norminf": float(np.abs(x).max()),
           "velocity_l2_error": float(lev.velocity_l2_error(x.reshape(lev.n_free, lev.N, lev.nq))),
           "slab_residuals_max": max(info),
           "index": idx.tolist(), "value": [float(v) for v in x[idx]],
           "seconds": time.time() - t}
    with open(os.path.join(HERE, "ns_p2p1_dg1_m32_n32_re100_reference.json"), "w") as f:
        json.dump(out, f)
    print(out["norm2"], out["seconds"])


if __name__ == "__main__":
    main()
