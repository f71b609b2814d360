"""Oracle mesh, DoF and patch structure against the paper's closed-form
counts (Sec. 3.1, App. A.1) and printed DoF tables (Secs. 4.1, 4.2)."""
import collections
import os

import numpy as np
import pytest

from oracle.mesh import Mesh

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def entity_counts(M):
    m = Mesh(M)
    nv = m.nv
    ne = len({tuple(sorted(e)) for c in m.cells for e in ((c[0], c[1]), (c[1], c[2]), (c[0], c[2]))})
    return nv, ne, m.nc


def ns_dofs_formula(Mx, k):
    # Sec. 3.1: NS spatial DoFs with Mx vertices per side, pressure degree k
    return 3 * (Mx - 1) ** 2 * k ** 2 + (4 * (Mx - 1) ** 2 + 6 * (Mx - 1)) * k \
        + 2 * (Mx - 1) ** 2 + 4 * (Mx - 1) + 3


def heat_dofs_formula(Mx, k):
    # Sec. 3.1, eq. PkDoFcount
    return Mx ** 2 + (3 * (Mx - 1) ** 2 + 2 * (Mx - 1)) * (k - 1) \
        + 2 * (Mx - 1) ** 2 * (k - 1) * (k - 2) // 2


@pytest.mark.parametrize("M", [2, 4, 5, 8, 16])
def test_ns_global_dofs_match_paper_formula(M):
    m = Mesh(M)
    total = 2 * m.nn + m.nv            # P2 velocity (2 comps) + P1 pressure, Dirichlet included
    assert total == ns_dofs_formula(M + 1, 1)
    nv, ne, nc = entity_counts(M)
    # P3-P2 from entity counts: P3 = v + 2e + c, P2 = v + e
    assert 2 * (nv + 2 * ne + nc) + (nv + ne) == ns_dofs_formula(M + 1, 2)
    assert m.n_free == 2 * (2 * M - 1) ** 2 + (M + 1) ** 2


@pytest.mark.parametrize("M", [3, 6])
def test_heat_dofs_formula_matches_entities(M):
    nv, ne, nc = entity_counts(M)
    for k in (1, 2, 3):
        assert nv + (k - 1) * ne + (k - 1) * (k - 2) // 2 * nc == heat_dofs_formula(M + 1, k)


def _sig2(x):
    return float(f"{x:.1e}")


def test_chorin_dof_table():
    nv, ne, nc = 81 * 81, 3 * 80 * 80 + 2 * 80, 2 * 80 * 80
    for line in open(os.path.join(GOLD, "chorin_dofs.txt")):
        if line.startswith("#") or not line.strip():
            continue
        q, k, N, val = line.split()
        q, k, N, val = int(q), int(k), int(N), float(val)
        assert ns_dofs_formula(81, k) * N * (q + 1) == pytest.approx(val, rel=0.05)
        assert _sig2(ns_dofs_formula(81, k) * N * (q + 1)) == val


def test_heat_dof_table():
    for line in open(os.path.join(GOLD, "heat_dofs.txt")):
        if line.startswith("#") or not line.strip():
            continue
        q, k, val = line.split()
        q, k, val = int(q), int(k), float(val)
        assert _sig2(heat_dofs_formula(81, k) * 20 * (q + 1)) == val


def test_mesh_geometry():
    m = Mesh(4)
    assert m.nc == 32
    # every square's diagonal runs from bottom-right to top-left (x + y const)
    for c in m.cells:
        xy = m.vxy[c]
        e1, e2 = xy[1] - xy[0], xy[2] - xy[0]
        area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
        assert area == pytest.approx(0.5 / 16)
    # vertex stars: 6 cells at interior vertices (Sec. 3.1)
    inc = collections.Counter(m.cells.ravel())
    assert inc[1 + 5 * 1] == 6


def test_patch_dofs_interior_is_39():
    # Sec. 3.1: 9k^2 + 15k + 15 DoFs per Vanka+star patch (k = 1)
    m = Mesh(8)
    P = m.patches()
    v = 4 + 9 * 4
    assert len(P[v]) == 9 + 15 + 15
    sizes = collections.Counter(len(p) for p in P)
    assert sizes[39] == 7 * 7 - 0 - 24  # interior vertices not adjacent to the boundary: 5x5
    assert set(sizes) == {3, 9, 11, 15, 27, 29, 33, 39}


def test_patch_nonzeros_is_728():
    """App. A.1: 12k^4 + 96k^3 + 240k^2 + 252k + 128 = 728 nonzeros in an interior
    patch matrix at k=1: 652 velocity-velocity, 38 in each velocity-pressure block."""
    from oracle.assembly import Level
    from oracle.mms import MMS
    import stwr_workloads as w
    p = w.small_problem(6, 1, 0, 1, 10.0, seed=7)
    mms = MMS(p.psi_ab, p.psi_coef, p.p_ab, p.p_coef, p.reynolds)
    L = Level(6, 0, 1, 1.0, mms)
    x = np.random.default_rng(3).standard_normal((L.n_free, 1, 1))
    J = L.jacobian(x).toarray()
    v = 3 + 7 * 3
    S = L.mesh.patches()[v]
    A = J[np.ix_(S, S)]
    po = L.mesh.p_offset
    isv = S < po
    assert np.count_nonzero(A) == 12 + 96 + 240 + 252 + 128
    assert np.count_nonzero(A[np.ix_(isv, isv)]) == 652
    assert np.count_nonzero(A[np.ix_(isv, ~isv)]) == 38
    assert np.count_nonzero(A[np.ix_(~isv, isv)]) == 38
    assert np.count_nonzero(A[np.ix_(~isv, ~isv)]) == 0


def test_vcycle_patch_count_model():
    # Sec. 3.1: 4 (Mx^2 + (Mx/2)^2 + ...) ~ 16/3 Mx^2 patches per V(2,2) cycle
    tot = sum(4 * (Mesh(128 >> l).nv) for l in range(6))
    assert tot / (16.0 / 3.0 * 129 ** 2) == pytest.approx(1.0, rel=0.02)
